"""Seeded synthetic inputs: voxel chunks and camera poses.

This module holds no part of the SVDAG method.  It only produces inputs that
both the CPU oracle and the GPU library consume:

* dense uint8 chunks (0 = empty, 1..255 = material ID; index
  ``x + S*(y + S*z)``), from the C generator ``libscenegen.so``, or for the
  terrain kinds from its GPU copy ``libscenegen_gpu.so`` straight into device
  memory (the same bytes, used where a map is too large to generate on the
  host in a reasonable time);
* camera poses (position, target, up, vertical FOV, resolution) in float32;
* tiny random worlds for exhaustive tests (numpy, seeded).

The paper's scenes (voxelised San Miguel, Sponza and the Greenfield Minecraft
city, Section 4) are not available; the procedural scenes below stand in for
them.  The workloads are:

``noise64``      one 64^3 chunk of 3D value noise (~30% fill), 256x256 rays.
``terrain1024``  one 1024^3 terrain chunk with caves, 1920x1080 rays.
``map512``       16x16 chunks of 512^3 terrain + box buildings, 4 LODs,
                 2560x1440 rays (the 1440p throughput workload).
``map1024``      32x32 chunks of 1024^3, 4 LODs.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

KINDS = {"noise64": 0, "terrain1024": 1, "map512": 2, "map1024": 3, "custom": 4}


def lib_path() -> str:
    return os.path.join(_HERE, "libscenegen.so")


def build(verbose: bool = False) -> str:
    """Compile the generator with gcc (host code only)."""
    import subprocess

    src = os.path.join(_HERE, "scenegen.c")
    out = lib_path()
    cmd = ["gcc", "-O2", "-Wall", "-fPIC", "-shared", "-fvisibility=hidden",
           "-o", out + ".tmp", src, "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


def gpu_lib_path() -> str:
    return os.path.join(_HERE, "libscenegen_gpu.so")


def build_gpu(verbose: bool = False) -> str:
    """Compile the GPU copy of the terrain generator (hipcc, gfx950)."""
    import subprocess

    src = os.path.join(_HERE, "scenegen_gpu.hip")
    out = gpu_lib_path()
    cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-O3", "-fPIC", "-std=c++17",
           "-ffp-contract=off", "-Wall", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-shared", "-fvisibility=hidden", "-o", out + ".tmp", src]
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"build failed: {' '.join(cmd)}\n{r.stdout}{r.stderr}")
    os.replace(out + ".tmp", out)
    return out


_GPU_LIB = None


def _gpu_lib():
    global _GPU_LIB
    if _GPU_LIB is None:
        import torch  # noqa: F401  (load torch's HIP runtime first: one runtime per process)
        p = gpu_lib_path()
        if not os.path.exists(p):
            raise RuntimeError(f"{p} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(p)
        i64p, f64p = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)
        L.sgg_work_bytes.restype = ctypes.c_size_t
        L.sgg_work_bytes.argtypes = [i64p, f64p, ctypes.c_uint32]
        L.sgg_gen_chunk.restype = ctypes.c_int
        L.sgg_gen_chunk.argtypes = [i64p, f64p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                    ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_uint32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        _GPU_LIB = L
    return _GPU_LIB


def _lib():
    global _LIB
    if _LIB is None:
        p = lib_path()
        if not os.path.exists(p):
            raise RuntimeError(f"{p} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(p)
        L.sg_world_new.restype = ctypes.c_void_p
        L.sg_world_new.argtypes = [ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32,
                                   ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32]
        L.sg_world_free.argtypes = [ctypes.c_void_p]
        L.sg_world_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                    ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_int)]
        L.sg_height.restype = ctypes.c_int64
        L.sg_height.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]
        L.sg_gen_chunk.restype = ctypes.c_int
        L.sg_gen_chunk.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                   ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int]
        L.sg_world_params.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_void_p)]
        L.sg_splitmix64.restype = ctypes.c_uint64
        L.sg_splitmix64.argtypes = [ctypes.c_uint64]
        _LIB = L
    return _LIB


def splitmix64(x: int) -> int:
    return int(_lib().sg_splitmix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


@dataclass
class Camera:
    """Pinhole camera in voxel units; +z is up, vertical FOV in degrees."""
    pos: tuple
    target: tuple
    up: tuple
    vfov_deg: float
    width: int
    height: int

    def as_f32(self):
        f = lambda v: tuple(float(np.float32(x)) for x in v)
        return Camera(f(self.pos), f(self.target), f(self.up),
                      float(np.float32(self.vfov_deg)), int(self.width), int(self.height))


class SceneWorld:
    """A seeded procedural world, generated one chunk at a time."""

    def __init__(self, kind: str, seed: int, chunk_log2: int = 0, grid=(1, 1, 1)):
        L = _lib()
        self.kind = kind
        self.seed = int(seed)
        h = L.sg_world_new(KINDS[kind], ctypes.c_uint64(self.seed), chunk_log2, *grid)
        if not h:
            raise ValueError(f"bad scene kind {kind!r}")
        self._h = h
        self._free = _lib().sg_world_free  # held: module globals may be gone at exit
        cl = ctypes.c_uint32()
        g = (ctypes.c_uint32 * 3)()
        nb = ctypes.c_int()
        L.sg_world_info(h, ctypes.byref(cl), g, ctypes.byref(nb))
        self.chunk_log2 = cl.value
        self.grid = (g[0], g[1], g[2])
        self.nbox = nb.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._free(h)
            self._h = None

    @property
    def S(self) -> int:
        return 1 << self.chunk_log2

    @property
    def extent(self):
        return tuple(g * self.S for g in self.grid)

    def chunks(self):
        gx, gy, gz = self.grid
        for cz in range(gz):
            for cy in range(gy):
                for cx in range(gx):
                    yield (cx, cy, cz)

    def chunk(self, c, out: np.ndarray | None = None, threads: int = 1) -> np.ndarray:
        S = self.S
        if out is None:
            out = np.empty(S * S * S, dtype=np.uint8)
        assert out.dtype == np.uint8 and out.size == S ** 3 and out.flags.c_contiguous
        rc = _lib().sg_gen_chunk(self._h, c[0], c[1], c[2], out.ctypes.data, int(threads))
        if rc != 0:
            raise ValueError(f"chunk {c} out of range")
        return out

    def _terrain_params(self):
        """(ip, dp, boxes): the generator's parameters and its boxes as an
        int32 array of rows {x0, y0, z0, x1, y1, z1, material, 0} in paint
        order."""
        if getattr(self, "_tp", None) is None:
            ip = (ctypes.c_int64 * 6)()
            dp = (ctypes.c_double * 2)()
            bp = ctypes.c_void_p()
            _lib().sg_world_params(self._h, ip, dp, ctypes.byref(bp))
            nb = int(ip[5])
            rec = np.dtype({"names": ["b", "m"], "formats": [("<i4", 6), "u1"], "offsets": [0, 24],
                            "itemsize": 28})
            raw = np.frombuffer(ctypes.string_at(bp.value, 28 * nb), dtype=rec) if nb else np.zeros(0, rec)
            boxes = np.zeros((nb, 8), np.int32)
            boxes[:, :6] = raw["b"]
            boxes[:, 6] = raw["m"]
            self._tp = (ip, dp, boxes)
        return self._tp

    def chunk_boxes(self, c) -> np.ndarray:
        """The boxes that meet chunk c, in paint order, as int32 rows {x0, y0,
        z0, x1, y1, z1, material, 0}."""
        boxes = self._terrain_params()[2]
        S = self.S
        keep = np.ones(len(boxes), bool)
        for a in range(3):
            lo = int(c[a]) * S
            keep &= (boxes[:, a] < lo + S) & (boxes[:, a + 3] > lo)
        return np.ascontiguousarray(boxes[keep])

    def chunk_device(self, c, out, work=None, stream=None):
        """Generate chunk c on the GPU into `out`, a contiguous uint8 device
        tensor of S^3 bytes: the same bytes as chunk(c).  Terrain kinds only
        (not noise64).  `work` is an optional uint8 device tensor reused as
        workspace; the call enqueues on `stream` (torch's current stream if
        None) and returns the workspace."""
        import torch
        L = _gpu_lib()
        ip, dp, boxes = self._terrain_params()
        S, cl = self.S, self.chunk_log2
        if int(ip[0]) != 1:
            raise ValueError(f"{self.kind}: the GPU generator covers the terrain kinds only")
        if not all(0 <= int(c[a]) < self.grid[a] for a in range(3)):
            raise ValueError(f"chunk {c} out of range")
        if not (out.is_cuda and out.dtype == torch.uint8 and out.is_contiguous() and out.numel() == S ** 3):
            raise ValueError("out must be a contiguous uint8 device tensor of S^3 bytes")
        sel = self.chunk_boxes(c)
        s = stream if stream is not None else torch.cuda.current_stream(out.device)
        need = int(L.sgg_work_bytes(ip, dp, cl))
        if need == 0:
            raise ValueError("bad generator parameters")
        if work is None or work.numel() < need:
            work = torch.empty(need, dtype=torch.uint8, device=out.device)
        with torch.cuda.stream(s):  # the box list's copy is ordered before the kernels that read it
            bd = torch.from_numpy(sel if len(sel) else np.zeros((1, 8), np.int32)).to(out.device)
            rc = L.sgg_gen_chunk(ip, dp, ctypes.c_uint64(self.seed), cl, int(c[0]), int(c[1]), int(c[2]),
                                 bd.data_ptr(), len(sel), out.data_ptr(), work.data_ptr(), work.numel(),
                                 ctypes.c_void_p(s.cuda_stream))
        bd.record_stream(s)
        work.record_stream(s)  # held until the stream has run the generation, even if dropped
        if rc != 0:
            raise RuntimeError(f"sgg_gen_chunk failed ({rc})")
        return work

    def height(self, x: int, y: int) -> int:
        return int(_lib().sg_height(self._h, int(x), int(y)))

    # -- camera poses ------------------------------------------------------
    def views(self, n: int, seed: int, width: int | None = None, height: int | None = None):
        """Seeded camera poses for this workload (float32-representable)."""
        rng = np.random.default_rng([self.seed, seed, 0xC0FFEE])
        cams = []
        X, Y, Z = self.extent
        for _ in range(n):
            if self.kind == "noise64":
                u = rng.normal(size=3)
                u /= np.linalg.norm(u)
                c = np.array([X / 2, Y / 2, Z / 2])
                pos = c + 96.0 * u
                cam = Camera(tuple(pos), tuple(c), (0.0, 0.0, 1.0), 60.0,
                             width or 256, height or 256)
            else:
                if self.kind == "terrain1024":
                    margin, pitch_lo, pitch_hi, W, H = 64, -30.0, 0.0, 1920, 1080
                elif self.kind == "custom":
                    margin, pitch_lo, pitch_hi, W, H = 2, -30.0, 10.0, 64, 48
                else:
                    margin, pitch_lo, pitch_hi, W, H = 256, -20.0, 5.0, 2560, 1440
                x = rng.uniform(margin, X - margin)
                y = rng.uniform(margin, Y - margin)
                hz = self.height(int(x), int(y))
                z = min(hz + 50.0, Z - 0.5) if self.kind != "custom" else min(hz + 3.5, Z - 0.5)
                yaw = rng.uniform(0.0, 2.0 * math.pi)
                if self.kind == "custom":
                    # small test worlds: look roughly towards the middle
                    yaw = math.atan2(Y / 2 - y, X / 2 - x) + rng.uniform(-0.6, 0.6)
                    pitch_lo, pitch_hi = -35.0, -5.0
                pitch = math.radians(rng.uniform(pitch_lo, pitch_hi))
                d = np.array([math.cos(pitch) * math.cos(yaw),
                              math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
                pos = np.array([x, y, z])
                cam = Camera(tuple(pos), tuple(pos + 100.0 * d), (0.0, 0.0, 1.0), 60.0,
                             width or W, height or H)
            cams.append(cam.as_f32())
        return cams


    def walk_requests(self, walkers: int, rate: float, duration: float, seed: int,
                      sizes=((320, 180), (640, 360), (1280, 720), (1920, 1080)),
                      speed: float = 150.0, height_above: float = 50.0):
        """Seeded serving load: Poisson arrivals (mean gap 1/rate seconds) over
        `duration` seconds; each request is a view from one of `walkers`
        cameras that wander the map at `speed` voxels/s, `height_above`
        voxels over the terrain, heading changing every second, looking
        roughly ahead with pitch in [-20, 5] degrees; resolution uniform over
        `sizes`.  Returns [(arrival_s, Camera)]."""
        rng = np.random.default_rng([self.seed, seed, 0x5E12])
        X, Y, Z = self.extent
        margin = min(256.0, X / 8, Y / 8)
        dt = 0.05
        steps = int(math.ceil(duration / dt)) + 2
        pos = np.empty((walkers, steps, 2))
        head = np.empty((walkers, steps))
        for w in range(walkers):
            p = np.array([rng.uniform(margin, X - margin), rng.uniform(margin, Y - margin)])
            h = rng.uniform(0, 2 * math.pi)
            for i in range(steps):
                if i and i % int(round(1 / dt)) == 0:
                    h += rng.normal(0, 0.6)
                p = p + speed * dt * np.array([math.cos(h), math.sin(h)])
                for a, hi in ((0, X), (1, Y)):  # reflect at the map's margin
                    if p[a] < margin or p[a] > hi - margin:
                        p[a] = min(max(p[a], margin), hi - margin)
                        h = math.pi - h if a == 0 else -h
                pos[w, i], head[w, i] = p, h
        out, t = [], 0.0
        while True:
            t += rng.exponential(1.0 / rate)
            if t >= duration:
                break
            w = int(rng.integers(walkers))
            i = min(int(t / dt), steps - 1)
            x, y = pos[w, i]
            z = min(self.height(int(x), int(y)) + height_above, Z - 0.5)
            yaw = head[w, i] + rng.uniform(-0.3, 0.3)
            pitch = math.radians(rng.uniform(-20.0, 5.0))
            W, H = sizes[int(rng.integers(len(sizes)))]
            d = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
            cam = Camera((x, y, z), tuple(np.array([x, y, z]) + 100.0 * d), (0.0, 0.0, 1.0), 60.0, W, H)
            out.append((t, cam.as_f32()))
        return out


# -- tiny random worlds (tests) -------------------------------------------

def random_grid(rng: np.random.Generator, R: int, fill: float, nmat: int = 15,
                structured: bool = True) -> np.ndarray:
    """Random R^3 uint8 grid (index x + R*(y + R*z)).

    With ``structured`` the occupancy is drawn per 2^3 block first and then
    per voxel, so that empty and full sub-cubes of several sizes occur.
    """
    if structured and R >= 4:
        blk = rng.random((R // 2, R // 2, R // 2)) < min(1.0, 2.5 * fill)
        occ = np.repeat(np.repeat(np.repeat(blk, 2, 0), 2, 1), 2, 2)
        occ &= rng.random((R, R, R)) < min(1.0, fill / max(1e-9, min(1.0, 2.5 * fill)) * 1.0)
    else:
        occ = rng.random((R, R, R)) < fill
    mat = rng.integers(1, nmat + 1, size=(R, R, R), dtype=np.uint8)
    g = np.where(occ, mat, 0).astype(np.uint8)  # axes (z, y, x) after flatten order below
    return np.ascontiguousarray(g).reshape(-1)
