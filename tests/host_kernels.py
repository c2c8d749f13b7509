"""Test infrastructure: ctypes wrapper of host_kernels.cpp (the library's
kernel logic compiled for the host) and its build step."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhost_kernels.so")


def build(verbose: bool = False) -> str:
    """hipcc the host build of kernels.hip (links libsvdag for the builder)."""
    pkg = os.path.join(ROOT, "paper_2505_02017_amd")
    cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread",
           "-ffp-contract=off", "-x", "hip", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           f"-I{os.path.join(ROOT, 'include')}", f"-I{os.path.join(pkg, 'csrc')}",
           os.path.join(HERE, "host_kernels.cpp"), "-o", LIB + ".tmp",
           f"-L{pkg}", "-lsvdag", f"-Wl,-rpath,{pkg}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("host kernel build failed:\n" + r.stdout + r.stderr)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise ImportError(f"{LIB} is missing: build it with __graft_entry__.build()")
        import torch  # noqa: F401  (its HIP runtime first: one runtime per process)
        L = ctypes.CDLL(LIB)
        vp, u32 = ctypes.c_void_p, ctypes.c_uint32
        L.hk_world_new.restype = vp
        L.hk_world_new.argtypes = [vp]
        L.hk_world_free.argtypes = [vp]
        L.hk_world_free.restype = None
        L.hk_upload.argtypes = [vp, u32, vp, ctypes.c_int]
        L.hk_trace.argtypes = [vp, vp, u32, vp, vp, u32]
        L.hk_trace_counts.argtypes = [vp, vp, u32, vp, u32, vp]
        L.hk_row_queue_tiles.argtypes = [u32, u32, vp]
        L.hk_row_queue_tiles.restype = u32
        L.hk_beam_cube.argtypes = [vp, vp, vp, vp, u32, u32, u32, u32, vp, ctypes.c_int32, vp]
        L.hk_beam_cube.restype = ctypes.c_int
        L.hk_scene_chunk.argtypes = [ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                     ctypes.c_uint64, u32, u32, u32, u32, vp, u32, vp, ctypes.c_int]
        L.hk_scene_chunk.restype = ctypes.c_int
        _lib = L
    return _lib


class HostWorld:
    """A world of chunk blobs traced by the host build of the kernels."""

    def __init__(self, svdag, chunk_log2, grid, lod_count, thr, blobs, describe_only=()):
        self.svdag = svdag
        self.desc = svdag.make_desc(chunk_log2, grid, lod_count, thr)
        self.n = grid[0] * grid[1] * grid[2]
        self._free = lib().hk_world_free
        self.w = lib().hk_world_new(ctypes.byref(self.desc))
        self.blobs = blobs
        for ci, b in blobs.items():
            assert lib().hk_upload(self.w, ci, b.ptr, int(ci in describe_only)) == 0

    def __del__(self):
        if getattr(self, "w", None):
            self._free(self.w)
            self.w = None

    def trace(self, frame, flags=0, threads=8):
        out = np.zeros((frame.width * frame.height, 4), np.uint32)
        view = np.zeros(self.n, np.uint32)
        assert lib().hk_trace(self.w, ctypes.byref(frame), flags, out.ctypes.data, view.ctypes.data, threads) == 0
        return out, view


WALK_EVENTS = ("iter", "descend", "exit", "sibling", "pop", "chunk_next", "chunk_visit", "chunk_enter", "hit",
               "tile_max_iter", "tiles")


def trace_counts(world, frame, flags=0, threads=8):
    """Records and walk-event counts of a host trace of `frame` (see
    hk_trace_counts): a dict over WALK_EVENTS."""
    out = np.zeros((frame.width * frame.height, 4), np.uint32)
    cnt = np.zeros(len(WALK_EVENTS), np.uint64)
    assert lib().hk_trace_counts(world.w, ctypes.byref(frame), flags, out.ctypes.data, threads,
                                 cnt.ctypes.data) == 0
    return out, dict(zip(WALK_EVENTS, (int(v) for v in cnt)))


def row_queue_tiles(tiles_x, tiles_y):
    """The per-view trace's tile queues, queue 0 first (see hk_row_queue_tiles)."""
    out = np.full(tiles_x * tiles_y + 64, 0xFFFFFFFF, np.uint32)
    n = lib().hk_row_queue_tiles(tiles_x, tiles_y, out.ctypes.data)
    return out[:n], out[n:]


def beam_cube(O, A, BX, BY, tile, lo, s):
    """(dropped, dist) of the beam pass for cube [lo, lo + s] and the tile with
    pixel corners tile = (x0, y0, x1, y1); dropped is None for a degenerate
    cone."""
    i64 = ctypes.c_int64 * 3
    d = ctypes.c_uint32(0)
    r = lib().hk_beam_cube(i64(*O), i64(*A), i64(*BX), i64(*BY), *tile, (ctypes.c_int32 * 3)(*lo), s,
                           ctypes.byref(d))
    return (None if r < 0 else bool(r)), d.value


def scene_chunk(sw, c, threads=8):
    """Chunk c of terrain world `sw` from the GPU generator's element code run
    on the host."""
    ip, dp, _ = sw._terrain_params()
    sel = sw.chunk_boxes(c)
    boxes = sel if len(sel) else np.zeros((1, 8), np.int32)
    out = np.empty(sw.S ** 3, np.uint8)
    rc = lib().hk_scene_chunk(ip, dp, ctypes.c_uint64(sw.seed), sw.chunk_log2, int(c[0]), int(c[1]), int(c[2]),
                              boxes.ctypes.data, len(sel), out.ctypes.data, threads)
    assert rc == 0, rc
    return out
