"""CPU oracle (ctypes binding of ``liboracle.so``).

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; the library never imports it.  It
shares no code with the GPU library (see ``oracle.c`` for the definitions it
follows).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

HIT_DTYPE = np.dtype([
    ("x", np.int32), ("y", np.int32), ("z", np.int32), ("hit", np.int32),
    ("lod", np.int32), ("face", np.int32), ("material", np.int32), ("chunk", np.int32),
    ("t", np.float64), ("t_num", np.float64), ("t_den", np.float64),
])


COUNT_DTYPE = np.dtype([("chunk_visits", np.int32), ("chunk_entries", np.int32),
                        ("node_cubes", np.int32), ("leaf_cubes", np.int32),
                        ("preceding_siblings", np.int32), ("run_probes", np.int32)])


class _Frame(ctypes.Structure):
    _fields_ = [("O", ctypes.c_int64 * 3), ("A", ctypes.c_int64 * 3),
                ("BX", ctypes.c_int64 * 3), ("BY", ctypes.c_int64 * 3),
                ("G", ctypes.c_int32), ("W", ctypes.c_uint32), ("H", ctypes.c_uint32)]


class _Dag(ctypes.Structure):
    _fields_ = [("R", ctypes.c_uint32), ("root_level", ctypes.c_uint32),
                ("n_words", ctypes.c_uint32), ("words", ctypes.POINTER(ctypes.c_uint32)),
                ("n_leaves", ctypes.c_uint32), ("leaves", ctypes.POINTER(ctypes.c_uint64)),
                ("n_solid", ctypes.c_uint32), ("n_rle", ctypes.c_uint32),
                ("rle_start", ctypes.POINTER(ctypes.c_uint32)),
                ("rle_mat", ctypes.POINTER(ctypes.c_uint8)),
                ("level_nodes", ctypes.c_uint32 * 16)]


def lib_path() -> str:
    return os.path.join(_HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    src = os.path.join(_HERE, "oracle.c")
    out = lib_path()
    cmd = ["gcc", "-O2", "-Wall", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", out + ".tmp", src, "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


class _Touched(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("rays", "hits", "child_words", "leaves", "prefixes",
                                               "run_starts", "run_materials", "chunks", "dags")]


def _lib():
    global _LIB
    if _LIB is None:
        p = lib_path()
        if not os.path.exists(p):
            raise RuntimeError(f"{p} is not built; run __graft_entry__.build()")
        L = ctypes.CDLL(p)
        vp, u32, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int
        L.or_camera_frame.restype = i32
        L.or_camera_frame.argtypes = [vp, vp, vp, ctypes.c_float, u32, u32, ctypes.POINTER(_Frame)]
        L.or_downsample.argtypes = [vp, u32, vp]
        L.or_dag_build.restype = ctypes.POINTER(_Dag)
        L.or_dag_build.argtypes = [vp, u32]
        L.or_dag_free.argtypes = [ctypes.POINTER(_Dag)]
        L.or_dag_lookup.restype = i32
        L.or_dag_lookup.argtypes = [ctypes.POINTER(_Dag), u32, u32, u32,
                                    ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]
        L.or_dag_material.restype = ctypes.c_uint8
        L.or_dag_material.argtypes = [ctypes.POINTER(_Dag), u32]
        L.or_dag_expand.argtypes = [ctypes.POINTER(_Dag), vp]
        L.or_world_new.restype = vp
        L.or_world_new.argtypes = [u32, vp, u32]
        L.or_world_free.argtypes = [vp]
        L.or_world_set_dag.restype = i32
        L.or_world_set_dag.argtypes = [vp, u32, u32, ctypes.POINTER(_Dag)]
        L.or_world_set_dense.restype = i32
        L.or_world_set_dense.argtypes = [vp, u32, u32, vp]
        L.or_lod_pick.argtypes = [vp, vp, vp, vp]
        L.or_trace.argtypes = [vp, vp, vp, vp, u32, vp, i32, i32]
        L.or_trace_frame.argtypes = [vp, vp, ctypes.POINTER(_Frame), vp, u32, vp, i32, i32, vp]
        L.or_touch_frame.argtypes = [vp, vp, ctypes.POINTER(_Frame), i32, ctypes.POINTER(_Touched)]
        L.or_touch_frame.restype = None
        _LIB = L
    return _LIB


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# -- camera ---------------------------------------------------------------

class Frame:
    """Integer ray frame: D(px,py) = A + px*BX + py*BY, origin O (voxels*2^16)."""

    def __init__(self, f: _Frame):
        self._f = f
        self.O = np.array(f.O[:], dtype=np.int64)
        self.A = np.array(f.A[:], dtype=np.int64)
        self.BX = np.array(f.BX[:], dtype=np.int64)
        self.BY = np.array(f.BY[:], dtype=np.int64)
        self.G = int(f.G)
        self.W = int(f.W)
        self.H = int(f.H)

    def directions(self, idx: np.ndarray) -> np.ndarray:
        px = (idx % self.W).astype(np.int64)[:, None]
        py = (idx // self.W).astype(np.int64)[:, None]
        return self.A[None, :] + px * self.BX[None, :] + py * self.BY[None, :]


def camera_frame(cam) -> Frame:
    pos = np.array(cam.pos, np.float32)
    tgt = np.array(cam.target, np.float32)
    up = np.array(cam.up, np.float32)
    f = _Frame()
    rc = _lib().or_camera_frame(_ptr(pos), _ptr(tgt), _ptr(up), ctypes.c_float(cam.vfov_deg),
                                int(cam.width), int(cam.height), ctypes.byref(f))
    if rc != 0:
        raise ValueError(f"camera rejected ({rc})")
    return Frame(f)


# -- LOD pyramid / DAG -----------------------------------------------------

def downsample(grid: np.ndarray, R: int) -> np.ndarray:
    g = np.ascontiguousarray(grid, dtype=np.uint8).reshape(-1)
    assert g.size == R ** 3
    out = np.empty((R // 2) ** 3, np.uint8)
    _lib().or_downsample(_ptr(g), R, _ptr(out))
    return out


def pyramid(grid: np.ndarray, R: int, lod_count: int):
    out = [np.ascontiguousarray(grid, dtype=np.uint8).reshape(-1)]
    for k in range(1, lod_count):
        out.append(downsample(out[-1], R >> (k - 1)))
    return out


class Dag:
    """Canonical SVDAG of one grid (paper's node format)."""

    def __init__(self, grid: np.ndarray, R: int):
        g = np.ascontiguousarray(grid, dtype=np.uint8).reshape(-1)
        assert g.size == R ** 3
        p = _lib().or_dag_build(_ptr(g), R)
        if not p:
            raise ValueError("bad grid size")
        self._p = p
        self._owned = True

    def release(self):
        """Hand the C object over (to a world); this wrapper no longer frees it."""
        self._owned = False
        return self._p

    def __del__(self):
        if getattr(self, "_owned", False):
            _lib().or_dag_free(self._p)

    @property
    def d(self) -> _Dag:
        return self._p.contents

    @property
    def R(self):
        return self.d.R

    @property
    def n_solid(self):
        return self.d.n_solid

    @property
    def words(self) -> np.ndarray:
        n = self.d.n_words
        return np.ctypeslib.as_array(self.d.words, (n,)).copy() if n else np.zeros(0, np.uint32)

    @property
    def leaves(self) -> np.ndarray:
        n = self.d.n_leaves
        return np.ctypeslib.as_array(self.d.leaves, (n,)).copy() if n else np.zeros(0, np.uint64)

    @property
    def rle_start(self) -> np.ndarray:
        n = self.d.n_rle
        return np.ctypeslib.as_array(self.d.rle_start, (n,)).copy() if n else np.zeros(0, np.uint32)

    @property
    def rle_mat(self) -> np.ndarray:
        n = self.d.n_rle
        return np.ctypeslib.as_array(self.d.rle_mat, (n,)).copy() if n else np.zeros(0, np.uint8)

    @property
    def level_nodes(self):
        return list(self.d.level_nodes)

    def lookup(self, x, y, z):
        dfs = ctypes.c_uint32()
        lev = ctypes.c_uint32()
        s = _lib().or_dag_lookup(self._p, x, y, z, ctypes.byref(dfs), ctypes.byref(lev))
        return (True, dfs.value) if s else (False, lev.value)

    def material(self, dfs: int) -> int:
        return int(_lib().or_dag_material(self._p, dfs))

    def expand(self) -> np.ndarray:
        out = np.empty(self.R ** 3, np.uint8)
        _lib().or_dag_expand(self._p, _ptr(out))
        return out


# -- world / traversal -------------------------------------------------------

class World:
    def __init__(self, chunk_log2: int, grid, lod_count: int):
        g = np.array(grid, np.uint32)
        p = _lib().or_world_new(chunk_log2, _ptr(g), lod_count)
        if not p:
            raise ValueError("bad world")
        self._p = p
        self.chunk_log2 = chunk_log2
        self.grid = tuple(int(x) for x in grid)
        self.lod_count = lod_count

    def __del__(self):
        if getattr(self, "_p", None):
            _lib().or_world_free(self._p)
            self._p = None

    @property
    def nchunks(self):
        return self.grid[0] * self.grid[1] * self.grid[2]

    def chunk_index(self, c):
        return c[0] + self.grid[0] * (c[1] + self.grid[1] * c[2])

    def set_dag(self, ci: int, lod: int, dag: Dag | None):
        p = dag.release() if dag is not None else ctypes.POINTER(_Dag)()
        if _lib().or_world_set_dag(self._p, ci, lod, p) != 0:
            raise ValueError("set_dag")

    def set_dense(self, ci: int, lod: int, g: np.ndarray):
        g = np.ascontiguousarray(g, np.uint8).reshape(-1)
        assert g.size == (1 << (self.chunk_log2 - lod)) ** 3
        if _lib().or_world_set_dense(self._p, ci, lod, _ptr(g)) != 0:
            raise ValueError("set_dense")

    def add_chunk(self, ci: int, dense: np.ndarray, lods=None, keep_dense=False):
        """Build the LOD pyramid and a DAG per requested LOD for one chunk."""
        R = 1 << self.chunk_log2
        pyr = pyramid(dense, R, self.lod_count)
        for k in (range(self.lod_count) if lods is None else lods):
            self.set_dag(ci, k, Dag(pyr[k], R >> k))
            if keep_dense:
                self.set_dense(ci, k, pyr[k])
        return pyr

    def lod_pick(self, O, thresholds=(256, 1024, 4096)) -> np.ndarray:
        O = np.ascontiguousarray(O, np.int64)
        thr = np.ascontiguousarray(list(thresholds) + [0] * (3 - len(thresholds)), np.uint32)
        out = np.zeros(self.nchunks, np.uint8)
        _lib().or_lod_pick(self._p, _ptr(O), _ptr(thr), _ptr(out))
        return out

    def trace(self, lods, O, D, mode=1, threads=1) -> np.ndarray:
        lods = np.ascontiguousarray(lods, np.uint8)
        O = np.ascontiguousarray(O, np.int64)
        D = np.ascontiguousarray(D, np.int32).reshape(-1, 3)
        out = np.zeros(D.shape[0], HIT_DTYPE)
        _lib().or_trace(self._p, _ptr(lods), _ptr(O), _ptr(D), D.shape[0], _ptr(out), mode, threads)
        return out

    def touch_frame(self, lods, frame: Frame, threads=1) -> dict:
        """Counting instrumentation: the parts of the device layout that the
        frame's rays touch, each counted once (child words, leaf bitmaps,
        prefix counts, run starts and materials, view-table entries, DAG
        descriptors), with the ray and hit counts."""
        lods = np.ascontiguousarray(lods, np.uint8)
        t = _Touched()
        _lib().or_touch_frame(self._p, _ptr(lods), ctypes.byref(frame._f), threads, ctypes.byref(t))
        return {n: int(getattr(t, n)) for n, _ in _Touched._fields_}

    def trace_frame(self, lods, frame: Frame, idx=None, mode=1, threads=1, counts=False):
        """Hits of the frame's pixels (all, or the indices `idx`).  With
        counts=True also returns the per-ray visit counts (COUNT_DTYPE)."""
        lods = np.ascontiguousarray(lods, np.uint8)
        if idx is None:
            n = frame.W * frame.H
            ip = ctypes.c_void_p(0)
        else:
            idx = np.ascontiguousarray(idx, np.uint32)
            n = idx.size
            ip = _ptr(idx)
        out = np.zeros(n, HIT_DTYPE)
        cnt = np.zeros(n, COUNT_DTYPE) if counts else None
        _lib().or_trace_frame(self._p, _ptr(lods), ctypes.byref(frame._f), ip, n, _ptr(out),
                              mode, threads, _ptr(cnt) if counts else ctypes.c_void_p(0))
        return (out, cnt) if counts else out
