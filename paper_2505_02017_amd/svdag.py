"""ctypes binding of libsvdag (include/svdag.h).

Argument marshalling only: every step of the build runs in the library's
C++ and every step of a traced view runs in its HIP kernels.  PyTorch is used
for device memory (pool and output tensors) and streams.  Importing this
module fails loudly if ``libsvdag.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvdag.so")

SVD_OK = 0
SVD_EINVAL = -1
SVD_ENOMEM = -2
SVD_EDEVICE = -3
SVD_EFORMAT = -4
SVD_ERANGE = -5
SVD_ENOTFOUND = -6
SVD_EIO = -7
SVD_NO_CULL = 1
SVD_BEAM = 2
SVD_MAX_TIMED_PASSES = 65536
FAULT_CHUNK = 0xFFFFFFFE  # written by the trace if its chunk-walk iteration guard fires (never expected)
CHUNK_NOT_LOADED = 0xFFFFFFFD  # a ray reached a chunk whose picked LOD is only described

_NAMES = {SVD_EINVAL: "EINVAL", SVD_ENOMEM: "ENOMEM", SVD_EDEVICE: "EDEVICE",
          SVD_EFORMAT: "EFORMAT", SVD_ERANGE: "ERANGE", SVD_ENOTFOUND: "ENOTFOUND",
          SVD_EIO: "EIO"}

EXPORTS = [
    "svd_last_error", "svd_chunk_build", "svd_blob_to_bytes", "svd_blob_from_bytes",
    "svd_blob_free", "svd_free", "svd_blob_stats_get", "svd_blob_canonical",
    "svd_world_create", "svd_world_destroy", "svd_world_pool_used", "svd_chunk_upload",
    "svd_chunk_evict", "svd_chunk_upload_lods", "svd_chunk_evict_lods", "svd_camera_frame", "svd_trace_view", "svd_trace_frame",
    "svd_view_stage", "svd_view_beam", "svd_view_trace", "svd_view_table",
    "svd_world_set_occupancy", "svd_world_get_occupancy",
    "svd_batch_create", "svd_batch_destroy", "svd_batch_trace", "svd_batch_trace_frames",
    "svd_batch_set_tiling", "svd_batch_set_occupancy", "svd_batch_get_tiling", "svd_batch_tune",
    "svd_server_create", "svd_server_set_chunk", "svd_server_submit", "svd_server_poll",
    "svd_server_stats_get", "svd_server_destroy", "svd_batch_trace_frames_static",
    "svd_world_set_tiling", "svd_world_get_tiling", "svd_world_tune", "svd_batch_tune_cached",
    "svd_kernel_hash", "svd_tune_cache_lookup", "svd_tune_cache_store",
    "svd_world_time_traces", "svd_world_trace_times",
]


class SvdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class svd_world_desc(ctypes.Structure):
    _fields_ = [("chunk_log2", ctypes.c_uint32), ("grid", ctypes.c_uint32 * 3),
                ("lod_count", ctypes.c_uint32), ("lod_threshold", ctypes.c_uint32 * 3)]


class svd_camera(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_float * 3), ("target", ctypes.c_float * 3),
                ("up", ctypes.c_float * 3), ("vfov_deg", ctypes.c_float),
                ("width", ctypes.c_uint32), ("height", ctypes.c_uint32)]


class svd_ray_frame(ctypes.Structure):
    _fields_ = [("O", ctypes.c_int64 * 3), ("A", ctypes.c_int64 * 3),
                ("BX", ctypes.c_int64 * 3), ("BY", ctypes.c_int64 * 3),
                ("G", ctypes.c_int32), ("width", ctypes.c_uint32), ("height", ctypes.c_uint32)]


class svd_server_desc(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_uint32), ("max_views", ctypes.c_uint32), ("inflight", ctypes.c_uint32),
                ("tile_w", ctypes.c_uint32), ("claim", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("max_rays", ctypes.c_uint64), ("streaming_factor", ctypes.c_float),
                ("reserved", ctypes.c_uint32)]


class svd_request_done(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("batch_views", ctypes.c_uint32),
                ("t_submit", ctypes.c_double), ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double)]


class svd_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in (
        "submitted", "completed", "failed", "launches", "uploads", "upload_bytes", "evictions",
        "evict_bytes", "memory_waits", "pool_used", "prefetches", "prefetch_bytes")]


class svd_tune_result(ctypes.Structure):
    _fields_ = [("tile_w", ctypes.c_uint32), ("claim", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32),
                ("from_cache", ctypes.c_uint32), ("ms", ctypes.c_float), ("configs_timed", ctypes.c_uint32),
                ("key", ctypes.c_char * 384)]

    def as_dict(self) -> dict:
        return {"tile": f"{self.tile_w}x{64 // self.tile_w}", "tile_w": self.tile_w, "claim": self.claim,
                "blocks_per_cu": self.blocks_per_cu, "from_cache": bool(self.from_cache),
                "ms": round(float(self.ms), 4), "configs_timed": self.configs_timed,
                "key": self.key.decode()}


class svd_blob_stats(ctypes.Structure):
    _fields_ = [("R", ctypes.c_uint32), ("n_words", ctypes.c_uint32),
                ("n_leaves", ctypes.c_uint32), ("n_rle", ctypes.c_uint32),
                ("n_solid", ctypes.c_uint32), ("level_nodes", ctypes.c_uint32 * 16),
                ("aabb_lo", ctypes.c_uint16 * 3), ("aabb_hi", ctypes.c_uint16 * 3),
                ("device_bytes", ctypes.c_uint64)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        # PyTorch ships its own HIP runtime under the same soname: load it
        # first so that the library binds to it.  Loaded the other way round,
        # the process would hold two HIP runtimes, and the library's would not
        # see the device or the memory that torch allocates.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        vp, u32, i32, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int, ctypes.c_size_t
        L.svd_last_error.restype = ctypes.c_char_p
        L.svd_last_error.argtypes = []
        L.svd_chunk_build.argtypes = [vp, u32, u32, ctypes.POINTER(vp)]
        L.svd_blob_to_bytes.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(sz)]
        L.svd_blob_from_bytes.argtypes = [vp, sz, ctypes.POINTER(vp)]
        L.svd_blob_free.argtypes = [vp]
        L.svd_blob_free.restype = None
        L.svd_free.argtypes = [vp]
        L.svd_free.restype = None
        L.svd_blob_stats_get.argtypes = [vp, u32, ctypes.POINTER(svd_blob_stats)]
        L.svd_blob_canonical.argtypes = [vp, u32, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                         ctypes.POINTER(vp), ctypes.POINTER(vp)]
        L.svd_world_create.argtypes = [ctypes.POINTER(svd_world_desc), vp, sz, ctypes.POINTER(vp)]
        L.svd_world_destroy.argtypes = [vp]
        L.svd_world_destroy.restype = None
        L.svd_world_pool_used.argtypes = [vp, ctypes.POINTER(sz)]
        L.svd_chunk_upload.argtypes = [vp, ctypes.POINTER(u32), vp, vp]
        L.svd_chunk_evict.argtypes = [vp, ctypes.POINTER(u32)]
        L.svd_chunk_upload_lods.argtypes = [vp, ctypes.POINTER(u32), vp, u32, vp]
        L.svd_chunk_evict_lods.argtypes = [vp, ctypes.POINTER(u32), u32, vp]
        L.svd_camera_frame.argtypes = [ctypes.POINTER(svd_camera), ctypes.POINTER(svd_ray_frame)]
        L.svd_trace_view.argtypes = [vp, ctypes.POINTER(svd_camera), vp, u32, vp]
        L.svd_trace_frame.argtypes = [vp, ctypes.POINTER(svd_ray_frame), vp, u32, vp]
        L.svd_view_table.argtypes = [vp, ctypes.POINTER(u32), u32, vp]
        L.svd_view_stage.argtypes = [vp, ctypes.POINTER(svd_ray_frame), u32, vp]
        L.svd_view_trace.argtypes = [vp, ctypes.POINTER(svd_ray_frame), vp, vp]
        L.svd_view_beam.argtypes = [vp, ctypes.POINTER(svd_ray_frame), vp, vp]
        L.svd_world_time_traces.argtypes = [vp, u32]
        L.svd_world_trace_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), u32, ctypes.POINTER(u32)]
        L.svd_world_set_occupancy.argtypes = [vp, u32]
        L.svd_world_get_occupancy.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32)]
        u64 = ctypes.c_uint64
        L.svd_batch_create.argtypes = [vp, u32, ctypes.POINTER(vp)]
        L.svd_batch_destroy.argtypes = [vp]
        L.svd_batch_destroy.restype = None
        L.svd_batch_trace.argtypes = [vp, ctypes.POINTER(svd_camera), u32, vp, u64, u32, vp]
        L.svd_batch_trace_frames.argtypes = [vp, ctypes.POINTER(svd_ray_frame), u32, vp, u64, u32, vp]
        L.svd_batch_set_tiling.argtypes = [vp, u32, u32]
        L.svd_batch_set_occupancy.argtypes = [vp, u32]
        L.svd_batch_get_tiling.argtypes = [vp, ctypes.POINTER(u32), ctypes.POINTER(u32), ctypes.POINTER(u32)]
        L.svd_batch_tune.argtypes = [vp, ctypes.POINTER(svd_camera), u32, vp, u64, u32, vp,
                                     ctypes.POINTER(ctypes.c_float)]
        L.svd_batch_trace_frames_static.argtypes = [vp, ctypes.POINTER(svd_ray_frame), u32, vp, u64, u32, vp]
        L.svd_world_set_tiling.argtypes = [vp, u32]
        L.svd_world_get_tiling.argtypes = [vp, ctypes.POINTER(u32)]
        L.svd_world_tune.argtypes = [vp, ctypes.POINTER(svd_ray_frame), u32, vp, u64, u32, u32, ctypes.c_char_p,
                                     vp, ctypes.POINTER(svd_tune_result)]
        L.svd_batch_tune_cached.argtypes = [vp, ctypes.POINTER(svd_camera), u32, vp, u64, u32, ctypes.c_char_p,
                                            vp, ctypes.POINTER(svd_tune_result)]
        L.svd_kernel_hash.argtypes = []
        L.svd_tune_cache_lookup.argtypes = [ctypes.c_char_p, ctypes.c_char_p, ctypes.POINTER(svd_tune_result)]
        L.svd_tune_cache_store.argtypes = [ctypes.c_char_p, ctypes.POINTER(svd_tune_result)]
        L.svd_server_create.argtypes = [vp, ctypes.POINTER(svd_server_desc), ctypes.POINTER(vp)]
        L.svd_server_set_chunk.argtypes = [vp, ctypes.POINTER(u32), vp]
        L.svd_server_submit.argtypes = [vp, ctypes.POINTER(svd_camera), vp, u32, u64]
        L.svd_server_poll.argtypes = [vp, ctypes.POINTER(svd_request_done), u32, ctypes.POINTER(u32), u32]
        L.svd_server_stats_get.argtypes = [vp, ctypes.POINTER(svd_server_stats)]
        L.svd_server_destroy.argtypes = [vp]
        L.svd_server_destroy.restype = None
        for n in EXPORTS:
            if n not in ("svd_last_error", "svd_blob_free", "svd_free", "svd_world_destroy",
                         "svd_batch_destroy", "svd_server_destroy", "svd_kernel_hash"):
                getattr(L, n).restype = i32
        L.svd_kernel_hash.restype = ctypes.c_char_p
        _lib = L
    return _lib


def svd_last_error() -> str:
    return lib().svd_last_error().decode()


def _check(rc: int):
    if rc != SVD_OK:
        raise SvdError(rc, svd_last_error())


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    if hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    return ctypes.c_void_p(int(stream))


# ------------------------------------------------------------------ blobs

class Blob:
    """Host-side built chunk (all LODs); frees itself."""

    def __init__(self, ptr: int):
        self._p = ctypes.c_void_p(ptr)
        self._free = lib().svd_blob_free  # held: module globals may be gone at exit

    def __del__(self):
        if getattr(self, "_p", None) and self._p.value:
            self._free(self._p)
            self._p = None

    @property
    def ptr(self):
        return self._p


def svd_chunk_build(dense: np.ndarray, chunk_log2: int, lod_count: int) -> Blob:
    d = np.ascontiguousarray(dense, dtype=np.uint8).reshape(-1)
    if d.size != (1 << (3 * chunk_log2)):
        raise SvdError(SVD_EINVAL, "dense grid has the wrong size")
    out = ctypes.c_void_p()
    _check(lib().svd_chunk_build(d.ctypes.data, chunk_log2, lod_count, ctypes.byref(out)))
    return Blob(out.value)


def svd_blob_to_bytes(b: Blob) -> bytes:
    p = ctypes.c_void_p()
    n = ctypes.c_size_t()
    _check(lib().svd_blob_to_bytes(b.ptr, ctypes.byref(p), ctypes.byref(n)))
    try:
        return ctypes.string_at(p, n.value)
    finally:
        lib().svd_free(p)


def svd_blob_from_bytes(data: bytes) -> Blob:
    buf = ctypes.create_string_buffer(bytes(data), len(data))
    out = ctypes.c_void_p()
    _check(lib().svd_blob_from_bytes(buf, len(data), ctypes.byref(out)))
    return Blob(out.value)


def svd_blob_stats_get(b: Blob, lod: int) -> dict:
    s = svd_blob_stats()
    _check(lib().svd_blob_stats_get(b.ptr, lod, ctypes.byref(s)))
    return dict(R=s.R, n_words=s.n_words, n_leaves=s.n_leaves, n_rle=s.n_rle, n_solid=s.n_solid,
                level_nodes=list(s.level_nodes), aabb_lo=list(s.aabb_lo), aabb_hi=list(s.aabb_hi),
                device_bytes=int(s.device_bytes))


def svd_blob_canonical(b: Blob, lod: int):
    """Copies of the canonical arrays (words, leaves, rle_start, rle_mat)."""
    st = svd_blob_stats_get(b, lod)
    w, l, rs, rm = (ctypes.c_void_p() for _ in range(4))
    _check(lib().svd_blob_canonical(b.ptr, lod, ctypes.byref(w), ctypes.byref(l),
                                    ctypes.byref(rs), ctypes.byref(rm)))

    def arr(p, n, t):
        if n == 0:
            return np.zeros(0, t)
        return np.ctypeslib.as_array(ctypes.cast(p, ctypes.POINTER(np.ctypeslib.as_ctypes_type(t))),
                                     (n,)).copy()
    return (arr(w, st["n_words"], np.uint32), arr(l, st["n_leaves"], np.uint64),
            arr(rs, st["n_rle"], np.uint32), arr(rm, st["n_rle"], np.uint8))


# ------------------------------------------------------------------ world

def make_desc(chunk_log2: int, grid, lod_count: int, thresholds=(256, 1024, 4096)) -> svd_world_desc:
    d = svd_world_desc()
    d.chunk_log2 = chunk_log2
    d.grid[:] = [int(g) for g in grid]
    d.lod_count = lod_count
    t = list(thresholds) + [0] * (3 - len(thresholds))
    d.lod_threshold[:] = [int(x) for x in t[:3]]
    return d


def table_bytes(grid) -> int:
    n = int(grid[0]) * int(grid[1]) * int(grid[2])
    return n * 4 * 64 + (n * 4 + 255) // 256 * 256 + 2048


def batch_bytes(nchunks: int, max_views: int) -> int:
    """Pool bytes a batch of max_views views takes (see svd_batch_create)."""
    return 2048 + 256 + 256 * max_views + (max_views * nchunks * 4 + 255) // 256 * 256


class World:
    """A device world over a caller-owned pool tensor (torch uint8, on a GPU)."""

    def __init__(self, ptr: int, pool, desc: svd_world_desc):
        self._p = ctypes.c_void_p(ptr)
        self.pool = pool          # keeps the device memory alive
        self.desc = desc
        self.grid = tuple(desc.grid)
        self.nchunks = self.grid[0] * self.grid[1] * self.grid[2]
        self._blobs = {}          # uploaded blobs stay alive until replaced or evicted
        self._free = lib().svd_world_destroy

    @property
    def ptr(self):
        return self._p

    def __del__(self):
        if getattr(self, "_p", None) and self._p.value:
            self._free(self._p)
            self._p = None


def svd_world_create(desc: svd_world_desc, pool) -> World:
    assert pool.dtype.itemsize == 1 and pool.is_contiguous()
    out = ctypes.c_void_p()
    _check(lib().svd_world_create(ctypes.byref(desc), ctypes.c_void_p(pool.data_ptr()),
                                  pool.numel(), ctypes.byref(out)))
    return World(out.value, pool, desc)


def svd_world_destroy(w: World):
    if w._p and w._p.value:
        lib().svd_world_destroy(w._p)
        w._p = None


def svd_world_pool_used(w: World) -> int:
    n = ctypes.c_size_t()
    _check(lib().svd_world_pool_used(w.ptr, ctypes.byref(n)))
    return n.value


def _c3(c):
    return (ctypes.c_uint32 * 3)(*[int(v) for v in c])


def svd_chunk_upload(w: World, c, b: Blob, stream=None):
    _check(lib().svd_chunk_upload(w.ptr, _c3(c), b.ptr, _stream_ptr(stream)))
    w._blobs[tuple(int(v) for v in c)] = b


def svd_chunk_evict(w: World, c):
    _check(lib().svd_chunk_evict(w.ptr, _c3(c)))
    w._blobs.pop(tuple(int(v) for v in c), None)


def svd_chunk_upload_lods(w: World, c, b: Blob, lod_mask: int, stream=None):
    _check(lib().svd_chunk_upload_lods(w.ptr, _c3(c), b.ptr, lod_mask, _stream_ptr(stream)))
    w._blobs[tuple(int(v) for v in c)] = b


def svd_chunk_evict_lods(w: World, c, lod_mask: int, stream=None):
    _check(lib().svd_chunk_evict_lods(w.ptr, _c3(c), lod_mask, _stream_ptr(stream)))


def to_camera(cam) -> svd_camera:
    c = svd_camera()
    c.pos[:] = [float(v) for v in cam.pos]
    c.target[:] = [float(v) for v in cam.target]
    c.up[:] = [float(v) for v in cam.up]
    c.vfov_deg = float(cam.vfov_deg)
    c.width = int(cam.width)
    c.height = int(cam.height)
    return c


def svd_camera_frame(cam) -> svd_ray_frame:
    f = svd_ray_frame()
    _check(lib().svd_camera_frame(ctypes.byref(to_camera(cam)), ctypes.byref(f)))
    return f


def make_frame(O, A, BX, BY, width, height, G=0) -> svd_ray_frame:
    f = svd_ray_frame()
    f.O[:] = [int(v) for v in O]
    f.A[:] = [int(v) for v in A]
    f.BX[:] = [int(v) for v in BX]
    f.BY[:] = [int(v) for v in BY]
    f.G = G
    f.width = width
    f.height = height
    return f


def _out_ptr(out, n: int):
    assert out.is_cuda and out.is_contiguous() and out.numel() * out.element_size() >= 16 * n
    return ctypes.c_void_p(out.data_ptr())


def svd_trace_view(w: World, cam, out, flags: int = 0, stream=None):
    c = cam if isinstance(cam, svd_camera) else to_camera(cam)
    _check(lib().svd_trace_view(w.ptr, ctypes.byref(c), _out_ptr(out, c.width * c.height),
                                flags, _stream_ptr(stream)))


def svd_trace_frame(w: World, frame: svd_ray_frame, out, flags: int = 0, stream=None):
    _check(lib().svd_trace_frame(w.ptr, ctypes.byref(frame), _out_ptr(out, frame.width * frame.height),
                                 flags, _stream_ptr(stream)))


def svd_view_stage(w: World, frame: svd_ray_frame, flags: int = 0, stream=None):
    _check(lib().svd_view_stage(w.ptr, ctypes.byref(frame), flags, _stream_ptr(stream)))


def svd_view_beam(w: World, frame: svd_ray_frame, out, stream=None):
    _check(lib().svd_view_beam(w.ptr, ctypes.byref(frame), _out_ptr(out, frame.width * frame.height),
                               _stream_ptr(stream)))


def svd_view_trace(w: World, frame: svd_ray_frame, out, stream=None):
    _check(lib().svd_view_trace(w.ptr, ctypes.byref(frame), _out_ptr(out, frame.width * frame.height),
                                _stream_ptr(stream)))


def svd_world_time_traces(w: World, n: int):
    _check(lib().svd_world_time_traces(w.ptr, n))


def svd_world_trace_times(w: World, n: int):
    """Durations (ms) of the first min(n, recorded) timed trace passes."""
    ms = (ctypes.c_float * max(1, n))()
    count = ctypes.c_uint32()
    _check(lib().svd_world_trace_times(w.ptr, ms, n, ctypes.byref(count)))
    return [ms[i] for i in range(count.value)]


def svd_world_set_occupancy(w: World, blocks_per_cu: int):
    _check(lib().svd_world_set_occupancy(w.ptr, blocks_per_cu))


def svd_world_get_occupancy(w: World):
    """(blocks per CU of the per-view trace, the most that fit a CU)."""
    cur, mx = ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().svd_world_get_occupancy(w.ptr, ctypes.byref(cur), ctypes.byref(mx)))
    return cur.value, mx.value


def svd_world_set_tiling(w: World, tile_w: int):
    _check(lib().svd_world_set_tiling(w.ptr, tile_w))


def svd_world_get_tiling(w: World) -> int:
    """Wave tile width of the per-view passes (tile = tile_w x 64/tile_w)."""
    tw = ctypes.c_uint32()
    _check(lib().svd_world_get_tiling(w.ptr, ctypes.byref(tw)))
    return tw.value


def svd_world_tune(w: World, frames, out, flags: int = 0, reps: int = 3, cache_path=None,
                   stream=None) -> "svd_tune_result":
    """Autotune the per-view tile and occupancy on these frames (see
    svd_world_tune in svdag.h); cache_path None: no cache."""
    arr = (svd_ray_frame * len(frames))(*frames)
    assert out.is_cuda and out.is_contiguous()
    res = svd_tune_result()
    _check(lib().svd_world_tune(w.ptr, arr, len(frames), ctypes.c_void_p(out.data_ptr()),
                                out.numel() * out.element_size() // 16, flags, reps, _cache_arg(cache_path),
                                _stream_ptr(stream), ctypes.byref(res)))
    return res


def svd_tune_cache_lookup(cache_path, key: str):
    """The cached entry for `key` (svd_tune_result), or None."""
    res = svd_tune_result()
    rc = lib().svd_tune_cache_lookup(os.fsencode(cache_path), key.encode(), ctypes.byref(res))
    if rc == SVD_ENOTFOUND:
        return None
    _check(rc)
    return res


def svd_tune_cache_store(cache_path, key: str, tile_w: int, claim: int, blocks_per_cu: int, ms: float = 0.0):
    res = svd_tune_result(tile_w=tile_w, claim=claim, blocks_per_cu=blocks_per_cu, ms=ms)
    res.key = key.encode()
    _check(lib().svd_tune_cache_store(os.fsencode(cache_path), ctypes.byref(res)))


def svd_kernel_hash() -> str:
    """Kernel source hash the loaded library was built from."""
    return lib().svd_kernel_hash().decode()


def svd_view_table(w: World, stream=None) -> np.ndarray:
    out = np.zeros(w.nchunks, np.uint32)
    _check(lib().svd_view_table(w.ptr, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                w.nchunks, _stream_ptr(stream)))
    return out


# ------------------------------------------------------------------ batches

class Batch:
    """Views traced together in one graph launch (see svd_batch_create)."""

    def __init__(self, ptr: int, world: World):
        self._p = ctypes.c_void_p(ptr)
        self.world = world  # the batch lives in the world's pool
        self._free = lib().svd_batch_destroy

    @property
    def ptr(self):
        return self._p

    def __del__(self):
        if getattr(self, "_p", None) and self._p.value:
            self._free(self._p)
            self._p = None


def svd_batch_create(w: World, max_views: int) -> Batch:
    out = ctypes.c_void_p()
    _check(lib().svd_batch_create(w.ptr, max_views, ctypes.byref(out)))
    return Batch(out.value, w)


def svd_batch_destroy(b: Batch):
    if b._p and b._p.value:
        lib().svd_batch_destroy(b._p)
        b._p = None


def _cam_array(cams):
    arr = (svd_camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = c if isinstance(c, svd_camera) else to_camera(c)
    return arr


def batch_records(cams) -> int:
    return sum(int(c.width) * int(c.height) for c in cams)


def _batch_out(out):
    """Device pointer and record capacity of a batch output (the library
    checks the capacity against the views)."""
    assert out.is_cuda and out.is_contiguous()
    return ctypes.c_void_p(out.data_ptr()), out.numel() * out.element_size() // 16


def svd_batch_trace(b: Batch, cams, out, flags: int = 0, stream=None):
    arr = _cam_array(cams)
    ptr, cap = _batch_out(out)
    _check(lib().svd_batch_trace(b.ptr, arr, len(cams), ptr, cap, flags, _stream_ptr(stream)))


def svd_batch_trace_frames(b: Batch, frames, out, flags: int = 0, stream=None):
    arr = (svd_ray_frame * len(frames))(*frames)
    ptr, cap = _batch_out(out)
    _check(lib().svd_batch_trace_frames(b.ptr, arr, len(frames), ptr, cap, flags, _stream_ptr(stream)))


def svd_batch_trace_frames_static(w: World, frames, out, flags: int = 0, stream=None):
    """Batch of frames without a batch object: nothing is allocated (the
    library's static per-GPU scratch holds the queue, views and tables)."""
    arr = (svd_ray_frame * len(frames))(*frames)
    ptr, cap = _batch_out(out)
    _check(lib().svd_batch_trace_frames_static(w.ptr, arr, len(frames), ptr, cap, flags, _stream_ptr(stream)))


def svd_batch_set_tiling(b: Batch, tile_w: int, claim: int):
    _check(lib().svd_batch_set_tiling(b.ptr, tile_w, claim))


def svd_batch_set_occupancy(b: Batch, blocks_per_cu: int):
    _check(lib().svd_batch_set_occupancy(b.ptr, blocks_per_cu))


def svd_batch_get_tiling(b: Batch):
    """(tile width, claim, blocks per CU) of the batch trace."""
    tw, cl, oc = ctypes.c_uint32(), ctypes.c_uint32(), ctypes.c_uint32()
    _check(lib().svd_batch_get_tiling(b.ptr, ctypes.byref(tw), ctypes.byref(cl), ctypes.byref(oc)))
    return tw.value, cl.value, oc.value


def _cache_arg(cache_path):
    return None if not cache_path else os.fsencode(cache_path)


def svd_batch_tune_cached(b: Batch, cams, out, reps: int = 3, cache_path=None, stream=None) -> svd_tune_result:
    """svd_batch_tune through the tuning cache file (None: no cache)."""
    arr = _cam_array(cams)
    ptr, cap = _batch_out(out)
    res = svd_tune_result()
    _check(lib().svd_batch_tune_cached(b.ptr, arr, len(cams), ptr, cap, reps, _cache_arg(cache_path),
                                       _stream_ptr(stream), ctypes.byref(res)))
    return res


def svd_batch_tune(b: Batch, cams, out, reps: int = 3, stream=None):
    """Autotune the batch's tiling and occupancy on these cameras; returns
    (tile_w, claim, blocks_per_cu, ms)."""
    arr = _cam_array(cams)
    ptr, cap = _batch_out(out)
    ms = ctypes.c_float()
    _check(lib().svd_batch_tune(b.ptr, arr, len(cams), ptr, cap, reps, _stream_ptr(stream),
                                ctypes.byref(ms)))
    tw, cl, oc = svd_batch_get_tiling(b)
    return tw, cl, oc, ms.value


# ------------------------------------------------------------------ serving

SVD_SERVE_BATCHED = 0
SVD_SERVE_PLAIN = 1
SVD_SERVE_PLAIN_CONCURRENT = 2


class Server:
    """A request server over a world (see svd_server_create).  Keeps the
    world and the chunk source blobs alive while it lives."""

    def __init__(self, ptr: int, world: World):
        self._p = ctypes.c_void_p(ptr)
        self.world = world
        self._sources = {}
        self._free = lib().svd_server_destroy

    @property
    def ptr(self):
        return self._p

    def __del__(self):
        if getattr(self, "_p", None) and self._p.value:
            self._free(self._p)
            self._p = None


def svd_server_create(w: World, mode: int = SVD_SERVE_BATCHED, max_views: int = 64, inflight: int = 2,
                      max_rays: int = 1 << 24, tile_w: int = 0, claim: int = 0, blocks_per_cu: int = 0,
                      streaming_factor: float = 0.0) -> Server:
    d = svd_server_desc(mode=mode, max_views=max_views, inflight=inflight, tile_w=tile_w, claim=claim,
                        blocks_per_cu=blocks_per_cu, max_rays=max_rays, streaming_factor=streaming_factor)
    out = ctypes.c_void_p()
    _check(lib().svd_server_create(w.ptr, ctypes.byref(d), ctypes.byref(out)))
    return Server(out.value, w)


def svd_server_set_chunk(s: Server, c, b: Blob):
    _check(lib().svd_server_set_chunk(s.ptr, _c3(c), b.ptr))
    s._sources[tuple(int(v) for v in c)] = b


def svd_server_submit(s: Server, cam, out, tag: int, flags: int = 0):
    c = cam if isinstance(cam, svd_camera) else to_camera(cam)
    _check(lib().svd_server_submit(s.ptr, ctypes.byref(c), _out_ptr(out, c.width * c.height), flags, tag))


def svd_server_poll(s: Server, max_n: int = 256, wait_us: int = 0) -> list:
    """Finished requests: list of dicts (tag, status, batch_views, t_submit,
    t_launch, t_done; seconds on the server's clock)."""
    arr = (svd_request_done * max_n)()
    n = ctypes.c_uint32()
    _check(lib().svd_server_poll(s.ptr, arr, max_n, ctypes.byref(n), wait_us))
    return [{k: getattr(arr[i], k) for k, _ in svd_request_done._fields_} for i in range(n.value)]


def svd_server_stats_get(s: Server) -> dict:
    st = svd_server_stats()
    _check(lib().svd_server_stats_get(s.ptr, ctypes.byref(st)))
    return {k: int(getattr(st, k)) for k, _ in svd_server_stats._fields_}


def svd_server_destroy(s: Server):
    if s._p and s._p.value:
        lib().svd_server_destroy(s._p)
        s._p = None


# ------------------------------------------------------------------ records

def decode_hits(raw: np.ndarray) -> dict:
    """Fields of svd_hit records (array of uint32 with 4 words per pixel)."""
    r = np.ascontiguousarray(raw).view(np.uint32).reshape(-1, 4)
    xy, zf, chunk = r[:, 0], r[:, 1], r[:, 3]
    return dict(
        x=(xy & 0xFFFF).astype(np.int32), y=(xy >> 16).astype(np.int32),
        z=(zf & 0xFFFF).astype(np.int32), lod=((zf >> 16) & 0xF).astype(np.int32),
        face=((zf >> 20) & 0x7).astype(np.int32), hit=((zf >> 23) & 1).astype(np.int32),
        material=(zf >> 24).astype(np.int32), t=r[:, 2].view(np.float32), chunk=chunk,
    )
