"""Helpers for GPU tests: build worlds on both sides and compare records."""
from __future__ import annotations

import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np

import oracle

REL_TOL_T = 1e-4


def note(msg: str):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def build_blobs(svdag, chunk_log2, lod_count, dense_by_ci, threads=8):
    def one(item):
        ci, g = item
        return ci, svdag.svd_chunk_build(g, chunk_log2, lod_count)
    with ThreadPoolExecutor(threads) as ex:
        return dict(ex.map(one, dense_by_ci.items()))


def gpu_world(svdag, torch, chunk_log2, grid, lod_count, blobs, thresholds=(256, 1024, 4096),
              extra_bytes=0):
    desc = svdag.make_desc(chunk_log2, grid, lod_count, thresholds)
    need = svdag.table_bytes(grid) + extra_bytes
    for b in blobs.values():
        need += sum(svdag.svd_blob_stats_get(b, k)["device_bytes"] for k in range(lod_count)) + 256
    pool = torch.empty(need, dtype=torch.uint8, device="cuda")
    w = svdag.svd_world_create(desc, pool)
    gx, gy, _ = grid
    for ci, b in blobs.items():
        c = (ci % gx, (ci // gx) % gy, ci // (gx * gy))
        svdag.svd_chunk_upload(w, c, b)
    torch.cuda.synchronize()
    return w


def oracle_world(chunk_log2, grid, lod_count, dense_by_ci, lods_needed=None):
    w = oracle.World(chunk_log2, grid, lod_count)
    for ci, g in dense_by_ci.items():
        w.add_chunk(ci, g, lods=None if lods_needed is None else [int(lods_needed[ci])])
    return w


def trace_gpu(svdag, torch, w, cam_or_frame, flags=0):
    n = cam_or_frame.width * cam_or_frame.height
    out = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    if isinstance(cam_or_frame, svdag.svd_ray_frame):
        svdag.svd_trace_frame(w, cam_or_frame, out, flags)
    else:
        svdag.svd_trace_view(w, cam_or_frame, out, flags)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def compare(svdag, raw: np.ndarray, ref: np.ndarray, idx=None, label=""):
    g = svdag.decode_hits(raw)
    if idx is not None:
        g = {k: v[idx] for k, v in g.items()}
    assert not np.any(g["chunk"] == svdag.FAULT_CHUNK), f"{label}: iteration guard fired"
    bad = np.nonzero(g["hit"] != ref["hit"])[0]
    assert bad.size == 0, f"{label}: hit flag differs at {bad[:10]} ({bad.size} rays)"
    h = ref["hit"] == 1
    for f in ("x", "y", "z", "lod", "face", "material"):
        exp = np.where(h, ref[f], 0)
        bad = np.nonzero(g[f] != exp)[0]
        assert bad.size == 0, f"{label}: {f} differs at {bad[:10]}: gpu {g[f][bad[:5]]} ref {exp[bad[:5]]}"
    ch = np.where(h, ref["chunk"].astype(np.int64), 0xFFFFFFFF)
    assert np.array_equal(g["chunk"].astype(np.int64), ch), f"{label}: chunk differs"
    gt, rt = g["t"].astype(np.float64), ref["t"]
    assert np.all(np.isinf(gt[~h])), f"{label}: miss t not inf"
    rel = np.abs(gt[h] - rt[h]) / np.maximum(np.abs(rt[h]), 1e-300)
    zero = rt[h] == 0
    assert np.all(gt[h][zero] == 0), f"{label}: t=0 not exact"
    assert np.all(rel[~zero] <= REL_TOL_T), f"{label}: t rel err {rel.max()}"
    return int(h.sum())
