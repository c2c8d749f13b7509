"""GPU parity at full workload sizes, in the launch configuration bench.py
times (svd_view_stage + svd_view_trace on torch's stream): whole frames
compared with the oracle, plus properties checked on every pixel."""
import os
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from gpu_util import compare, note
from paper_2505_02017_amd import scenes

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_02017_amd import svdag
    svdag.lib()
    return svdag, torch


def _build(svdag, torch, kind, seed, lod_count, thr, nviews):
    """Generate every chunk once; library blobs for all LODs, oracle DAGs only
    for the LODs the first `nviews` views pick."""
    sw = scenes.SceneWorld(kind, seed)
    CL, (gx, gy, gz) = sw.chunk_log2, sw.grid
    nch = gx * gy * gz
    cams = sw.views(nviews, 1)
    ow = oracle.World(CL, sw.grid, lod_count)
    frames = [oracle.camera_frame(c) for c in cams]
    vlods = [ow.lod_pick(f.O, thr) for f in frames]
    need = [sorted({int(v[ci]) for v in vlods}) for ci in range(nch)]
    t0 = time.time()

    def work(ci):
        c = (ci % gx, (ci // gx) % gy, ci // (gx * gy))
        g = sw.chunk(c, threads=1 if nch > 1 else NT)
        b = svdag.svd_chunk_build(g, CL, lod_count)
        pyr = oracle.pyramid(g, 1 << CL, max(need[ci]) + 1)
        return ci, c, b, [(k, oracle.Dag(pyr[k], (1 << CL) >> k)) for k in need[ci]]

    blobs = {}
    with ThreadPoolExecutor(NT if nch > 1 else 1) as ex:
        for ci, c, b, od in ex.map(work, range(nch)):
            blobs[c] = b
            for k, d in od:
                ow.set_dag(ci, k, d)
    note(f"{kind}: built {nch} chunks in {time.time() - t0:.1f}s")
    desc = svdag.make_desc(CL, sw.grid, lod_count, thr)
    dev = sum(svdag.svd_blob_stats_get(b, k)["device_bytes"] for b in blobs.values() for k in range(lod_count))
    pool = torch.empty(svdag.table_bytes(sw.grid) + dev + 256 * nch, dtype=torch.uint8, device="cuda")
    w = svdag.svd_world_create(desc, pool)
    for c, b in blobs.items():
        svdag.svd_chunk_upload(w, c, b)
    torch.cuda.synchronize()
    return sw, w, ow, cams, frames, vlods


def _trace_like_bench(svdag, torch, w, cam):
    f = svdag.svd_camera_frame(cam)
    out = torch.empty((f.width * f.height, 4), dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    svdag.svd_view_stage(w, f, 0, s)
    svdag.svd_view_trace(w, f, out, s)
    torch.cuda.synchronize()
    return out.cpu().numpy(), svdag.svd_view_table(w)


def _properties(svdag, raw, vt, sw):
    """Per-pixel properties that hold at any size."""
    g = svdag.decode_hits(raw)
    assert not np.any(g["chunk"] == svdag.FAULT_CHUNK)
    h = g["hit"] == 1
    S = sw.S
    gx, gy, _ = sw.grid
    ci = (g["x"][h] // S) + gx * ((g["y"][h] // S) + gy * (g["z"][h] // S))
    assert np.array_equal(ci, g["chunk"][h].astype(np.int64))          # voxel lies in its chunk
    assert np.array_equal(g["lod"][h], (vt[g["chunk"][h]] & 3).astype(np.int32))  # chunk's picked LOD
    for a in ("x", "y", "z"):                                           # LOD-aligned cell corner
        assert np.all(g[a][h] % (1 << g["lod"][h]) == 0)
    assert np.all((g["material"][h] >= 1) & np.isfinite(g["t"][h]) & (g["t"][h] >= 0))
    assert np.all((vt[g["chunk"][h]] & 12) == 0)                        # never in a culled/empty chunk
    return h.mean()


def test_terrain1024_full_frames(env):
    svdag, torch = env
    note("terrain1024: one 1024^3 chunk, 1920x1080")
    sw, w, ow, cams, frames, vlods = _build(svdag, torch, "terrain1024", 2025, 1, (256, 1024, 4096), 2)
    for v in range(2):
        raw, vt = _trace_like_bench(svdag, torch, w, cams[v])
        _properties(svdag, raw, vt, sw)
        t0 = time.time()
        ref = ow.trace_frame(vlods[v], frames[v], mode=1, threads=NT)
        note(f"terrain1024 view {v}: oracle {ref.size} rays in {time.time() - t0:.1f}s")
        n = compare(svdag, raw, ref, label=f"terrain1024 view {v}")
        assert n > 0.3 * ref.size


def test_map512_full_frames(env):
    svdag, torch = env
    note("map512: 16x16 chunks of 512^3, 4 LODs, 2560x1440")
    sw, w, ow, cams, frames, vlods = _build(svdag, torch, "map512", 2025, 4, (256, 1024, 4096), 3)
    lods_seen = set()
    for v in range(3):
        raw, vt = _trace_like_bench(svdag, torch, w, cams[v])
        assert np.array_equal(vt & 3, vlods[v])
        _properties(svdag, raw, vt, sw)
        t0 = time.time()
        ref = ow.trace_frame(vlods[v], frames[v], mode=1, threads=NT)
        note(f"map512 view {v}: oracle {ref.size} rays in {time.time() - t0:.1f}s")
        compare(svdag, raw, ref, label=f"map512 view {v}")
        lods_seen |= set(ref["lod"][ref["hit"] == 1].tolist())
    assert len(lods_seen) >= 2
