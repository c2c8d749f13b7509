"""GPU parity at full workload sizes, in the launch configurations bench.py
times: per-view frames (svd_view_stage + svd_view_trace on torch's stream)
compared whole with the oracle, plus properties checked on every pixel; the
64-view mixed batch (tuned graph launch) and served requests over a pool
holding a quarter of the map, compared with the oracle on sampled pixels."""
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


def _build(svdag, torch, kind, seed, lod_count, thr, nviews, extra_cams=()):
    """Generate every chunk once; library blobs for all LODs, oracle DAGs only
    for the LODs that the first `nviews` views and `extra_cams` pick."""
    sw = scenes.SceneWorld(kind, seed)
    CL, (gx, gy, gz) = sw.chunk_log2, sw.grid
    nch = gx * gy * gz
    cams = sw.views(nviews, 1)
    ow = oracle.World(CL, sw.grid, lod_count)
    frames = [oracle.camera_frame(c) for c in cams]
    vlods = [ow.lod_pick(f.O, thr) for f in frames]
    xlods = [ow.lod_pick(oracle.camera_frame(c).O, thr) for c in extra_cams]
    need = [sorted({int(v[ci]) for v in vlods + xlods}) for ci in range(nch)]
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
    pool = torch.empty(svdag.table_bytes(sw.grid) + dev + 256 * nch + svdag.batch_bytes(nch, 64),
                       dtype=torch.uint8, device="cuda")
    w = svdag.svd_world_create(desc, pool)
    for c, b in blobs.items():
        svdag.svd_chunk_upload(w, c, b)
    torch.cuda.synchronize()
    return sw, w, ow, cams, frames, vlods, blobs


def _trace_like_bench(svdag, torch, w, cam, flags=0):
    f = svdag.svd_camera_frame(cam)
    out = torch.empty((f.width * f.height, 4), dtype=torch.int32, device="cuda")
    s = torch.cuda.current_stream()
    svdag.svd_view_stage(w, f, flags, s)
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
    sw, w, ow, cams, frames, vlods, _ = _build(svdag, torch, "terrain1024", 2025, 1, (256, 1024, 4096), 2)
    for v in range(2):
        raw, vt = _trace_like_bench(svdag, torch, w, cams[v])
        _properties(svdag, raw, vt, sw)
        t0 = time.time()
        ref = ow.trace_frame(vlods[v], frames[v], mode=1, threads=NT)
        note(f"terrain1024 view {v}: oracle {ref.size} rays in {time.time() - t0:.1f}s")
        n = compare(svdag, raw, ref, label=f"terrain1024 view {v}")
        assert n > 0.3 * ref.size


THR = (256, 1024, 4096)
SIZES = [(320, 180), (640, 360), (1280, 720), (1920, 1080)]


def _batch_cams(sw, n=64, seed=2025):
    """The batched workload: n seeded poses, resolutions uniform over SIZES."""
    rng = np.random.default_rng([seed, 64])
    cams = []
    for i in range(n):
        W, H = SIZES[int(rng.integers(0, len(SIZES)))]
        cams.append(sw.views(1, 1000 + i, W, H)[0])
    return cams


@pytest.fixture(scope="module")
def map512(env):
    svdag, torch = env
    note("map512: 16x16 chunks of 512^3, 4 LODs")
    sw0 = scenes.SceneWorld("map512", 2025)
    extra = _batch_cams(sw0) + [c for _, c in sw0.walk_requests(8, 2000.0, 0.05, seed=7, speed=600.0)]
    return _build(svdag, torch, "map512", 2025, 4, THR, 3, extra)


def _sampled(svdag, ow, raw, cam, n, label, rng):
    """Compare n sampled pixels of a view (its corners included) with the oracle."""
    fr = oracle.camera_frame(cam)
    npx = cam.width * cam.height
    idx = np.unique(np.concatenate([[0, cam.width - 1, npx - cam.width, npx - 1],
                                    rng.integers(0, npx, min(n, npx))])).astype(np.uint32)
    ref = ow.trace_frame(ow.lod_pick(fr.O, THR), fr, idx, mode=1, threads=NT)
    return compare(svdag, raw, ref, idx=idx, label=label)


def test_map512_full_frames(env, map512):
    svdag, torch = env
    sw, w, ow, cams, frames, vlods, _ = map512
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


@pytest.fixture(scope="module")
def map1024_region(env):
    """The 32x32-chunk map of 1024^3 chunks, around the bench's view 0: the
    7x7 chunks around that camera hold the map's content (generated on the
    GPU, byte-equal to the host generator) and every other chunk is empty (an
    empty blob in the library's world, no DAG in the oracle's).  The oracle
    holds LODs 1 to 3 of the real chunks; cameras near view 0 pick only
    those (LOD 0 needs a chunk centre within 256 voxels)."""
    svdag, torch = env
    sw = scenes.SceneWorld("map1024", 2025)
    CL, S, (gx, gy, gz) = sw.chunk_log2, sw.S, sw.grid
    thr = (256, 1024, 4096)
    cam = sw.views(1, 1)[0]
    ccx, ccy = int(cam.pos[0]) // S, int(cam.pos[1]) // S
    region = [(cx, cy, 0) for cy in range(max(0, ccy - 3), min(gy, ccy + 4))
              for cx in range(max(0, ccx - 3), min(gx, ccx + 4))]
    ow = oracle.World(CL, sw.grid, 4)
    dev = torch.empty(S ** 3, dtype=torch.uint8, device="cuda")
    work_dev = None
    blobs = {}

    def build(c, g):
        ci = c[0] + gx * c[1]
        b = svdag.svd_chunk_build(g, CL, 4)
        pyr = oracle.pyramid(g, S, 4)
        return c, ci, b, [(k, oracle.Dag(pyr[k], S >> k)) for k in (1, 2, 3)]

    t0 = time.time()
    with ThreadPoolExecutor(NT) as ex:
        for i in range(0, len(region), NT):
            futs = []
            for c in region[i:i + NT]:
                work_dev = sw.chunk_device(c, dev, work_dev)
                futs.append(ex.submit(build, c, dev.cpu().numpy()))
            for f in futs:
                c, ci, b, dags = f.result()
                blobs[c] = b
                for k, d in dags:
                    ow.set_dag(ci, k, d)
    note(f"map1024: {len(region)} chunks around ({ccx}, {ccy}) built in {time.time() - t0:.1f}s")
    del dev
    empty = svdag.svd_chunk_build(np.zeros(S ** 3, np.uint8), CL, 4)
    nbytes = lambda b: sum((svdag.svd_blob_stats_get(b, k)["device_bytes"] + 255) // 256 * 256 for k in range(4))
    nch = gx * gy * gz
    pool = torch.empty(svdag.table_bytes(sw.grid) + sum(nbytes(b) for b in blobs.values())
                       + nch * (nbytes(empty) + 256), dtype=torch.uint8, device="cuda")
    w = svdag.svd_world_create(svdag.make_desc(CL, sw.grid, 4, thr), pool)
    srcs = {(cx, cy, 0): blobs.get((cx, cy, 0), empty) for cy in range(gy) for cx in range(gx)}
    for c, b in srcs.items():
        svdag.svd_chunk_upload(w, c, b)
    torch.cuda.synchronize()
    yield dict(sw=sw, thr=thr, cam=cam, region=region, ow=ow, w=w, srcs=srcs,
               region_bytes=sum(nbytes(b) for b in blobs.values()))
    del pool


def test_map1024_region_full_frame(env, map1024_region):
    """Every pixel of the bench's view 0 of the map (2560x1440) against the
    oracle: chunk edge 1024 with LODs 1 to 3 picked (7, 6 and 5 internal DAG
    levels)."""
    svdag, torch = env
    m = map1024_region
    sw, cam, ow, w, thr, region = m["sw"], m["cam"], m["ow"], m["w"], m["thr"], m["region"]
    gx = sw.grid[0]
    fr = oracle.camera_frame(cam)
    lods = ow.lod_pick(fr.O, thr)
    raw, vt = _trace_like_bench(svdag, torch, w, cam)
    assert np.array_equal(vt & 3, lods)
    _properties(svdag, raw, vt, sw)
    t0 = time.time()
    ref = ow.trace_frame(lods, fr, mode=1, threads=NT)
    note(f"map1024 region: oracle {ref.size} rays in {time.time() - t0:.1f}s")
    compare(svdag, raw, ref, label="map1024 region view 0")
    seen = set(ref["lod"][ref["hit"] == 1].tolist())
    assert {int(lods[c[0] + gx * c[1]]) for c in region} == {1, 2, 3}
    assert len(seen) >= 2, seen


def _region_requests(sw, ow, thr, cam, n, seed):
    """Requests from cameras around `cam` (within 128 voxels, 50 above the
    terrain, any heading, pitch in [-20, 5] degrees) that pick no LOD 0,
    resolutions uniform over 320x180 .. 1920x1080, Poisson arrivals at 200/s."""
    rng = np.random.default_rng(seed)
    sizes = ((320, 180), (640, 360), (1280, 720), (1920, 1080))
    out, t = [], 0.0
    while len(out) < n:
        x = float(cam.pos[0]) + rng.uniform(-128, 128)
        y = float(cam.pos[1]) + rng.uniform(-128, 128)
        z = min(sw.height(int(x), int(y)) + 50.0, sw.extent[2] - 0.5)
        yaw, pitch = rng.uniform(0, 2 * np.pi), np.radians(rng.uniform(-20.0, 5.0))
        d = np.array([np.cos(pitch) * np.cos(yaw), np.cos(pitch) * np.sin(yaw), np.sin(pitch)])
        W, H = sizes[int(rng.integers(len(sizes)))]
        c = scenes.Camera((x, y, z), tuple(np.array([x, y, z]) + 100.0 * d), (0.0, 0.0, 1.0), 60.0, W, H).as_f32()
        if np.any(ow.lod_pick(oracle.camera_frame(c).O, thr) == 0):
            continue
        t += rng.exponential(1 / 200.0)
        out.append((t, c))
    return out


@pytest.mark.parametrize("mode", [0, 2])
def test_map1024_region_served_sampled(env, map1024_region, mode):
    """About 50 requests served on the map of 1024^3 chunks through a pool
    holding a quarter of the region's chunk bytes (streaming uploads),
    batched or as concurrent per-request launches: every request equals its
    view traced alone on the full world, and sampled pixels equal the
    oracle's."""
    svdag, torch = env
    m = map1024_region
    sw, ow, thr, w_full = m["sw"], m["ow"], m["thr"], m["w"]
    sched = _region_requests(sw, ow, thr, m["cam"], 48, seed=11 + mode)
    nch = sw.grid[0] * sw.grid[1] * sw.grid[2]
    budget = m["region_bytes"] // 4 // 256 * 256
    pool = torch.empty(svdag.table_bytes(sw.grid) + 2 * svdag.batch_bytes(nch, 8) + budget,
                       dtype=torch.uint8, device="cuda")
    w = svdag.svd_world_create(svdag.make_desc(sw.chunk_log2, sw.grid, 4, thr), pool)
    s = svdag.svd_server_create(w, mode=mode, max_views=8 if mode == 0 else 1, inflight=2, max_rays=1 << 23)
    for c, b in m["srcs"].items():
        svdag.svd_server_set_chunk(s, c, b)
    outs = [torch.full((c.width * c.height, 4), -1, dtype=torch.int32, device="cuda") for _, c in sched]
    torch.cuda.synchronize()
    note(f"map1024 region: serving {len(sched)} requests (mode {mode}), pool {budget >> 20} of "
         f"{m['region_bytes'] >> 20} MiB")
    t0 = time.perf_counter()
    for i, (t, c) in enumerate(sched):
        while time.perf_counter() - t0 < t:
            pass
        svdag.svd_server_submit(s, c, outs[i], tag=i)
    done = []
    while len(done) < len(sched) and time.perf_counter() - t0 < 60:
        done += svdag.svd_server_poll(s, 256, wait_us=100000)
    st = svdag.svd_server_stats_get(s)
    svdag.svd_server_destroy(s)
    note(f"served: {st}")
    assert len(done) == len(sched) and all(d["status"] == 0 for d in done)
    assert st["uploads"] > 0 and st["pool_used"] <= budget
    rng = np.random.default_rng(5)
    hits = 0
    for i, (_, c) in enumerate(sched):
        got = outs[i].cpu().numpy()
        alone, _ = _trace_like_bench(svdag, torch, w_full, c)
        assert np.array_equal(got, alone), f"request {i}"
        hits += _sampled(svdag, ow, got, c, 1000, f"request {i} ({c.width}x{c.height})", rng)
    assert hits > 0
    del pool


def test_map512_beam_pass_changes_no_record(env, map512):
    """The exact beam pass on full 1440p map views: every record equals the
    plain trace's (which the test above checks against the oracle)."""
    svdag, torch = env
    sw, w, ow, cams, frames, vlods, _ = map512
    for v in range(3):
        plain, _ = _trace_like_bench(svdag, torch, w, cams[v])
        beam, _ = _trace_like_bench(svdag, torch, w, cams[v], flags=svdag.SVD_BEAM)
        diff = int(np.count_nonzero((plain != beam).any(axis=1)))
        note(f"map512 view {v}: beam pass, {diff} records differ")
        assert diff == 0


def test_map512_batch_of_64_sampled(env, map512):
    """The 64-view mixed batch in the bench's launch configuration (tuned
    tiling and occupancy, one graph launch) against the oracle."""
    svdag, torch = env
    sw, w, ow, cams, frames, vlods, _ = map512
    bc = _batch_cams(sw)
    nrec = svdag.batch_records(bc)
    b = svdag.svd_batch_create(w, len(bc))
    out = torch.empty((nrec, 4), dtype=torch.int32, device="cuda")
    tw, claim, occ, ms = svdag.svd_batch_tune(b, bc, out, reps=1)
    note(f"batch of {len(bc)} views ({nrec} rays): tile {tw}x{64 // tw}, claim {claim}, {occ}/CU, {ms:.2f} ms")
    out.fill_(-1)
    svdag.svd_batch_trace(b, bc, out)
    torch.cuda.synchronize()
    raw = out.cpu().numpy()
    svdag.svd_batch_destroy(b)
    rng = np.random.default_rng(64)
    off, hits = 0, 0
    for v, c in enumerate(bc):
        n = c.width * c.height
        hits += _sampled(svdag, ow, raw[off:off + n], c, 1500, f"batch view {v} ({c.width}x{c.height})", rng)
        off += n
    assert hits > 0


def test_map512_served_sampled(env, map512):
    """Requests served through a pool holding a quarter of the map's bytes
    (uploads, evictions, prefetch, batched launches) against the oracle."""
    svdag, torch = env
    sw, w_full, ow, cams, frames, vlods, blobs = map512
    sched = sw.walk_requests(8, 2000.0, 0.05, seed=7, speed=600.0)
    nch = sw.grid[0] * sw.grid[1] * sw.grid[2]
    all_bytes = sum((svdag.svd_blob_stats_get(b, k)["device_bytes"] + 255) // 256 * 256
                    for b in blobs.values() for k in range(4))
    budget = all_bytes // 4 // 256 * 256
    pool = torch.empty(svdag.table_bytes(sw.grid) + 2 * svdag.batch_bytes(nch, 16) + budget,
                       dtype=torch.uint8, device="cuda")
    w = svdag.svd_world_create(svdag.make_desc(sw.chunk_log2, sw.grid, 4, THR), pool)
    s = svdag.svd_server_create(w, max_views=16, inflight=2, max_rays=1 << 23, streaming_factor=1.5)
    for c, b in blobs.items():
        svdag.svd_server_set_chunk(s, c, b)
    outs = [torch.empty((c.width * c.height, 4), dtype=torch.int32, device="cuda") for _, c in sched]
    torch.cuda.synchronize()
    note(f"serving {len(sched)} requests, pool {budget >> 20} MiB of {all_bytes >> 20} MiB")
    t0 = time.perf_counter()
    for i, (t, c) in enumerate(sched):
        while time.perf_counter() - t0 < t:
            pass
        svdag.svd_server_submit(s, c, outs[i], tag=i)
    done = []
    while len(done) < len(sched) and time.perf_counter() - t0 < 60:
        done += svdag.svd_server_poll(s, 256, wait_us=100000)
    st = svdag.svd_server_stats_get(s)
    svdag.svd_server_destroy(s)
    note(f"served: {st}")
    assert len(done) == len(sched) and all(d["status"] == 0 for d in done)
    rng = np.random.default_rng(7)
    for i, (_, c) in enumerate(sched):
        _sampled(svdag, ow, outs[i].cpu().numpy(), c, 1500, f"request {i} ({c.width}x{c.height})", rng)
