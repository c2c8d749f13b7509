"""Per-LOD residency and the request server: a view whose LOD is not loaded
is marked, never read; every served request equals the same camera traced
alone on a world with every chunk resident, whether batched or plain (serial
or concurrent), with the pool large or too small for the map (forced
evictions)."""
import time

import numpy as np
import pytest

import oracle
from gpu_util import build_blobs, gpu_world, note
from paper_2505_02017_amd import scenes

pytestmark = pytest.mark.gpu
THR = (48, 96, 160)
CL, NL = 6, 4


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_02017_amd import svdag
    svdag.lib()
    return svdag, torch


@pytest.fixture(scope="module")
def world(env):
    svdag, torch = env
    sw = scenes.SceneWorld("custom", 43, chunk_log2=CL, grid=(4, 4, 2))
    dense = {ci: sw.chunk(c) for ci, c in enumerate(sw.chunks())}
    blobs = build_blobs(svdag, CL, NL, dense)
    note("serve world: 4x4x2 x 64^3, 4 LODs")
    ref = gpu_world(svdag, torch, CL, sw.grid, NL, blobs, THR)
    return sw, blobs, ref


def _coords(sw, ci):
    gx, gy, _ = sw.grid
    return (ci % gx, (ci // gx) % gy, ci // (gx * gy))


def _cams(sw, seed, n, sizes=((64, 48), (33, 17), (160, 90), (96, 96), (7, 5), (250, 3), (128, 72))):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        out.append(sw.views(1, seed * 1000 + i, W, H)[0])
    return out


def _alone(svdag, torch, w, cam, flags=0):
    o = torch.empty((cam.width * cam.height, 4), dtype=torch.int32, device="cuda")
    svdag.svd_trace_view(w, svdag.to_camera(cam), o, flags)
    torch.cuda.synchronize()
    return o.cpu().numpy()


def _slot_bytes(svdag, blobs):
    return {(ci, k): svdag.svd_blob_stats_get(b, k)["device_bytes"] for ci, b in blobs.items() for k in range(NL)}


def _need_no_cull(svdag, sw, blobs, cam):
    """(chunk, LOD) slots an unculled view reads: every chunk with solid cells
    at the LOD the camera distance picks."""
    fr = oracle.camera_frame(cam)
    ow = oracle.World(CL, sw.grid, NL)
    lods = ow.lod_pick(fr.O, THR)
    need = set()
    for ci, b in blobs.items():
        k = int(lods[ci])
        if svdag.svd_blob_stats_get(b, k)["n_solid"] > 0:
            need.add((ci, k))
    return need


def _server_world(svdag, torch, sw, budget, views, inflight):
    n = sw.grid[0] * sw.grid[1] * sw.grid[2]
    size = svdag.table_bytes(sw.grid) + inflight * svdag.batch_bytes(n, views) + budget
    pool = torch.empty(size, dtype=torch.uint8, device="cuda")
    return svdag.svd_world_create(svdag.make_desc(CL, sw.grid, NL, THR), pool)


def test_lod_residency_marks_not_loaded(env, world):
    svdag, torch = env
    sw, blobs, ref_w = world
    cams = _cams(sw, 1, 6)
    refs = [_alone(svdag, torch, ref_w, c) for c in cams]
    w = gpu_world(svdag, torch, CL, sw.grid, NL, blobs, THR)
    for ci in blobs:
        svdag.svd_chunk_evict_lods(w, _coords(sw, ci), 0b0011)       # the two finest LODs
    used_evicted = svdag.svd_world_pool_used(w)
    marked = 0
    for v, (c, ref) in enumerate(zip(cams, refs)):
        got = _alone(svdag, torch, w, c)
        g, r = svdag.decode_hits(got), svdag.decode_hits(ref)
        nl = g["chunk"] == svdag.CHUNK_NOT_LOADED
        assert np.all(g["hit"][nl] == 0) and np.all(np.isinf(g["t"][nl]))
        assert np.array_equal(got[~nl], ref[~nl]), f"view {v}: a loaded path changed"
        assert np.all(nl[(r["hit"] == 1) & (r["lod"] < 2)]), f"view {v}: a ray read an unloaded LOD"
        marked += int(nl.sum())
    assert marked > 0
    for ci, b in blobs.items():                                     # load them again
        svdag.svd_chunk_upload_lods(w, _coords(sw, ci), b, 0b0011)
    for v, (c, ref) in enumerate(zip(cams, refs)):
        assert np.array_equal(_alone(svdag, torch, w, c), ref), f"view {v} after reload"
    note(f"pool used with LODs 0-1 evicted: {used_evicted}, reloaded: {svdag.svd_world_pool_used(w)}")
    # a world that only knows the chunks' boxes: every ray that would hit is marked
    w2 = _server_world(svdag, torch, sw, 0, 1, 0)
    for ci, b in blobs.items():
        svdag.svd_chunk_upload_lods(w2, _coords(sw, ci), b, 0)
    assert svdag.svd_world_pool_used(w2) == 0
    for v, (c, ref) in enumerate(zip(cams, refs)):
        g, r = svdag.decode_hits(_alone(svdag, torch, w2, c)), svdag.decode_hits(ref)
        nl = g["chunk"] == svdag.CHUNK_NOT_LOADED
        assert np.all(nl[r["hit"] == 1]) and np.all(g["hit"] == 0), f"view {v}"
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_chunk_upload_lods(w2, (0, 0, 0), blobs[0], 1 << NL)  # no such LOD
    assert e.value.code == svdag.SVD_EINVAL


def _serve(svdag, torch, sw, blobs, cams, mode, views, inflight, budget, flags, seed, sf=0.0):
    w = _server_world(svdag, torch, sw, budget, views, inflight)
    s = svdag.svd_server_create(w, mode=mode, max_views=views, inflight=inflight, max_rays=40000,
                                streaming_factor=sf)
    for ci, b in blobs.items():
        svdag.svd_server_set_chunk(s, _coords(sw, ci), b)
    outs = [torch.full((c.width * c.height, 4), -1, dtype=torch.int32, device="cuda") for c in cams]
    torch.cuda.synchronize()                      # the server's streams do not wait for torch's
    rng = np.random.default_rng(seed)
    done = []
    for i, c in enumerate(cams):                  # arrivals while earlier requests run
        svdag.svd_server_submit(s, c, outs[i], tag=i, flags=flags)
        if rng.random() < 0.3:
            time.sleep(float(rng.uniform(0, 0.002)))
        done += svdag.svd_server_poll(s)
    t0 = time.time()
    while len(done) < len(cams) and time.time() - t0 < 60:
        done += svdag.svd_server_poll(s, wait_us=100000)
    stats = svdag.svd_server_stats_get(s)
    svdag.svd_server_destroy(s)
    torch.cuda.synchronize()
    return w, outs, done, stats


@pytest.mark.parametrize("mode,views,inflight,tight,sf", [(0, 8, 2, False, 0.0), (0, 8, 2, True, 0.0),
                                                          (0, 3, 3, True, 0.0), (1, 1, 3, True, 0.0),
                                                          (2, 1, 3, True, 0.0), (2, 1, 4, False, 0.0),
                                                          (0, 8, 2, False, 2.0), (0, 4, 2, True, 1.5)])
def test_server_results_equal_alone(env, world, mode, views, inflight, tight, sf):
    svdag, torch = env
    sw, blobs, ref_w = world
    flags = svdag.SVD_NO_CULL
    cams = _cams(sw, 7 + views + 10 * mode + int(tight), 24)
    sb = _slot_bytes(svdag, blobs)
    needs = [_need_no_cull(svdag, sw, blobs, c) for c in cams]
    per = [sum((sb[x] + 255) // 256 * 256 for x in n) for n in needs]
    union = set().union(*needs)
    total = sum((sb[x] + 255) // 256 * 256 for x in union)
    budget = max(per) if tight else sum((v + 255) // 256 * 256 for v in sb.values())
    note(f"mode {mode} views {views} inflight {inflight} streaming factor {sf}: budget {budget}, "
         f"largest view {max(per)}, union {total}")
    w, outs, done, st = _serve(svdag, torch, sw, blobs, cams, mode, views, inflight, budget, flags, 3, sf)
    note(f"stats {st}")
    assert len(done) == len(cams) and sorted(d["tag"] for d in done) == list(range(len(cams)))
    assert all(d["status"] == 0 for d in done), [d for d in done if d["status"]]
    for d in done:
        assert d["t_submit"] <= d["t_launch"] <= d["t_done"]
        assert 1 <= d["batch_views"] <= (views if mode == 0 else 1)
    for i, c in enumerate(cams):
        assert np.array_equal(outs[i].cpu().numpy(), _alone(svdag, torch, ref_w, c, flags)), f"request {i}"
    assert st["completed"] == len(cams) and st["failed"] == 0
    assert st["uploads"] + st["prefetches"] >= len(union)
    assert st["upload_bytes"] + st["prefetch_bytes"] >= total
    if sf > 0:
        assert st["prefetches"] > 0
    else:
        assert st["prefetches"] == 0
    if total > budget:
        assert st["evictions"] > 0
    n = sw.grid[0] * sw.grid[1] * sw.grid[2]
    spare = inflight * svdag.batch_bytes(n, views) if mode == 1 else 0  # serial plain mode makes no batch areas
    assert st["pool_used"] <= budget + spare
    if mode == 0:
        assert st["launches"] <= len(cams)


def test_server_single_view_launches_then_burst(env, world):
    """Batched mode where each launch holds one request (the batch's tables
    without its graph), with and without the beam pass and culling, then a
    burst that packs several views per launch over the same batch areas:
    every request equals its view traced alone."""
    svdag, torch = env
    sw, blobs, ref_w = world
    cams = _cams(sw, 31, 12)
    flag_set = [0, svdag.SVD_NO_CULL, svdag.SVD_BEAM, svdag.SVD_NO_CULL | svdag.SVD_BEAM]
    w = _server_world(svdag, torch, sw, 1 << 22, 6, 2)
    s = svdag.svd_server_create(w, mode=0, max_views=6, inflight=2, max_rays=40000)
    for ci, b in blobs.items():
        svdag.svd_server_set_chunk(s, _coords(sw, ci), b)
    outs = [torch.full((c.width * c.height, 4), -1, dtype=torch.int32, device="cuda") for c in cams * 2]
    torch.cuda.synchronize()
    flags = [flag_set[i % 4] for i in range(len(outs))]
    for i, c in enumerate(cams):                     # one at a time: single-view launches
        svdag.svd_server_submit(s, c, outs[i], tag=i, flags=flags[i])
        got = []
        while not got:
            got = svdag.svd_server_poll(s, wait_us=100000)
        assert got[0]["tag"] == i and got[0]["status"] == 0 and got[0]["batch_views"] == 1
    for i, c in enumerate(cams):                     # a burst with one flag: packed launches
        svdag.svd_server_submit(s, c, outs[len(cams) + i], tag=len(cams) + i, flags=svdag.SVD_NO_CULL)
        flags[len(cams) + i] = svdag.SVD_NO_CULL
    done = []
    t0 = time.time()
    while len(done) < len(cams) and time.time() - t0 < 60:
        done += svdag.svd_server_poll(s, wait_us=100000)
    svdag.svd_server_destroy(s)
    torch.cuda.synchronize()
    assert len(done) == len(cams) and all(d["status"] == 0 for d in done)
    assert max(d["batch_views"] for d in done) > 1
    for i, c in enumerate(cams * 2):
        assert np.array_equal(outs[i].cpu().numpy(), _alone(svdag, torch, ref_w, c, flags[i])), f"request {i}"


def test_server_culled_views_and_oversized_requests(env, world):
    svdag, torch = env
    sw, blobs, ref_w = world
    cams = _cams(sw, 99, 6)
    # culling on: requests are served with the cull's smaller slot sets
    w, outs, done, st = _serve(svdag, torch, sw, blobs, cams, 0, 4, 2, 1 << 20, 0, 5)
    assert all(d["status"] == 0 for d in done)
    for i, c in enumerate(cams):
        assert np.array_equal(outs[i].cpu().numpy(), _alone(svdag, torch, ref_w, c)), f"request {i}"
    # a pool with no room for chunk data: every request that reads a chunk fails, the server goes on
    w, outs, done, st = _serve(svdag, torch, sw, blobs, cams[:3], 0, 4, 2, 0, svdag.SVD_NO_CULL, 6)
    assert len(done) == 3 and all(d["status"] == svdag.SVD_ENOMEM for d in done)
    assert st["failed"] == 3


def test_server_errors(env, world):
    svdag, torch = env
    sw, blobs, ref_w = world
    w = _server_world(svdag, torch, sw, 1 << 20, 4, 1)
    with pytest.raises(svdag.SvdError):
        svdag.svd_server_create(w, mode=7)
    with pytest.raises(svdag.SvdError):
        svdag.svd_server_create(w, inflight=0)
    s = svdag.svd_server_create(w, max_views=4, inflight=1)
    cam = _cams(sw, 5, 1)[0]
    out = torch.empty((cam.width * cam.height, 4), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_server_submit(s, cam, out, tag=0)                # chunks without a source
    assert e.value.code == svdag.SVD_EINVAL
    for ci, b in blobs.items():
        svdag.svd_server_set_chunk(s, _coords(sw, ci), b)
    with pytest.raises(svdag.SvdError):
        svdag.svd_server_submit(s, cam, out, tag=0, flags=8)      # unknown flag
    svdag.svd_server_submit(s, cam, out, tag=5)
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_server_set_chunk(s, (0, 0, 0), blobs[0])        # sources are fixed now
    assert e.value.code == svdag.SVD_EINVAL
    got = []
    while not got:
        got = svdag.svd_server_poll(s, wait_us=100000)
    assert got[0]["tag"] == 5 and got[0]["status"] == 0
    svdag.svd_server_destroy(s)
    assert np.array_equal(out.cpu().numpy(), _alone(svdag, torch, ref_w, cam))
