"""Batched views (one graph launch, persistent trace over a shared tile
queue): every view's records equal those of its own per-view launch and
the oracle's, for every tiling, across repeated graph replays."""
import os
import re

import numpy as np
import pytest

import oracle
from gpu_util import build_blobs, compare, gpu_world, note, oracle_world
from paper_2505_02017_amd import scenes

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)
THR = (48, 96, 160)


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
    sw = scenes.SceneWorld("custom", 41, chunk_log2=6, grid=(4, 4, 2))
    dense = {ci: sw.chunk(c) for ci, c in enumerate(sw.chunks())}
    note("batch world: 4x4x2 x 64^3, 4 LODs")
    w = gpu_world(svdag, torch, 6, sw.grid, 4, build_blobs(svdag, 6, 4, dense), THR, extra_bytes=1 << 22)
    ow = oracle_world(6, sw.grid, 4, dense)
    return sw, w, ow


def _cams(sw, seed, n):
    rng = np.random.default_rng(seed)
    sizes = [(1, 1), (7, 5), (64, 48), (33, 17), (160, 90), (96, 96), (250, 3), (2, 130)]
    cams = []
    for i in range(n):
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        cams.append(sw.views(1, seed * 100 + i, W, H)[0])
    return cams


def _per_view(svdag, torch, w, cams):
    outs = []
    for c in cams:
        o = torch.empty((c.width * c.height, 4), dtype=torch.int32, device="cuda")
        svdag.svd_trace_view(w, svdag.to_camera(c), o)
        outs.append(o)
    torch.cuda.synchronize()
    return np.concatenate([o.cpu().numpy() for o in outs])


def test_batch_equals_per_view_all_tilings(env, world):
    svdag, torch = env
    sw, w, ow = world
    cams = _cams(sw, 1, 12)
    ref = _per_view(svdag, torch, w, cams)
    b = svdag.svd_batch_create(w, 16)
    out = torch.empty((svdag.batch_records(cams), 4), dtype=torch.int32, device="cuda")
    for tw in (8, 16, 32, 64):
        for claim in (1, 3):
            note(f"tiling {tw}x{64 // tw} claim {claim}")
            svdag.svd_batch_set_tiling(b, tw, claim)
            out.fill_(-1)
            svdag.svd_batch_trace(b, cams, out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), (tw, claim)
    out_nb = torch.full_like(out, -1)
    svdag.svd_batch_trace(b, cams, out_nb, svdag.SVD_BEAM)
    torch.cuda.synchronize()
    assert np.array_equal(out_nb.cpu().numpy(), ref), "batch with the beam pass"
    # and the batch agrees with the oracle view by view
    raw, off = out.cpu().numpy(), 0
    for v, c in enumerate(cams):
        n = c.width * c.height
        fr = oracle.camera_frame(c)
        compare(svdag, raw[off:off + n], ow.trace_frame(ow.lod_pick(fr.O, THR), fr, threads=NT),
                label=f"batch view {v}")
        off += n
    svdag.svd_batch_destroy(b)


def test_graph_replays_with_changing_batches(env, world):
    svdag, torch = env
    sw, w, ow = world
    b = svdag.svd_batch_create(w, 24)
    big = torch.empty((24 * 250 * 130, 4), dtype=torch.int32, device="cuda")
    for rep in range(6):
        cams = _cams(sw, 10 + rep, 5 + 3 * rep)
        n = svdag.batch_records(cams)
        big[:n].fill_(-1)
        svdag.svd_batch_trace(b, cams, big)
        # eager work of the program between replays
        scratch = torch.arange(1 << 16, device="cuda").float().sum()
        torch.cuda.synchronize()
        ref = _per_view(svdag, torch, w, cams)
        assert np.array_equal(big[:n].cpu().numpy(), ref), f"replay {rep}"
        assert float(scratch) > 0
    svdag.svd_batch_destroy(b)


def test_tuner_and_errors(env, world):
    svdag, torch = env
    sw, w, ow = world
    cams = _cams(sw, 3, 10)
    b = svdag.svd_batch_create(w, 10)
    out = torch.empty((svdag.batch_records(cams), 4), dtype=torch.int32, device="cuda")
    tw, claim, occ, ms = svdag.svd_batch_tune(b, cams, out, reps=2)
    assert tw in (8, 16, 32, 64) and claim in (1, 2, 4) and occ >= 1 and ms > 0
    svdag.svd_batch_trace(b, cams, out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), _per_view(svdag, torch, w, cams))
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_batch_trace(b, cams + cams[:1], out)          # more views than max_views
    assert e.value.code == svdag.SVD_EINVAL
    small = torch.empty((svdag.batch_records(cams) - 1, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_batch_trace(b, cams, small)                   # output too small
    assert e.value.code == svdag.SVD_EINVAL
    with pytest.raises(svdag.SvdError):
        svdag.svd_batch_set_tiling(b, 12, 1)
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_batch_set_occupancy(b, 1000)                   # more blocks than fit a CU
    assert e.value.code == svdag.SVD_EINVAL
    svdag.svd_batch_destroy(b)


def test_occupancy_does_not_change_results(env, world):
    """The persistent grid size (blocks per CU) of both the batch and the
    per-view trace changes the schedule only, never a record."""
    svdag, torch = env
    sw, w, ow = world
    cams = _cams(sw, 5, 9)
    ref = _per_view(svdag, torch, w, cams)
    b = svdag.svd_batch_create(w, 9)
    _, _, mx = svdag.svd_batch_get_tiling(b)
    out = torch.empty((svdag.batch_records(cams), 4), dtype=torch.int32, device="cuda")
    for occ in sorted({1, 2, mx, 0}):
        note(f"batch occupancy {occ}")
        svdag.svd_batch_set_occupancy(b, occ)
        assert svdag.svd_batch_get_tiling(b)[2] == (occ or mx)
        for _ in range(2):                                      # two launches of the re-captured graph
            out.fill_(-1)
            svdag.svd_batch_trace(b, cams, out)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), occ
    svdag.svd_batch_destroy(b)
    cur, wmx = svdag.svd_world_get_occupancy(w)
    assert cur == min(wmx, 6) and wmx >= 1
    try:
        for occ in (1, 2):
            note(f"per-view occupancy {occ}")
            svdag.svd_world_set_occupancy(w, occ)
            assert svdag.svd_world_get_occupancy(w) == (occ, wmx)
            assert np.array_equal(_per_view(svdag, torch, w, cams), ref), occ
        with pytest.raises(svdag.SvdError) as e:
            svdag.svd_world_set_occupancy(w, wmx + 1)
        assert e.value.code == svdag.SVD_EINVAL
    finally:
        svdag.svd_world_set_occupancy(w, 0)


def _per_view_flags(svdag, torch, w, cams, flags):
    outs = []
    for c in cams:
        o = torch.full((c.width * c.height, 4), -1, dtype=torch.int32, device="cuda")
        svdag.svd_trace_view(w, svdag.to_camera(c), o, flags)
        outs.append(o)
    torch.cuda.synchronize()
    return np.concatenate([o.cpu().numpy() for o in outs])


def test_per_view_tilings_and_tuning_cache(env, world, tmp_path):
    """The per-view tile (8x8, 16x4, 32x2, 64x1) changes the schedule only,
    with and without the beam pass; the per-view and batch tuners apply
    their choice, store it in the cache file and take it from there on the
    next call without timing."""
    svdag, torch = env
    sw, w, ow = world
    cams = _cams(sw, 7, 8)
    ref = _per_view(svdag, torch, w, cams)                     # default tile 16x4
    frames = [svdag.svd_camera_frame(svdag.to_camera(c)) for c in cams]
    assert svdag.svd_world_get_tiling(w) == 16
    path = str(tmp_path / "tune.txt")
    try:
        for tw in (8, 16, 32, 64):
            svdag.svd_world_set_tiling(w, tw)
            assert svdag.svd_world_get_tiling(w) == tw
            for flags in (0, svdag.SVD_BEAM):
                note(f"per-view tile {tw}x{64 // tw} flags {flags}")
                assert np.array_equal(_per_view_flags(svdag, torch, w, cams, flags), ref), (tw, flags)
        with pytest.raises(svdag.SvdError) as e:
            svdag.svd_world_set_tiling(w, 12)
        assert e.value.code == svdag.SVD_EINVAL
        svdag.svd_world_set_tiling(w, 0)
        assert svdag.svd_world_get_tiling(w) == 16

        big = torch.empty((max(c.width * c.height for c in cams), 4), dtype=torch.int32, device="cuda")
        with pytest.raises(svdag.SvdError) as e:                 # output smaller than the largest frame
            svdag.svd_world_tune(w, frames, big[:-1], reps=1, cache_path=path)
        assert e.value.code == svdag.SVD_EINVAL
        assert not os.path.exists(path)
        note("per-view tuner, cache miss")
        r1 = svdag.svd_world_tune(w, frames, big, svdag.SVD_BEAM, reps=2, cache_path=path)
        key = r1.key.decode()
        assert not r1.from_cache and r1.configs_timed >= 4 and r1.ms > 0
        assert r1.tile_w in (8, 16, 32, 64) and r1.claim == 1
        assert re.match(r"dev=gfx\S*/\d+cu/\d+mhz kernel=%s kind=view cl=6 grid=4x4x2 lods=4 flags=2 views=8 res="
                        % svdag.svd_kernel_hash(), key), key
        assert svdag.svd_world_get_tiling(w) == r1.tile_w
        assert svdag.svd_world_get_occupancy(w)[0] == r1.blocks_per_cu
        assert np.array_equal(_per_view_flags(svdag, torch, w, cams, svdag.SVD_BEAM), ref)
        svdag.svd_world_set_tiling(w, 0)
        svdag.svd_world_set_occupancy(w, 0)
        note("per-view tuner, cache hit")
        r2 = svdag.svd_world_tune(w, frames, big, svdag.SVD_BEAM, reps=2, cache_path=path)
        assert r2.from_cache and r2.configs_timed == 0 and r2.key.decode() == key
        assert (r2.tile_w, r2.blocks_per_cu) == (r1.tile_w, r1.blocks_per_cu)
        assert svdag.svd_world_get_tiling(w) == r1.tile_w
        assert svdag.svd_world_get_occupancy(w)[0] == r1.blocks_per_cu
        # other flags are another workload
        r3 = svdag.svd_world_tune(w, frames, big, 0, reps=1, cache_path=path)
        assert not r3.from_cache and "flags=0 " in r3.key.decode()

        note("batch tuner through the cache")
        b = svdag.svd_batch_create(w, len(cams))
        out = torch.empty((svdag.batch_records(cams), 4), dtype=torch.int32, device="cuda")
        rb1 = svdag.svd_batch_tune_cached(b, cams, out, reps=1, cache_path=path)
        assert not rb1.from_cache and "kind=batch" in rb1.key.decode()
        svdag.svd_batch_set_tiling(b, 16, 1)
        svdag.svd_batch_set_occupancy(b, 0)
        rb2 = svdag.svd_batch_tune_cached(b, cams, out, reps=1, cache_path=path)
        assert rb2.from_cache and (rb2.tile_w, rb2.claim, rb2.blocks_per_cu) == \
            (rb1.tile_w, rb1.claim, rb1.blocks_per_cu)
        assert svdag.svd_batch_get_tiling(b) == (rb1.tile_w, rb1.claim, rb1.blocks_per_cu)
        out.fill_(-1)
        svdag.svd_batch_trace(b, cams, out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref)
        svdag.svd_batch_destroy(b)
        assert len(open(path).read().splitlines()) == 4          # header + view x2 + batch
    finally:
        svdag.svd_world_set_tiling(w, 0)
        svdag.svd_world_set_occupancy(w, 0)


def test_trace_pass_timing(env, world):
    """Armed trace passes take their kernel time from the dispatches, with and
    without the beam pass, and records do not change; passes beyond the armed
    count run untimed, arming again drops earlier records, and a pass split
    into stage, beam and trace calls is timed once."""
    svdag, torch = env
    sw, w, ow = world
    cams = _cams(sw, 11, 5)
    ref = _per_view(svdag, torch, w, cams)
    try:
        for flags in (0, svdag.SVD_BEAM):
            note(f"timed passes, flags {flags}")
            svdag.svd_world_time_traces(w, 3)
            assert svdag.svd_world_trace_times(w, 3) == []
            assert np.array_equal(_per_view_flags(svdag, torch, w, cams, flags), ref), flags  # 5 passes
            ms = svdag.svd_world_trace_times(w, 8)
            assert len(ms) == 3 and all(0.0 < m < 1000.0 for m in ms), ms
            assert svdag.svd_world_trace_times(w, 2) == ms[:2]
        c = cams[2]
        n = c.width * c.height
        start = sum(x.width * x.height for x in cams[:2])
        f = svdag.svd_camera_frame(svdag.to_camera(c))
        o = torch.full((n, 4), -1, dtype=torch.int32, device="cuda")
        svdag.svd_world_time_traces(w, 1)
        svdag.svd_view_stage(w, f, svdag.SVD_BEAM)
        svdag.svd_view_beam(w, f, o)
        svdag.svd_view_trace(w, f, o)
        ms = svdag.svd_world_trace_times(w, 4)
        assert len(ms) == 1 and ms[0] > 0.0, ms
        assert np.array_equal(o.cpu().numpy(), ref[start:start + n])
        with pytest.raises(svdag.SvdError) as e:
            svdag.svd_world_time_traces(w, svdag.SVD_MAX_TIMED_PASSES + 1)
        assert e.value.code == svdag.SVD_EINVAL
    finally:
        svdag.svd_world_time_traces(w, 0)
    assert svdag.svd_world_trace_times(w, 4) == []
