"""The library's kernel logic (chunk stage, beam pass, per-pixel trace of
kernels.hip, compiled for the host by tests/host_kernels.cpp) against the
oracle, on the CPU: bit-exact records on adversarial frames over tiny
multi-chunk, multi-LOD worlds and on terrain views; the beam pass and
culling change no record; a LOD that is only described yields not-loaded
records, never a read.  The GPU tests check the same code on the device."""
import os

import numpy as np
import pytest

import oracle
from gpu_util import compare
from paper_2505_02017_amd import scenes
import test_gpu_parity as gp

NT = min(8, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def env():
    from paper_2505_02017_amd import svdag
    import host_kernels
    if not os.path.exists(host_kernels.LIB):
        pytest.skip("host kernel build missing: run __graft_entry__.build()")
    svdag.lib()
    host_kernels.lib()
    return svdag, host_kernels


@pytest.mark.parametrize("cfg", [
    (3, (1, 1, 1), 1, 0.3, (256, 1024, 4096)),
    (3, (2, 2, 1), 1, 0.15, (256, 1024, 4096)),
    (4, (2, 1, 1), 2, 0.25, (12, 0, 0)),
    (5, (2, 2, 2), 3, 0.1, (16, 40, 0)),
    (6, (2, 1, 1), 4, 0.05, (20, 50, 90)),
])
def test_adversarial_frames(env, cfg):
    svdag, hk = env
    chunk_log2, grid, lod_count, fill, thr = cfg
    rng = np.random.default_rng(sum(grid) * 1000 + chunk_log2 * 10 + lod_count + 5)
    S = 1 << chunk_log2
    nch = grid[0] * grid[1] * grid[2]
    dense = {ci: scenes.random_grid(rng, S, fill) for ci in range(nch)}
    blobs = {ci: svdag.svd_chunk_build(g, chunk_log2, lod_count) for ci, g in dense.items()}
    hw = hk.HostWorld(svdag, chunk_log2, grid, lod_count, thr, blobs)
    ow = oracle.World(chunk_log2, grid, lod_count)
    for ci, g in dense.items():
        ow.add_chunk(ci, g)
    ext = [g * S for g in grid]
    hits = 0
    for i, (O, A, BX, BY, W, H) in enumerate(gp._frames(rng, ext, 150, 16, 8)):
        fr = svdag.make_frame(O, A, BX, BY, W, H)
        raw, view = hw.trace(fr, threads=NT)
        lods = ow.lod_pick(np.array(O, np.int64), thr)
        assert np.array_equal(view & 3, lods), f"frame {i}: LOD pick"
        ref = ow.trace_frame(lods, gp._oracle_frame(fr), mode=1, threads=NT)
        hits += compare(svdag, raw, ref, label=f"{cfg} frame {i}")
        raw_b, _ = hw.trace(fr, svdag.SVD_BEAM, threads=NT)
        assert np.array_equal(raw, raw_b), f"{cfg} frame {i}: the beam pass changed a record"
    assert hits > 0


def test_terrain_views_beam_cull_and_not_loaded(env):
    svdag, hk = env
    sw = scenes.SceneWorld("custom", 23, chunk_log2=6, grid=(4, 4, 2))
    dense = {ci: sw.chunk(c) for ci, c in enumerate(sw.chunks())}
    thr = (48, 96, 160)
    blobs = {ci: svdag.svd_chunk_build(g, 6, 4) for ci, g in dense.items()}
    hw = hk.HostWorld(svdag, 6, sw.grid, 4, thr, blobs)
    ow = oracle.World(6, sw.grid, 4)
    for ci, g in dense.items():
        ow.add_chunk(ci, g)
    half = set(range(0, len(blobs), 2))
    hw_half = hk.HostWorld(svdag, 6, sw.grid, 4, thr, blobs, describe_only=half)
    marked = 0
    for v, cam in enumerate(sw.views(4, 5, 96, 64)):
        f = svdag.svd_camera_frame(cam)
        raw, _ = hw.trace(f, threads=NT)
        for flags in (svdag.SVD_NO_CULL, svdag.SVD_BEAM, svdag.SVD_BEAM | svdag.SVD_NO_CULL):
            assert np.array_equal(raw, hw.trace(f, flags, threads=NT)[0]), f"view {v} flags {flags}"
        fr = oracle.camera_frame(cam)
        compare(svdag, raw, ow.trace_frame(ow.lod_pick(fr.O, thr), fr, mode=1, threads=NT), label=f"terrain {v}")
        # half the chunks only described: their rays are marked, every other record unchanged
        for flags in (0, svdag.SVD_BEAM):
            got, _ = hw_half.trace(f, flags, threads=NT)
            g = svdag.decode_hits(got)
            nl = g["chunk"] == svdag.CHUNK_NOT_LOADED
            assert np.array_equal(got[~nl], raw[~nl]), f"view {v}: a loaded path changed"
            r = svdag.decode_hits(raw)
            hit_in_half = (r["hit"] == 1) & np.isin(r["chunk"], list(half))
            assert np.all(nl[hit_in_half]), f"view {v}: a ray read a chunk that is not loaded"
            marked += int(nl.sum())
    assert marked > 0


def test_gpu_scene_generator_code_equals_host_generator(env):
    """The GPU scene generator's per-element code (scenegen_gpu.hip: column
    heights, cave lattice tables, voxels), run on the host, against the host
    generator byte for byte: worlds with several z layers, chunk edges below
    the cave wavelength, and map512 chunks where boxes meet."""
    _, hk = env
    cases = [(scenes.SceneWorld("custom", 7, chunk_log2=5, grid=(2, 2, 2)), None),
             (scenes.SceneWorld("custom", 3, chunk_log2=3, grid=(4, 4, 2)), [(0, 0, 0), (3, 2, 1), (1, 3, 0)]),
             (scenes.SceneWorld("custom", 11, chunk_log2=6, grid=(3, 2, 1)), None),
             (scenes.SceneWorld("map512", 2025), [(3, 5, 0), (15, 15, 0)])]
    nboxes = 0
    for sw, chunks in cases:
        for c in (chunks or list(sw.chunks())):
            nboxes += len(sw.chunk_boxes(c))
            a = sw.chunk(c, threads=NT)
            b = hk.scene_chunk(sw, c, threads=NT)
            bad = np.flatnonzero(a != b)
            assert bad.size == 0, f"{sw.kind} {c}: {bad.size} bytes differ"
    assert nboxes > 10


@pytest.mark.parametrize("cfg", [
    (4, (3, 3, 2), 2, (10, 0, 0)),
    (5, (2, 3, 1), 3, (16, 40, 0)),
])
def test_small_tight_boxes_adversarial(env, cfg):
    """Chunks holding one small solid block each (or nothing), so that their
    tight boxes are much smaller than the chunks and the trace often crosses
    a chunk because the ray is already past its box: the adversarial ray
    families (integer and half-voxel origins, rays lying in grid planes,
    through edges and corners, all direction signs) against the oracle."""
    svdag, hk = env
    chunk_log2, grid, lod_count, thr = cfg
    rng = np.random.default_rng(chunk_log2 * 100 + lod_count)
    S = 1 << chunk_log2
    nch = grid[0] * grid[1] * grid[2]
    dense = {}
    for ci in range(nch):
        g = np.zeros((S, S, S), np.uint8)  # indexed [z, y, x]
        if rng.random() < 0.85:
            lo = rng.integers(0, S - 1, 3)
            hi = np.minimum(lo + rng.integers(1, S // 2 + 1, 3), S)
            g[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = rng.integers(1, 16, (hi[2] - lo[2], hi[1] - lo[1],
                                                                              hi[0] - lo[0]), dtype=np.uint8)
        dense[ci] = g.reshape(-1)
    blobs = {ci: svdag.svd_chunk_build(g, chunk_log2, lod_count) for ci, g in dense.items()}
    hw = hk.HostWorld(svdag, chunk_log2, grid, lod_count, thr, blobs)
    ow = oracle.World(chunk_log2, grid, lod_count)
    for ci, g in dense.items():
        ow.add_chunk(ci, g)
    ext = [g * S for g in grid]
    hits = 0
    for i, (O, A, BX, BY, W, H) in enumerate(gp._frames(rng, ext, 200, 16, 8)):
        fr = svdag.make_frame(O, A, BX, BY, W, H)
        raw, view = hw.trace(fr, threads=NT)
        lods = ow.lod_pick(np.array(O, np.int64), thr)
        ref = ow.trace_frame(lods, gp._oracle_frame(fr), mode=1, threads=NT)
        hits += compare(svdag, raw, ref, label=f"{cfg} frame {i}")
    assert hits > 0


@pytest.mark.parametrize("seed", [1, 2])
def test_material_runs_of_every_length(env, seed):
    """Material lookup through the run directory: solid chunks whose
    materials come in runs from one voxel to most of the chunk along the DFS
    order (so a directory bucket holds zero, one or many run starts), at
    every LOD; every hit's material equals the oracle's."""
    svdag, hk = env
    chunk_log2, grid, lod_count, thr = 5, (2, 1, 1), 3, (20, 40, 0)
    rng = np.random.default_rng(seed)
    S = 1 << chunk_log2
    dense = {}
    for ci in range(2):
        g = np.zeros((S, S, S), np.uint8)
        # boxes of one material of sizes 1..S/2, then single-voxel noise, then holes
        for _ in range(60):
            s = int(rng.integers(1, S // 2 + 1))
            z, y, x = (int(v) for v in rng.integers(0, S - s + 1, 3))
            g[z:z + s, y:y + s, x:x + s] = int(rng.integers(1, 256))
        noise = rng.random((S, S, S)) < 0.02
        g[noise] = rng.integers(1, 256, int(noise.sum()))
        g[rng.random((S, S, S)) < 0.05] = 0
        dense[ci] = g
    blobs = {ci: svdag.svd_chunk_build(g, chunk_log2, lod_count) for ci, g in dense.items()}
    runs = [svdag.svd_blob_stats_get(blobs[0], k)["n_rle"] for k in range(lod_count)]
    solid = [svdag.svd_blob_stats_get(blobs[0], k)["n_solid"] for k in range(lod_count)]
    assert all(r < s for r, s in zip(runs, solid)), "runs longer than a voxel exist"
    hw = hk.HostWorld(svdag, chunk_log2, grid, lod_count, thr, blobs)
    ow = oracle.World(chunk_log2, grid, lod_count)
    for ci, g in dense.items():
        ow.add_chunk(ci, g)
    ext = [g * S for g in grid]
    hits = 0
    for i, (O, A, BX, BY, W, H) in enumerate(gp._frames(rng, ext, 40, 24, 16)):
        fr = svdag.make_frame(O, A, BX, BY, W, H)
        raw, _ = hw.trace(fr, threads=NT)
        ref = ow.trace_frame(ow.lod_pick(np.array(O, np.int64), thr), gp._oracle_frame(fr), mode=1, threads=NT)
        hits += compare(svdag, raw, ref, label=f"material runs frame {i}")
    assert hits > 1000


def test_walk_event_counts_are_consistent(env):
    """The host build's walk-event counts (the per-step evidence behind the
    trace's instruction budget) add up: every exit is a sibling step, a pop
    to an ancestor or a move to the next chunk; every hit record is one hit
    event; every loop iteration ends in a hit, an exit, or a descent into a
    non-empty cell."""
    svdag, hk = env
    sw = scenes.SceneWorld("custom", 23, chunk_log2=6, grid=(4, 4, 2))
    dense = {ci: sw.chunk(c) for ci, c in enumerate(sw.chunks())}
    thr = (48, 96, 160)
    blobs = {ci: svdag.svd_chunk_build(g, 6, 4) for ci, g in dense.items()}
    hw = hk.HostWorld(svdag, 6, sw.grid, 4, thr, blobs)
    for i, cam in enumerate(sw.views(3, 9, 96, 64)):
        fr = svdag.svd_camera_frame(svdag.to_camera(cam))
        raw, c = hk.trace_counts(hw, fr, threads=NT)
        raw2, _ = hw.trace(fr, threads=NT)
        assert np.array_equal(raw, raw2)
        hits = int((svdag.decode_hits(raw)["hit"] == 1).sum())
        assert c["hit"] == hits > 0
        assert c["exit"] == c["sibling"] + c["pop"] + c["chunk_next"]
        assert c["hit"] + c["exit"] <= c["iter"] <= c["hit"] + c["exit"] + c["descend"]
        assert c["chunk_enter"] <= c["chunk_visit"]
        assert c["tiles"] == ((96 + 15) // 16) * ((64 + 3) // 4)
        assert c["iter"] / (96 * 64) <= c["tile_max_iter"] / c["tiles"]


def test_zero_direction_rays(env):
    """Pixels whose direction is exactly zero never move: a hit at the
    origin's cell when it is solid at the picked LOD, else a miss; on the
    oracle the same."""
    svdag, hk = env
    chunk_log2, grid, lod_count, thr = 4, (2, 2, 1), 2, (20, 0, 0)
    rng = np.random.default_rng(77)
    S = 1 << chunk_log2
    dense = {ci: scenes.random_grid(rng, S, 0.5) for ci in range(4)}
    blobs = {ci: svdag.svd_chunk_build(g, chunk_log2, lod_count) for ci, g in dense.items()}
    hw = hk.HostWorld(svdag, chunk_log2, grid, lod_count, thr, blobs)
    ow = oracle.World(chunk_log2, grid, lod_count)
    for ci, g in dense.items():
        ow.add_chunk(ci, g)
    F = 1 << 16
    hits = misses = 0
    for i in range(90):
        # pixel (0, 0) has D = A = 0; the rest of the row points along +-x.
        # A third of the origins lie in the world's low corner, where cell
        # and chunk coordinates coincide (so a walk that went on from such a
        # cell would not leave the world by accident).
        hi = [2, 2, 2] if i % 3 == 0 else [2 * S, 2 * S, S]
        O = [int(rng.integers(-F if i % 3 else 0, hi[a] * F + (F if i % 3 else 0))) for a in range(3)]
        O = [min(max(o, -F), (2 * S + 1) * F) for o in O]
        sx = 1 if i % 2 else -1
        fr = svdag.make_frame(O, [0, 0, 0], [sx * 977, 31, -17], [0, 0, 0], 5, 1)
        raw, _ = hw.trace(fr, threads=1)
        ref = ow.trace_frame(ow.lod_pick(np.array(O, np.int64), thr), gp._oracle_frame(fr), mode=1, threads=1)
        compare(svdag, raw, ref, label=f"zero-direction frame {i}")
        h = svdag.decode_hits(raw[:1])["hit"][0]
        hits += int(h == 1)
        misses += int(h == 0)
    assert hits > 5 and misses > 5


@pytest.mark.parametrize("tiles_x,tiles_y", [(1, 1), (1, 7), (5, 1), (3, 8), (3, 9), (7, 15), (160, 360),
                                             (240, 180), (4, 17), (2, 65)])
def test_row_queue_tiles_cover_every_tile_once(env, tiles_x, tiles_y):
    """The per-view trace's queues hand out every tile of the image exactly
    once (queue q: the tile rows y with y % 8 == q, each left to right)."""
    svdag, hk = env
    tiles, spare = hk.row_queue_tiles(tiles_x, tiles_y)
    assert np.array_equal(np.sort(tiles), np.arange(tiles_x * tiles_y))
    assert np.all(spare == 0xFFFFFFFF)
    # queue order: each queue's rows in increasing order, every 8th row
    pos, q_rows = 0, []
    for q in range(8):
        n = len(range(q, tiles_y, 8)) * tiles_x
        q_rows.append(tiles[pos:pos + n] // tiles_x)
        pos += n
        assert np.all(q_rows[-1] % 8 == q) and np.all(np.diff(q_rows[-1]) >= 0)
