"""Pins of the oracle's visit counts (the algorithmic-bytes model of the
bench rests on them): an exact brute force over every non-empty cube of
tiny multi-chunk, multi-LOD worlds, closed forms, and the run search's
probe count against the bisection bound."""
import math

import numpy as np
import pytest

import oracle
from brute import brute_counts, morton_rank, run_count
from paper_2505_02017_amd import scenes
from test_oracle_traversal import _adversarial_rays, _tiny_world

F = 1 << 16
FIELDS = ("chunk_visits", "chunk_entries", "node_cubes", "leaf_cubes")


def _frame(O, D):
    f = oracle._Frame()
    f.O[:] = [int(v) for v in O]
    f.A[:] = [int(v) for v in D]
    f.BX[:] = [0, 0, 0]
    f.BY[:] = [0, 0, 0]
    f.G = 0
    f.W = 1
    f.H = 1
    return oracle.Frame(f)


def _counts(w, lods, O, D, mode=1):
    h, c = w.trace_frame(np.asarray(lods, np.uint8), _frame(O, D), mode=mode, counts=True)
    return h[0], c[0]


@pytest.mark.parametrize("cfg", [
    (3, (2, 2, 2), 1, 0.2),
    (4, (2, 1, 1), 2, 0.25),
    (4, (2, 2, 1), 2, 0.08),
    (4, (1, 2, 2), 2, 0.4),
])
def test_counts_equal_brute_force(cfg):
    """Every count equals its definition, evaluated cube by cube with exact
    slab intervals, in both traversal modes (cell by cell and skipping)."""
    chunk_log2, grid, lod_count, fill = cfg
    rng = np.random.default_rng(1000 + hash(cfg) % 997)
    w, lod_grids = _tiny_world(rng, chunk_log2, grid, lod_count, fill)
    # one empty chunk (at every LOD) in each world, so entries < visits occur
    empty = int(rng.integers(0, grid[0] * grid[1] * grid[2]))
    S = 1 << chunk_log2
    w.add_chunk(empty, np.zeros(S ** 3, np.uint8))
    lod_grids[empty] = [np.zeros((S >> k,) * 3, np.uint8) for k in range(lod_count)]
    ext = [g << chunk_log2 for g in grid]
    O_list, D_list = _adversarial_rays(rng, ext, 45)
    nch = grid[0] * grid[1] * grid[2]
    seen = dict(hits=0, node=0, leaf=0, sib=0, skipped_entry=0)
    for O, D in zip(O_list, D_list):
        lods = rng.integers(0, lod_count, nch).astype(np.uint8)
        hit, ref = brute_counts(chunk_log2, grid, lod_grids, lods, O, D)
        for mode in (0, 1):
            h, c = _counts(w, lods, O, D, mode)
            assert h["hit"] == hit["hit"]
            got = {f: int(c[f]) for f in FIELDS}
            got["preceding_siblings"] = int(c["preceding_siblings"])
            assert got == ref, (O, D, mode, got, ref)
        seen["hits"] += hit["hit"]
        seen["node"] += ref["node_cubes"] > 0
        seen["leaf"] += ref["leaf_cubes"] > 0
        seen["sib"] += ref["preceding_siblings"] > 0
        seen["skipped_entry"] += ref["chunk_visits"] > ref["chunk_entries"]
    assert seen["hits"] >= 5 and seen["leaf"] >= 5 and seen["sib"] >= 3 and seen["skipped_entry"] >= 3
    if chunk_log2 >= 4:
        assert seen["node"] >= 5


def test_counts_across_chunks_of_different_lods():
    """Rays that leave a chunk at one LOD for a chunk at another: the cubes
    of the new chunk are new even where their coordinates, in the other
    LOD's cells, coincide with the last cubes of the old one."""
    rng = np.random.default_rng(31)
    w, lod_grids = _tiny_world(rng, 4, (2, 1, 1), 2, 0.1)
    n = 0
    for lods in ((0, 1), (1, 0)):
        for _ in range(40):
            y, z = (int(v) for v in rng.integers(0, 16 * F, 2))
            sgn = 1 if rng.random() < 0.5 else -1
            O = [-3 * F if sgn > 0 else 35 * F, y, z]
            D = [sgn * F, int(rng.integers(-F // 16, F // 16)), int(rng.integers(-F // 16, F // 16))]
            hit, ref = brute_counts(4, (2, 1, 1), lod_grids, lods, O, D)
            h, c = _counts(w, lods, O, D)
            got = {f: int(c[f]) for f in FIELDS + ("preceding_siblings",)}
            assert got == ref, (lods, O, D, got, ref)
            n += ref["chunk_entries"] == 2
    assert n >= 10


def test_counts_on_camera_frames_equal_brute_force():
    rng = np.random.default_rng(77)
    w, lod_grids = _tiny_world(rng, 4, (2, 2, 1), 2, 0.12)
    for _ in range(3):
        pos = rng.uniform(-6, 38, 3)
        cam = scenes.Camera(tuple(pos), (16.0, 16.0, 8.0), (0.0, 0.0, 1.0), 70.0, 6, 5).as_f32()
        fr = oracle.camera_frame(cam)
        lods = rng.integers(0, 2, 4).astype(np.uint8)
        idx = np.arange(30, dtype=np.uint32)
        _, cnt = w.trace_frame(lods, fr, idx, counts=True)
        for i, D in zip(idx, fr.directions(idx)):
            _, ref = brute_counts(4, (2, 2, 1), lod_grids, lods, fr.O.tolist(), D.tolist())
            got = {f: int(cnt[i][f]) for f in FIELDS + ("preceding_siblings",)}
            assert got == ref


def test_counts_closed_forms():
    S = 16
    # a +x ray through a full 16^3 chunk hits the entry cell (0, y, z): one
    # chunk, one 8^3 node cube, one leaf cube; preceding siblings = the path's
    # octant codes (every sibling is set), here 6 at the root (y, z >= 8) and
    # 2 at the 8^3 node (y bit 2 set, z bit 2 clear); one material run, so no
    # search probe
    w = oracle.World(4, (1, 1, 1), 1)
    w.add_chunk(0, np.full(S ** 3, 3, np.uint8))
    h, c = _counts(w, [0], [-5 * F, 13 * F + F // 2, 9 * F + F // 2], [F, 0, 0])
    assert (h["hit"], h["x"], h["y"], h["z"]) == (1, 0, 13, 9)
    assert tuple(int(c[f]) for f in FIELDS + ("preceding_siblings", "run_probes")) == (1, 1, 1, 1, 8, 0)
    # a single solid voxel (11, 6, 13): the ray along its row enters the
    # chunk, its 8^3 cube and its 4^3 cube; no sibling precedes it anywhere
    g = np.zeros((S, S, S), np.uint8)
    g[13, 6, 11] = 9
    w = oracle.World(4, (1, 1, 1), 1)
    w.add_chunk(0, g.reshape(-1))
    h, c = _counts(w, [0], [-5 * F, 6 * F + F // 2, 13 * F + F // 2], [3 * F, 0, 0])
    assert (h["hit"], h["x"], h["material"]) == (1, 11, 9)
    assert tuple(int(c[f]) for f in FIELDS + ("preceding_siblings", "run_probes")) == (1, 1, 1, 1, 0, 0)
    # the same cubes entered by a ray that misses the voxel: y = 6.5 but
    # z = 12.5 (inside the voxel's 4^3 cube, z 12..15, not in its row)
    h, c = _counts(w, [0], [-5 * F, 6 * F + F // 2, 12 * F + F // 2], [3 * F, 0, 0])
    assert h["hit"] == 0
    assert tuple(int(c[f]) for f in FIELDS) == (1, 1, 1, 1)
    # ... and one through the chunk that never enters the voxel's 8^3 cube
    h, c = _counts(w, [0], [-5 * F, 2 * F + F // 2, 2 * F + F // 2], [3 * F, 0, 0])
    assert h["hit"] == 0 and tuple(int(c[f]) for f in FIELDS) == (1, 1, 0, 0)
    # an empty world: chunks are visited, no DAG is entered
    w = oracle.World(4, (3, 1, 1), 1)
    for ci in range(3):
        w.add_chunk(ci, np.zeros(S ** 3, np.uint8))
    h, c = _counts(w, [0, 0, 0], [-5 * F, 7 * F, 7 * F], [F, 1, 0])
    assert h["hit"] == 0 and tuple(int(c[f]) for f in FIELDS) == (3, 0, 0, 0)
    # a ray pointing away from the world visits nothing
    h, c = _counts(w, [0, 0, 0], [-5 * F, 7 * F, 7 * F], [-F, 0, 0])
    assert tuple(int(c[f]) for f in FIELDS) == (0, 0, 0, 0)


@pytest.mark.parametrize("nmat", [1, 2, 3, 15])
def test_run_probes_follow_bisection_bound(nmat):
    """The run search halves [0, runs) per probe until one run is left:
    between floor(log2 runs) and ceil(log2 runs) probes, exactly log2 runs
    when that is a power of two, none for a single run."""
    rng = np.random.default_rng(nmat)
    S = 16
    g = scenes.random_grid(rng, S, 0.3, nmat=nmat).reshape(S, S, S)
    runs = run_count(g)
    w = oracle.World(4, (1, 1, 1), 1)
    w.add_chunk(0, g.reshape(-1))
    ext = [S, S, S]
    O_list, D_list = _adversarial_rays(rng, ext, 80)
    probes = set()
    for O, D in zip(O_list, D_list):
        h, c = _counts(w, [0], O, D)
        if h["hit"]:
            probes.add(int(c["run_probes"]))
        else:
            assert c["run_probes"] == 0 and c["preceding_siblings"] == 0
    lo, hi = math.floor(math.log2(runs)), math.ceil(math.log2(runs))
    assert probes and probes <= {lo, hi}, (runs, probes)
    if runs & (runs - 1) == 0:
        assert probes == {lo}
    # a full chunk whose materials alternate in 2^m equal blocks of the
    # depth-first order has 2^m runs: every hit takes m probes
    zz, yy, xx = np.meshgrid(np.arange(S), np.arange(S), np.arange(S), indexing="ij")
    rank = morton_rank(S, xx.ravel(), yy.ravel(), zz.ravel()).reshape(S, S, S)
    for m in range(0, 6):
        g2 = (1 + ((rank >> (12 - m)) & 1)).astype(np.uint8)
        assert run_count(g2) == 1 << m
        w2 = oracle.World(4, (1, 1, 1), 1)
        w2.add_chunk(0, g2.reshape(-1))
        for y in (1, 5, 9, 14):
            h, c = _counts(w2, [0], [-3 * F, y * F + F // 2, (15 - y) * F + F // 3], [F, 0, 0])
            assert h["hit"] == 1 and int(c["run_probes"]) == m, (m, y)
