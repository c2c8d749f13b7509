"""The oracle's touch counter (the compulsory-traffic figure of the bench):
a closed-form single-voxel case, and bounds against the per-ray visit
counts (a part touched by several rays is counted once)."""
import numpy as np

import oracle
from paper_2505_02017_amd import scenes

F = 1 << 16


def _frame(O, A, BX, BY, W, H):
    f = oracle._Frame()
    f.O[:] = list(O)
    f.A[:] = list(A)
    f.BX[:] = list(BX)
    f.BY[:] = list(BY)
    f.G = 0
    f.W = W
    f.H = H
    return oracle.Frame(f)


def test_single_voxel_closed_form():
    g = np.zeros(512, np.uint8)
    g[3 + 8 * (4 + 8 * 5)] = 7  # voxel (3, 4, 5), index x + R*(y + R*z)
    w = oracle.World(3, (1, 1, 1), 1)
    w.add_chunk(0, g.reshape(8, 8, 8))
    lods = np.zeros(1, np.uint8)
    # one ray along +x through the voxel's row (y = 4.5, z = 5.5)
    fr = _frame((-2 * F, 4 * F + F // 2, 5 * F + F // 2), (F, 0, 0), (0, 0, 0), (0, 0, 0), 1, 1)
    ref = w.trace_frame(lods, fr, mode=1)
    assert ref["hit"][0] == 1 and (ref["x"][0], ref["y"][0], ref["z"][0]) == (3, 4, 5)
    t = w.touch_frame(lods, fr)
    # 8^3 chunk: the root (level 3) has leaf children only: one child word,
    # one leaf bitmap, one prefix count on the hit path; one run, so no probe
    assert t == {"rays": 1, "hits": 1, "child_words": 1, "leaves": 1, "prefixes": 1,
                 "run_starts": 0, "run_materials": 1, "chunks": 1, "dags": 1}
    # a ray pointing away from the chunk touches nothing
    fr2 = _frame((-2 * F, 4 * F + F // 2, 5 * F + F // 2), (-F, 0, 0), (0, 0, 0), (0, 0, 0), 1, 1)
    t2 = w.touch_frame(lods, fr2)
    assert t2["hits"] == 0 and t2["chunks"] == 0 and t2["child_words"] == 0


def test_touched_parts_bounded_by_visit_counts():
    rng = np.random.default_rng(4)
    CL, grid, NL = 5, (2, 2, 1), 2
    S = 1 << CL
    w = oracle.World(CL, grid, NL)
    for ci in range(4):
        w.add_chunk(ci, scenes.random_grid(rng, S, 0.08))
    ext = [g * S for g in grid]
    for i in range(12):
        O = [int(rng.integers(-F, (e + 1) * F)) for e in ext]
        A = [int(v) for v in rng.integers(-(1 << 20), 1 << 20, 3)]
        BX = [int(v) for v in rng.integers(-(1 << 14), 1 << 14, 3)]
        BY = [int(v) for v in rng.integers(-(1 << 14), 1 << 14, 3)]
        fr = _frame(O, A, BX, BY, 16, 12)
        lods = w.lod_pick(np.array(O, np.int64), (40, 0, 0))
        ref, cnt = w.trace_frame(lods, fr, mode=1, threads=4, counts=True)
        t = w.touch_frame(lods, fr, threads=4)
        assert t["rays"] == 16 * 12 and t["hits"] == int(ref["hit"].sum())
        # each part counted once, while the visit counts count every ray
        assert t["child_words"] <= int(cnt["node_cubes"].sum() + cnt["leaf_cubes"].sum())
        assert t["leaves"] <= int(cnt["leaf_cubes"].sum())
        assert t["chunks"] <= int(cnt["chunk_visits"].sum()) and t["chunks"] <= 4
        assert t["dags"] <= int(cnt["chunk_entries"].sum()) and t["dags"] <= 4
        assert t["prefixes"] <= t["child_words"] and t["run_materials"] <= t["hits"]
        if t["hits"]:
            assert t["prefixes"] > 0 and t["run_materials"] > 0 and t["dags"] > 0
        # the same frame twice: the counts do not depend on threads
        assert w.touch_frame(lods, fr, threads=1) == t
