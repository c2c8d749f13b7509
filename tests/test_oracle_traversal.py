"""Pins of the oracle's traversal: hand-derived cases, an exact brute force
on tiny worlds, closed forms and the invariants the method must satisfy."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from brute import brute_trace, euclid_t
from paper_2505_02017_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F = 1 << 16


def _fix(s):
    return int(Fraction(s) * F)


def _parse_cases():
    cases, cur = [], None
    for line in open(os.path.join(GOLDEN, "traversal_cases.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "case":
            cur = dict(name=tok[1], vox=[])
        elif tok[0] == "vox":
            cur["vox"].append(tuple(int(v) for v in tok[1].split(",")))
        elif tok[0] == "O":
            cur["O"] = [_fix(v) for v in tok[1:]]
        elif tok[0] == "D":
            cur["D"] = [_fix(v) for v in tok[1:]]
        elif tok[0] == "expect":
            cur["expect"] = tok[1:]
        elif tok[0] == "end":
            cases.append(cur)
    return cases


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", _parse_cases(), ids=lambda c: c["name"])
def test_golden_cases(case, mode):
    g = np.zeros((8, 8, 8), np.uint8)
    for x, y, z, m in case["vox"]:
        g[z, y, x] = m
    w = oracle.World(3, (1, 1, 1), 1)
    w.add_chunk(0, g.reshape(-1))
    h = w.trace([0], case["O"], [case["D"]], mode=mode)[0]
    e = case["expect"]
    if e[0] == "miss":
        assert h["hit"] == 0 and math.isinf(h["t"])
    else:
        x, y, z, m, face = (int(v) for v in e[1:6])
        assert (h["hit"], h["x"], h["y"], h["z"], h["material"], h["face"]) == (1, x, y, z, m, face)
        assert abs(h["t"] - float(e[6])) <= 1e-12 * max(1.0, float(e[6]))


# ----------------------------------------------------------- brute force

def _tiny_world(rng, chunk_log2, grid, lod_count, fill):
    S = 1 << chunk_log2
    w = oracle.World(chunk_log2, grid, lod_count)
    lod_grids = []
    for ci in range(grid[0] * grid[1] * grid[2]):
        g = scenes.random_grid(rng, S, fill)
        pyr = w.add_chunk(ci, g)
        lod_grids.append([p.reshape(S >> k, S >> k, S >> k) for k, p in enumerate(pyr)])
    return w, lod_grids


def _adversarial_rays(rng, ext, n_random):
    """Origins on integer/half grid points, inside and outside the world;
    directions along axes, diagonals, in grid planes and random."""
    O, D = [], []
    dirs = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, 0, -1), (1, 1, 0), (1, -1, 0), (-1, -1, -1),
            (1, 1, 1), (1, 2, 0), (2, -1, 1), (0, 1, -1), (3, 0, -2)]
    for _ in range(n_random):
        kind = rng.integers(0, 4)
        if kind == 0:   # integer lattice origin
            o = [int(rng.integers(-2, e + 2)) * F for e in ext]
        elif kind == 1:  # half-integer
            o = [int(rng.integers(-2, e + 2)) * F + F // 2 for e in ext]
        elif kind == 2:  # arbitrary fixed point
            o = [int(rng.integers(-3 * F, (e + 3) * F)) for e in ext]
        else:            # on a chunk corner / plane
            o = [int(rng.integers(0, 3)) * (ext[a] // 2) * F for a, e in enumerate(ext)]
        if rng.random() < 0.5:
            d = np.array(dirs[rng.integers(0, len(dirs))], np.int64) * int(rng.integers(1, 1 << 14)) * 17
        else:
            d = rng.integers(-(1 << 30), 1 << 30, 3)
            if rng.random() < 0.3:
                d[rng.integers(0, 3)] = 0
        if not np.any(d):
            d[0] = 1
        O.append(o)
        D.append([int(v) for v in d])
    return O, D


def _compare(h, b, D):
    assert h["hit"] == b["hit"]
    if not b["hit"]:
        return
    assert (h["x"], h["y"], h["z"], h["lod"], h["material"], h["chunk"], h["face"]) == \
           (b["x"], b["y"], b["z"], b["lod"], b["material"], b["chunk"], b["face"])
    t = euclid_t(b["t_rational"], D)
    assert abs(h["t"] - t) <= 1e-9 * max(1.0, t)


@pytest.mark.parametrize("cfg", [
    (3, (1, 1, 1), 1, 0.3),
    (3, (2, 2, 1), 1, 0.15),
    (4, (2, 1, 1), 2, 0.25),
    (4, (1, 2, 2), 2, 0.1),
])
def test_brute_force_tiny_worlds(cfg):
    chunk_log2, grid, lod_count, fill = cfg
    rng = np.random.default_rng(hash(cfg) & 0xFFFF)
    w, lod_grids = _tiny_world(rng, chunk_log2, grid, lod_count, fill)
    ext = [g << chunk_log2 for g in grid]
    O_list, D_list = _adversarial_rays(rng, ext, 60)
    nch = grid[0] * grid[1] * grid[2]
    for O, D in zip(O_list, D_list):
        lods = rng.integers(0, lod_count, nch).astype(np.uint8)
        b = brute_trace(chunk_log2, grid, lod_grids, lods, O, D)
        for mode in (0, 1):
            h = w.trace(lods, O, [D], mode=mode)[0]
            _compare(h, b, D)


def test_brute_force_camera_rays():
    rng = np.random.default_rng(99)
    w, lod_grids = _tiny_world(rng, 4, (2, 2, 1), 2, 0.12)
    for _ in range(3):
        pos = rng.uniform(-6, 38, 3)
        cam = scenes.Camera(tuple(pos), (16.0, 16.0, 8.0), (0.0, 0.0, 1.0), 70.0, 6, 5).as_f32()
        fr = oracle.camera_frame(cam)
        lods = rng.integers(0, 2, 4).astype(np.uint8)
        idx = np.arange(30, dtype=np.uint32)
        hs = w.trace_frame(lods, fr, idx)
        for i, D in zip(idx, fr.directions(idx)):
            b = brute_trace(4, (2, 2, 1), lod_grids, lods, fr.O.tolist(), D.tolist())
            _compare(hs[i], b, D.tolist())


# ------------------------------------------------------- invariants / closed forms

def test_dense_equals_dag_and_skip_equals_plain():
    """DDA on the dense LOD grids == the DAG walk; skipping empty DAG
    subtrees changes nothing."""
    sw = scenes.SceneWorld("custom", 5, chunk_log2=5, grid=(3, 2, 2))
    w = oracle.World(5, sw.grid, 3)
    for c in sw.chunks():
        w.add_chunk(w.chunk_index(c), sw.chunk(c), keep_dense=True)
    for cam in sw.views(3, 1, 40, 30):
        fr = oracle.camera_frame(cam)
        lods = w.lod_pick(fr.O, (8, 24, 0))
        ref = w.trace_frame(lods, fr, mode=0, threads=4)
        for mode in (1, 2):
            h = w.trace_frame(lods, fr, mode=mode, threads=4)
            for f in ("hit", "x", "y", "z", "lod", "material", "chunk", "face"):
                assert np.array_equal(h[f], ref[f]), (mode, f)
            assert np.array_equal(h["t"], ref["t"])
        assert ref["hit"].mean() > 0.2


def test_lod_k_equals_downsampled_grid():
    """Tracing a chunk at LOD k equals tracing its level-k grid: replicate
    each level-k cell into 2^k^3 voxels, trace at LOD 0; the first fine voxel
    lies in the coarse hit cell, with the same t and material."""
    rng = np.random.default_rng(8)
    S = 64
    g = scenes.random_grid(rng, S, 0.08)
    wc = oracle.World(6, (1, 1, 1), 4)
    pyr = wc.add_chunk(0, g)
    O_list, D_list = _adversarial_rays(rng, [S, S, S], 80)
    for k in (1, 2, 3):
        Rk = S >> k
        up = pyr[k].reshape(Rk, Rk, Rk)
        for ax in range(3):
            up = np.repeat(up, 1 << k, axis=ax)
        wf = oracle.World(6, (1, 1, 1), 1)
        wf.add_chunk(0, up.reshape(-1))
        for O, D in zip(O_list, D_list):
            hc = wc.trace([k], O, [D])[0]
            hf = wf.trace([0], O, [D])[0]
            assert hc["hit"] == hf["hit"]
            if hc["hit"]:
                assert (hf["x"] >> k, hf["y"] >> k, hf["z"] >> k) == \
                       (hc["x"] >> k, hc["y"] >> k, hc["z"] >> k)
                assert hc["material"] == hf["material"]
                assert hc["t"] == hf["t"]


def test_closed_forms():
    S = 16
    # empty world: every ray misses
    w = oracle.World(4, (2, 1, 1), 1)
    w.add_chunk(0, np.zeros(S ** 3, np.uint8))
    w.add_chunk(1, np.zeros(S ** 3, np.uint8))
    rng = np.random.default_rng(2)
    O_list, D_list = _adversarial_rays(rng, [32, 16, 16], 50)
    for O, D in zip(O_list, D_list):
        assert w.trace([0, 0], O, [D])[0]["hit"] == 0
    # full chunk: the first visited cell inside it, t = slab entry
    w = oracle.World(4, (1, 1, 1), 1)
    w.add_chunk(0, np.full(S ** 3, 3, np.uint8))
    O = [-5 * F, 3 * F + F // 2, 7 * F]
    h = w.trace([0], O, [[F, 0, 0]])[0]
    assert (h["hit"], h["x"], h["y"], h["z"], h["face"], h["t"]) == (1, 0, 3, 7, 1, 5.0)
    O = [20 * F, 20 * F, 20 * F]
    h = w.trace([0], O, [[-F, -F, -F]])[0]
    assert (h["x"], h["y"], h["z"], h["face"]) == (15, 15, 15, 2)
    assert abs(h["t"] - 4 * math.sqrt(3)) < 1e-12
    # axis-parallel rays: first solid cell of the row
    g = np.zeros((S, S, S), np.uint8)
    g[4, 9, [2, 11]] = [5, 6]
    w = oracle.World(4, (1, 1, 1), 1)
    w.add_chunk(0, g.reshape(-1))
    assert w.trace([0], [0, 9 * F + 1, 4 * F + 1], [[F, 0, 0]])[0]["x"] == 2
    h = w.trace([0], [15 * F, 9 * F + 1, 4 * F + 1], [[-3, 0, 0]])[0]
    assert (h["x"], h["material"], h["face"]) == (11, 6, 2)
    assert abs(h["t"] - 3.0) < 1e-12  # enters x=11 through its upper face x=12


def test_oracle_on_generated_terrain_skip_modes():
    """Empty-subtree skipping agrees with cell-by-cell stepping on a
    generated multi-chunk terrain with 4 LODs (subsampled pixels)."""
    sw = scenes.SceneWorld("custom", 17, chunk_log2=6, grid=(4, 4, 1))
    w = oracle.World(6, sw.grid, 4)
    for c in sw.chunks():
        w.add_chunk(w.chunk_index(c), sw.chunk(c))
    seen = set()
    for cam in sw.views(3, 3, 96, 64):
        fr = oracle.camera_frame(cam)
        lods = w.lod_pick(fr.O, (48, 96, 160))
        idx = np.arange(0, 96 * 64, 7, dtype=np.uint32)
        a = w.trace_frame(lods, fr, idx, mode=0, threads=4)
        b = w.trace_frame(lods, fr, idx, mode=1, threads=4)
        assert np.array_equal(a, b)
        seen |= set(a["lod"][a["hit"] == 1].tolist())
    assert len(seen) >= 3
