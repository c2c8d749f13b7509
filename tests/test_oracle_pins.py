"""Pins of the CPU oracle against the paper and against mathematics.

None of these checks re-runs the oracle's own formula: each compares it with
a hand-derived fixture, a closed form, an exhaustive enumeration or an
invariant the paper states.
"""
import math
import os

import numpy as np
import pytest

import oracle
from brute import downsample_counts, morton_rank
from paper_2505_02017_amd import scenes

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _grid3(flat, R):
    return np.asarray(flat).reshape(R, R, R)  # [z, y, x]


# ---------------------------------------------------------------- golden DAGs

def _parse_dag_cases():
    cases, cur = [], None
    for line in open(os.path.join(GOLDEN, "dag_small.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "case":
            cur = dict(name=tok[1], vox=[], fill=None)
        elif tok[0] == "R":
            cur["R"] = int(tok[1])
        elif tok[0] == "vox":
            cur["vox"].append(tuple(int(v) for v in tok[1].split(",")))
        elif tok[0] == "fill":
            cur["fill"] = int(tok[1])
        elif tok[0] == "words":
            cur["words"] = [int(v) for v in tok[1:]]
        elif tok[0] == "leaves":
            cur["leaves"] = [int(v, 16) for v in tok[1:]]
        elif tok[0] == "rle":
            cur["rle"] = [tuple(int(x) for x in v.split(":")) for v in tok[1:]]
        elif tok[0] == "end":
            cases.append(cur)
    return cases


@pytest.mark.parametrize("case", _parse_dag_cases(), ids=lambda c: c["name"])
def test_dag_golden(case):
    R = case["R"]
    g = np.zeros((R, R, R), np.uint8)
    if case["fill"]:
        g[:] = case["fill"]
    for x, y, z, m in case["vox"]:
        g[z, y, x] = m
    d = oracle.Dag(g.reshape(-1), R)
    assert d.words.tolist() == case["words"]
    assert d.leaves.tolist() == case["leaves"]
    assert list(zip(d.rle_start.tolist(), d.rle_mat.tolist())) == case["rle"]


# ---------------------------------------------------------- LOD downsampling

def test_downsample_density_rule_exhaustive():
    """Section 3.4: solid iff >= density (= 2) of the 8 children are solid.
    All 256 occupancy patterns of one 2x2x2 block, as 8 blocks of a 4^3 grid
    per call."""
    pats = np.arange(256)
    for base in range(0, 256, 8):
        g = np.zeros((4, 4, 4), np.uint8)
        for j in range(8):
            p = int(pats[base + j])
            bz, by, bx = (j >> 2) & 1, (j >> 1) & 1, j & 1
            for i in range(8):
                if (p >> i) & 1:
                    g[2 * bz + ((i >> 2) & 1), 2 * by + ((i >> 1) & 1), 2 * bx + (i & 1)] = 1
        out = _grid3(oracle.downsample(g.reshape(-1), 4), 2)
        for j in range(8):
            p = int(pats[base + j])
            bz, by, bx = (j >> 2) & 1, (j >> 1) & 1, j & 1
            assert (out[bz, by, bx] > 0) == (bin(p).count("1") >= 2), p


@pytest.mark.parametrize("mats,expect", [
    ([5], 0),                      # a single voxel vanishes
    ([5, 3], 3),                   # tie 1:1 -> smallest ID
    ([5, 5, 3], 5),                # mode
    ([3, 5, 5, 3, 7], 3),          # tie 2:2 -> smallest
    ([9, 2, 9, 2, 9, 2, 1, 1], 2), # tie 3:3 -> smallest
    ([7] * 8, 7),                  # full block
    ([250, 250], 250),
])
def test_downsample_material_mode(mats, expect):
    g = np.zeros((2, 2, 2), np.uint8).reshape(-1)
    g[: len(mats)] = mats
    # embed the block in a 4^3 grid (needs R >= 4 for symmetry of the call)
    G = np.zeros((4, 4, 4), np.uint8)
    G[2:4, 0:2, 2:4] = g.reshape(2, 2, 2)
    out = _grid3(oracle.downsample(G.reshape(-1), 4), 2)
    assert out[1, 0, 1] == expect
    assert out.sum() == expect


def test_downsample_random_counts():
    rng = np.random.default_rng(3)
    g = scenes.random_grid(rng, 16, 0.3)
    out = _grid3(oracle.downsample(g, 16), 8)
    cnt = downsample_counts(_grid3(g, 16))
    assert np.array_equal(out > 0, cnt >= 2)


# --------------------------------------------------------------- DAG invariants

def _check_dag(g, R):
    d = oracle.Dag(g, R)
    G = _grid3(g, R)
    # expand(DAG) reproduces the grid exactly, materials included
    assert np.array_equal(d.expand(), g)
    # root count = number of solid voxels
    assert d.n_solid == int((g > 0).sum())
    words = d.words
    if d.n_solid == 0:
        assert words.size == 0
        return d
    assert words[1] == d.n_solid
    # minimality: unique nodes per level = number of distinct non-empty
    # sub-cube contents (occupancy only) of that size
    L = R.bit_length() - 1
    occ = (G > 0)
    for lev in range(2, L + 1):
        e = 1 << lev
        n = R // e
        blocks = occ.reshape(n, e, n, e, n, e).transpose(0, 2, 4, 1, 3, 5).reshape(n ** 3, -1)
        nonempty = blocks[blocks.any(axis=1)]
        distinct = len({b.tobytes() for b in np.packbits(nonempty, axis=1)})
        assert d.level_nodes[lev] == distinct, (lev, d.level_nodes[lev], distinct)
    # node format: header bits 8..31 zero, node size 8..40 bytes (Section 3.2)
    i, sizes = 0, []
    while i < words.size:
        mask = int(words[i])
        assert mask & ~0xFF == 0 and mask != 0
        k = bin(mask).count("1")
        sizes.append(8 + 4 * k)
        i += 2 + k
    assert i == words.size
    assert 8 <= min(sizes) and max(sizes) <= 40
    # run blocks: start at 0, strictly increasing, adjacent materials differ
    rs, rm = d.rle_start, d.rle_mat
    assert rs[0] == 0 and np.all(np.diff(rs.astype(np.int64)) > 0)
    assert np.all(rm[1:] != rm[:-1])
    assert rs[-1] < d.n_solid
    return d


def test_dag_invariants_random():
    rng = np.random.default_rng(11)
    for R, fill in [(8, 0.1), (8, 0.5), (16, 0.05), (16, 0.3), (32, 0.2), (32, 0.7)]:
        for structured in (True, False):
            _check_dag(scenes.random_grid(rng, R, fill, structured=structured), R)


def test_dag_full_and_empty():
    R = 32
    d = _check_dag(np.full(R ** 3, 4, np.uint8), R)
    # one node per internal level plus one all-ones bitmap
    assert d.level_nodes[2:6] == [1, 1, 1, 1]
    assert d.leaves.tolist() == [0xFFFFFFFFFFFFFFFF]
    assert d.words.size == 3 * 10
    e = oracle.Dag(np.zeros(R ** 3, np.uint8), R)
    assert e.words.size == 0 and e.n_solid == 0


def test_dag_subtree_counts_bruteforce():
    """The count word of every node equals the number of solid voxels of the
    cube it stands for (checked by walking the tree with positions)."""
    rng = np.random.default_rng(5)
    R = 32
    g = scenes.random_grid(rng, R, 0.25)
    G = _grid3(g, R) > 0
    d = oracle.Dag(g, R)
    W, Lv = d.words, d.leaves
    L = R.bit_length() - 1

    def walk(off, lev, x0, y0, z0):
        mask, cnt = int(W[off]), int(W[off + 1])
        e = 1 << lev
        assert cnt == int(G[z0:z0 + e, y0:y0 + e, x0:x0 + e].sum())
        h, slot = e // 2, 0
        for o in range(8):
            cx, cy, cz = x0 + h * (o & 1), y0 + h * ((o >> 1) & 1), z0 + h * ((o >> 2) & 1)
            sub = G[cz:cz + h, cy:cy + h, cx:cx + h]
            assert bool((mask >> o) & 1) == bool(sub.any())
            if not (mask >> o) & 1:
                continue
            p = int(W[off + 2 + slot])
            slot += 1
            if lev > 3:
                walk(p, lev - 1, cx, cy, cz)
            else:
                assert bin(int(Lv[p])).count("1") == int(sub.sum())
    walk(0, L, 0, 0, 0)


def test_dfs_index_is_morton_rank_and_materials():
    """Section 3.3: the DFS index from summed preceding-sibling counts is the
    rank of the cell in depth-first (Morton) order, and the run-block lookup
    of that index returns the cell's material."""
    rng = np.random.default_rng(21)
    R = 16
    g = scenes.random_grid(rng, R, 0.3)
    G = _grid3(g, R)
    d = oracle.Dag(g, R)
    zs, ys, xs = np.nonzero(G)
    rank = morton_rank(R, xs, ys, zs)
    for x, y, z, r in zip(xs, ys, zs, rank):
        solid, dfs = d.lookup(int(x), int(y), int(z))
        assert solid and dfs == int(r)
        assert d.material(dfs) == G[z, y, x]
    # empty cells: not solid, with a correct empty cube level
    ez, ey, ex = np.nonzero(G == 0)
    for x, y, z in list(zip(ex, ey, ez))[:500]:
        solid, lev = d.lookup(int(x), int(y), int(z))
        assert not solid
        e = 1 << lev
        bx, by, bz = (int(x) // e) * e, (int(y) // e) * e, (int(z) // e) * e
        assert not G[bz:bz + e, by:by + e, bx:bx + e].any()
        if lev < R.bit_length() - 1:
            e2 = 2 * e
            bx, by, bz = (int(x) // e2) * e2, (int(y) // e2) * e2, (int(z) // e2) * e2
            assert G[bz:bz + e2, by:by + e2, bx:bx + e2].any()


def test_dag_on_generated_chunk():
    w = scenes.SceneWorld("noise64", 1)
    g = w.chunk((0, 0, 0))
    d = _check_dag(g, 64)
    assert 0.25 < d.n_solid / 64 ** 3 < 0.35


# ---------------------------------------------------------------------- camera

def test_camera_closed_form_axis_aligned():
    """Looking along +x with +z up: right = -y, up' = +z; pixel directions
    follow the pinhole formula; G is the largest exponent that fits."""
    cam = scenes.Camera((10.0, 20.0, 30.0), (11.0, 20.0, 30.0), (0.0, 0.0, 1.0), 90.0, 4, 2)
    f = oracle.camera_frame(cam)
    assert f.O.tolist() == [10 << 16, 20 << 16, 30 << 16]
    tau, a = math.tan(math.radians(45.0)), 2.0
    for py in range(2):
        for px in range(4):
            u = (2 * (px + 0.5) / 4 - 1) * tau * a
            v = (1 - 2 * (py + 0.5) / 2) * tau
            ideal = np.array([1.0, -u, v])
            D = f.A + px * f.BX + py * f.BY
            assert np.all(np.abs(D) < 2 ** 31)
            assert np.allclose(D / 2.0 ** f.G, ideal, atol=2.0 ** -(f.G - 3))
    # maximality: at G+1 some corner component reaches 2^31
    corners = [f.A + px * f.BX + py * f.BY for px in (0, 3) for py in (0, 1)]
    assert max(np.abs(c).max() for c in corners) * 2 >= 2 ** 31 - 8


def test_camera_symmetry_and_range():
    rng = np.random.default_rng(4)
    for _ in range(50):
        pos = rng.uniform(-1000, 5000, 3)
        d = rng.normal(size=3)
        W, H = int(rng.integers(1, 3000)), int(rng.integers(1, 2000))
        cam = scenes.Camera(tuple(pos), tuple(pos + d), (0.0, 0.0, 1.0),
                            float(rng.uniform(10, 120)), W, H).as_f32()
        try:
            f = oracle.camera_frame(cam)
        except ValueError:
            continue
        for px, py in [(0, 0), (W - 1, 0), (0, H - 1), (W - 1, H - 1)]:
            D = f.A + px * f.BX + py * f.BY
            assert np.all(np.abs(D) < 2 ** 31)
        # direction of the middle of the image is the forward vector
        fwd = np.array(cam.target, np.float64) - np.array(cam.pos, np.float64)
        mid = f.A + (W - 1) / 2 * f.BX + (H - 1) / 2 * f.BY
        cosang = mid @ fwd / np.linalg.norm(mid) / np.linalg.norm(fwd)
        assert cosang > 1 - 1e-9
        # vertical FOV: angle between top-centre and bottom-centre rays (H >= 2)
        if H >= 50:
            top = f.A + (W - 1) / 2 * f.BX - 0.5 * f.BY
            bot = f.A + (W - 1) / 2 * f.BX + (H - 0.5) * f.BY
            ang = math.degrees(math.acos(top @ bot / np.linalg.norm(top) / np.linalg.norm(bot)))
            # each of A, BX, BY is rounded by <= 1/2 unit at scale 2^G, so a
            # direction errs by <= (1 + W + H)/2 units of a vector of length
            # >= 2^(G-2); the angle by at most twice that ratio
            tol = math.degrees(2 * (1 + W + H) / 2 / 2.0 ** (f.G - 2))
            assert abs(ang - cam.vfov_deg) < tol


def test_camera_rejects():
    bad = [
        scenes.Camera((0, 0, 0), (0, 0, 0), (0, 0, 1), 60, 8, 8),        # no direction
        scenes.Camera((0, 0, 0), (0, 0, 5), (0, 0, 1), 60, 8, 8),        # up parallel
        scenes.Camera((0, 0, 0), (1, 0, 0), (0, 0, 1), 0, 8, 8),         # zero FOV
        scenes.Camera((0, 0, 0), (1, 0, 0), (0, 0, 1), 60, 0, 8),        # no pixels
        scenes.Camera((70000, 0, 0), (1, 0, 0), (0, 0, 1), 60, 8, 8),    # outside guard band
        scenes.Camera((-40000, 0, 0), (1, 0, 0), (0, 0, 1), 60, 8, 8),
    ]
    for c in bad:
        with pytest.raises(ValueError):
            oracle.camera_frame(c)


# -------------------------------------------------------------------- LOD pick

def test_lod_pick_closed_forms():
    """Eq. 1 distance term: LOD = number of thresholds the camera-to-centre
    distance reaches.  Exact at the threshold."""
    w = oracle.World(9, (4, 1, 1), 4)  # chunk centres at x = 256, 768, 1280, 1792
    F = 1 << 16
    y, z = 256 * F, 256 * F
    O = [256 * F, y, z]
    assert w.lod_pick(O).tolist() == [0, 1, 2, 2]   # d = 0, 512, 1024, 1536
    O = [(768 + 256) * F, y, z]                      # d = 768, 256, 256, 768
    assert w.lod_pick(O).tolist() == [1, 1, 1, 1]
    O = [(768 + 256) * F - 1, y, z]                  # 256 - 2^-16 from chunk 1
    assert w.lod_pick(O).tolist() == [1, 0, 1, 1]
    O = [256 * F, y + 4096 * F, z]                   # d = 4096 exactly
    assert w.lod_pick(O).tolist()[0] == 3
    O = [256 * F, y + 4096 * F - 1, z]
    assert w.lod_pick(O).tolist()[0] == 2
    # 3D distance, not per-axis: (3,4,0)*205 = 1025 >= 1024
    O = [(256 + 3 * 205) * F, y + 4 * 205 * F, z]
    assert w.lod_pick(O).tolist()[0] == 2
    # fewer LODs cap the count
    w2 = oracle.World(9, (4, 1, 1), 2)
    assert w2.lod_pick([256 * F, y, z]).tolist() == [0, 1, 1, 1]
