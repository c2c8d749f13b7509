"""Exact brute-force references for tiny worlds (pure Python, test-only).

These restate the *definitions* in a form unrelated to the oracle's cell
stepping, so that they can pin it:

* ``brute_trace``: a ray p(t) = (O + t D) / 2^16, t >= 0, visits cell v iff
  the per-axis half-open slab intervals of v intersect; the hit is the solid
  cell (at its chunk's LOD) whose intersection starts first.  An interval
  lower bound is closed ([t) for D > 0) or open ((t) for D < 0); at equal t a
  closed start comes first.  No stepping, no tie rule is coded: it falls out
  of the interval arithmetic.
* ``morton_rank``: depth-first order of cells in an octree with child code
  x | y<<1 | z<<2, computed from interleaved coordinate bits.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

FIX = 1 << 16


def _interval(o: int, d: int, lo: int, hi: int):
    """t-interval where lo <= o + t d < hi (fixed-point units).

    Returns (lower, lower_open, upper, upper_closed) or None if empty for all
    t; bounds are Fractions or +-inf."""
    if d > 0:
        return (Fraction(lo - o, d), False, Fraction(hi - o, d), False)
    if d < 0:
        return (Fraction(o - hi, -d), True, Fraction(o - lo, -d), True)
    if lo <= o < hi:
        return (-math.inf, False, math.inf, False)
    return None


def cell_entry(O, D, box_lo, box_hi):
    """Entry instant (t, open) of the ray into the half-open box, t >= 0, or None."""
    lower, lower_open = Fraction(0), False
    upper, upper_closed = math.inf, False
    per_axis = []
    for a in range(3):
        iv = _interval(O[a], D[a], box_lo[a], box_hi[a])
        if iv is None:
            return None
        per_axis.append(iv)
        lv, lo_open, uv, up_closed = iv
        if lv > lower or (lv == lower and lo_open and not lower_open):
            lower, lower_open = lv, lo_open
        if uv < upper or (uv == upper and not up_closed and upper_closed):
            upper, upper_closed = uv, up_closed
    if lower < upper or (lower == upper and not lower_open and upper_closed):
        return (lower, lower_open, per_axis)
    return None


def downsample_counts(g: np.ndarray) -> np.ndarray:
    """Per coarse cell: number of solid children (g is (R,R,R) indexed [z,y,x])."""
    R = g.shape[0]
    s = (g > 0).reshape(R // 2, 2, R // 2, 2, R // 2, 2)
    return s.sum(axis=(1, 3, 5))


def brute_trace(chunk_log2, grid, lod_grids, lods, O, D):
    """First solid cell along the ray.

    lod_grids[ci][k]: (R_k, R_k, R_k) uint8 array indexed [z, y, x].
    Returns dict(hit, x, y, z, lod, material, chunk, face, t_rational).
    """
    best = None
    S = 1 << chunk_log2
    # float prefilter ordering only: exact comparison decides
    cands = []
    for cz in range(grid[2]):
        for cy in range(grid[1]):
            for cx in range(grid[0]):
                ci = cx + grid[0] * (cy + grid[1] * cz)
                k = int(lods[ci])
                g = lod_grids[ci][k]
                zz, yy, xx = np.nonzero(g)
                cs = 1 << k
                for x, y, z in zip(xx.tolist(), yy.tolist(), zz.tolist()):
                    v = (cx * S + x * cs, cy * S + y * cs, cz * S + z * cs)
                    cands.append((ci, k, v, int(g[z, y, x])))
    # rough float lower bound to visit cells in a good order; exactness below
    def approx(c):
        v, cs = c[2], 1 << c[1]
        lo = 0.0
        for a in range(3):
            if D[a] > 0:
                lo = max(lo, (v[a] * FIX - O[a]) / D[a])
            elif D[a] < 0:
                lo = max(lo, (O[a] - (v[a] + cs) * FIX) / -D[a])
        return lo
    cands.sort(key=approx)
    for ci, k, v, m in cands:
        a0 = approx((ci, k, v, m))
        if best is not None and a0 > float(best[0]) * (1 + 1e-9) + 1e-12:
            break
        cs = 1 << k
        e = cell_entry(O, D, [v[a] * FIX for a in range(3)], [(v[a] + cs) * FIX for a in range(3)])
        if e is None:
            continue
        key = (e[0], 1 if e[1] else 0)
        if best is None or key < (best[0], best[1]):
            face = 0
            for a in range(3):
                lv, lo_open = e[2][a][0], e[2][a][1]
                if D[a] != 0 and lv == e[0] and lo_open == e[1]:
                    face = 1 + 2 * a + (1 if D[a] < 0 else 0)
                    break
            best = (e[0], key[1], dict(hit=1, x=v[0], y=v[1], z=v[2], lod=k, material=m,
                                       chunk=ci, face=face, t_rational=e[0], key=key))
    if best is None:
        return dict(hit=0, x=0, y=0, z=0, lod=0, material=0, chunk=-1, face=0, t_rational=None, key=None)
    return best[2]


def _occupied_cubes(g: np.ndarray, level: int) -> np.ndarray:
    """Per cube of 2^level cells: does it hold a solid cell ([z, y, x])."""
    n = g.shape[0] >> level
    e = 1 << level
    return (g > 0).reshape(n, e, n, e, n, e).any(axis=(1, 3, 5))


def brute_counts(chunk_log2, grid, lod_grids, lods, O, D):
    """Visit counts by definition, from the grids alone (no stepping):

    * chunk_visits: chunks whose box the ray enters at or before its hit
      (all it enters, on a miss);
    * chunk_entries: those of them whose grid at the picked LOD is not empty;
    * node_cubes / leaf_cubes: non-empty cubes of 2^l cells (3 <= l < root,
      resp. l = 2) of those grids that the ray enters at or before its hit;
    * preceding_siblings: at a hit, over the internal levels l = root .. 3 of
      the hit cell's path, the non-empty child cubes whose octant comes
      before the path's (the counts the DFS index of Section 3.3 adds up).

    An entry instant is compared with the hit's by (t, open-after-closed),
    as the interval arithmetic gives them."""
    hit = brute_trace(chunk_log2, grid, lod_grids, lods, O, D)
    hk = hit["key"]
    S = 1 << chunk_log2

    def before(e):
        return e is not None and (hk is None or (e[0], 1 if e[1] else 0) <= hk)

    out = dict(chunk_visits=0, chunk_entries=0, node_cubes=0, leaf_cubes=0, preceding_siblings=0)
    for cz in range(grid[2]):
        for cy in range(grid[1]):
            for cx in range(grid[0]):
                ci = cx + grid[0] * (cy + grid[1] * cz)
                base = (cx * S, cy * S, cz * S)
                e = cell_entry(O, D, [b * FIX for b in base], [(b + S) * FIX for b in base])
                if not before(e):
                    continue
                out["chunk_visits"] += 1
                k = int(lods[ci])
                g = lod_grids[ci][k]
                if not g.any():
                    continue
                out["chunk_entries"] += 1
                top = g.shape[0].bit_length() - 1
                for l in range(2, top):
                    edge = 1 << (l + k)  # voxels
                    for z, y, x in zip(*np.nonzero(_occupied_cubes(g, l))):
                        lo = (base[0] + int(x) * edge, base[1] + int(y) * edge, base[2] + int(z) * edge)
                        e = cell_entry(O, D, [v * FIX for v in lo], [(v + edge) * FIX for v in lo])
                        if before(e):
                            out["node_cubes" if l >= 3 else "leaf_cubes"] += 1
    if hit["hit"]:
        ci, k = hit["chunk"], hit["lod"]
        c = (ci % grid[0], (ci // grid[0]) % grid[1], ci // (grid[0] * grid[1]))
        v = [(hit[ax] - c[a] * S) >> k for a, ax in enumerate("xyz")]
        g = lod_grids[ci][k]
        top = g.shape[0].bit_length() - 1
        for l in range(top, 2, -1):
            occ = _occupied_cubes(g, l - 1)
            node = [(v[a] >> l) << 1 for a in range(3)]  # first child cube of the node, per axis
            o = sum(((v[a] >> (l - 1)) & 1) << a for a in range(3))
            for i in range(o):
                if occ[node[2] + ((i >> 2) & 1), node[1] + ((i >> 1) & 1), node[0] + (i & 1)]:
                    out["preceding_siblings"] += 1
    return hit, out


def run_count(g: np.ndarray) -> int:
    """Maximal runs of equal material along the depth-first order of the
    solid cells of g ([z, y, x])."""
    R = g.shape[0]
    zz, yy, xx = np.nonzero(g)
    if zz.size == 0:
        return 0
    mats = g[zz, yy, xx][np.argsort(morton_rank(R, xx, yy, zz))]
    return 1 + int(np.count_nonzero(mats[1:] != mats[:-1]))


def euclid_t(t_rational: Fraction, D) -> float:
    n = math.sqrt(sum(int(d) * int(d) for d in D))
    return float(t_rational) * n / FIX


def morton_rank(R: int, xs, ys, zs) -> np.ndarray:
    """Rank of each cell in depth-first octree order (child code x|y<<1|z<<2)."""
    xs, ys, zs = (np.asarray(a, np.int64) for a in (xs, ys, zs))
    key = np.zeros(xs.shape, np.int64)
    L = R.bit_length() - 1
    for b in range(L - 1, -1, -1):
        oct_ = ((xs >> b) & 1) | (((ys >> b) & 1) << 1) | (((zs >> b) & 1) << 2)
        key = (key << 3) | oct_
    order = np.argsort(key, kind="stable")
    rank = np.empty_like(order)
    rank[order] = np.arange(order.size)
    return rank
