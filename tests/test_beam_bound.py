"""The beam pass's per-cube decisions, as the kernels compute them (host
build of kernels.hip), against exact integer arithmetic.

The pass may drop a cube only if it lies strictly outside the closed cone of
the tile's corner rays, and may report a distance only up to the cube's true
Chebyshev distance from the camera; both are what makes its start bound
exact.  Its cone test runs in FP32 with a margin of 1 (in units of the
normal scaled to a largest component in [1/2, 1)) against a rounding error
bounded by 0.14, so a cube more than 1.2 outside some side plane must be
dropped.  Cubes are placed around the corner rays, where the planes are."""
from __future__ import annotations

import numpy as np
import pytest

import host_kernels as hk


def _corners(A, BX, BY, tile):
    x0, y0, x1, y1 = tile
    return [[A[a] + px * BX[a] + py * BY[a] for a in range(3)]
            for px, py in ((x0, y0), (x1, y0), (x1, y1), (x0, y1))]


def _cross(u, v):
    return [u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]]


def _dot(u, v):
    return sum(x * y for x, y in zip(u, v))


def exact_planes(A, BX, BY, tile):
    """Side planes (normal, sign) with sign * normal . C >= 0 inside, or None
    for a degenerate cone."""
    C = _corners(A, BX, BY, tile)
    planes = []
    for i in range(4):
        m = _cross(C[i], C[(i + 1) % 4])
        s0, s1 = _dot(m, C[(i + 2) % 4]), _dot(m, C[(i + 3) % 4])
        if s0 >= 0 and s1 >= 0 and (s0 or s1):
            planes.append((m, 1))
        elif s0 <= 0 and s1 <= 0 and (s0 or s1):
            planes.append((m, -1))
        else:
            return None
    return planes


def outside_margin(planes, O, lo, s):
    """min over the side planes of the farthest corner's signed value, in
    units of the normal scaled to a largest component in [1/2, 1), voxels."""
    best = None
    for m, sg in planes:
        e = max(abs(x) for x in m).bit_length()  # 2^(e-1) <= max|m| < 2^e
        v = 0
        for a in range(3):
            n = sg * m[a]
            X = (lo[a] + s) if n > 0 else lo[a]
            v += n * ((X << 16) - O[a])
        val = v / float(1 << (e + 16))  # exact sign; magnitude to ~1e-16 relative
        if v < 0 and val == 0.0:
            val = -1e-300
        best = val if best is None else min(best, val)
    return best


def cheb_floor(O, lo, s):
    d = 0
    for a in range(3):
        l, h = lo[a] << 16, (lo[a] + s) << 16
        d = max(d, l - O[a], O[a] - h)
    return d >> 16


def _cases(seed, n):
    """Frames whose corner rays pass through chosen points of the world, with
    cubes of every size around those points (and some anywhere)."""
    rng = np.random.default_rng(seed)
    made = 0
    while made < n:
        A = [int(rng.integers(-(1 << 29), 1 << 29)) for _ in range(3)]
        k = int(rng.integers(8, 18))
        BX = [int(rng.integers(-(1 << k), 1 << k)) for _ in range(3)]
        BY = [int(rng.integers(-(1 << k), 1 << k)) for _ in range(3)]
        x0, y0 = int(rng.integers(0, 2000)), int(rng.integers(0, 1000))
        w, h = [(15, 3), (7, 7), (31, 1), (1, 1), (3, 15)][int(rng.integers(0, 5))]
        tile = (x0, y0, x0 + w, y0 + h)
        C = _corners(A, BX, BY, tile)
        # camera placed so that corner ray i passes through P, d voxels on
        i = int(rng.integers(0, 4))
        c = C[i]
        mx = max(abs(x) for x in c)
        if mx == 0:
            continue
        P = [float(rng.uniform(0, 32768)) for _ in range(3)]
        d = float(rng.uniform(1, 20000))
        O = [int(round(P[a] * 65536 - d * 65536 * c[a] / mx)) for a in range(3)]
        if not all(-(1 << 31) < x < (1 << 32) for x in O):
            continue
        made += 1
        cubes = []
        for _ in range(12):
            s = 1 << int(rng.integers(0, 11))
            if rng.random() < 0.85:
                lo = [int(np.floor(P[a])) - int(rng.integers(0, s + 1)) + int(rng.integers(-3, 4)) for a in range(3)]
            else:
                lo = [int(rng.integers(0, 32768)) for _ in range(3)]
            lo = [min(max(x, 0), 32768 - s) for x in lo]
            cubes.append((lo, s))
        yield O, A, BX, BY, tile, cubes


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_beam_cube_decisions_are_conservative(seed):
    hk.lib()
    checked = dropped = near = 0
    for O, A, BX, BY, tile, cubes in _cases(seed, 1500):
        planes = exact_planes(A, BX, BY, tile)
        for lo, s in cubes:
            drop, dist = hk.beam_cube(O, A, BX, BY, tile, lo, s)
            assert dist <= cheb_floor(O, lo, s), (O, lo, s, dist)
            if planes is None:
                assert drop is None
                continue
            assert drop is not None
            margin = outside_margin(planes, O, lo, s)
            checked += 1
            if drop:
                dropped += 1
                # dropped only when strictly outside the closed cone
                assert margin < 0, (O, A, BX, BY, tile, lo, s, margin)
            if margin < -1.2:
                assert drop, (O, A, BX, BY, tile, lo, s, margin)
            if -3.0 < margin < 3.0:
                near += 1
    # the cases reach both outcomes and the band around the planes
    assert checked > 10000 and dropped > 1000 and near > 500, (checked, dropped, near)


def test_beam_distance_is_tight_for_whole_voxels():
    """For a camera at a whole voxel, the distance bound equals the cube's
    Chebyshev distance exactly."""
    hk.lib()
    rng = np.random.default_rng(7)
    A, BX, BY = [1 << 20, 3, 5], [0, 1 << 10, 0], [0, 0, 1 << 10]
    for _ in range(2000):
        O = [int(rng.integers(-32767, 65536)) << 16 for _ in range(3)]
        s = 1 << int(rng.integers(0, 11))
        lo = [int(rng.integers(0, 32768 - s + 1)) for _ in range(3)]
        _, dist = hk.beam_cube(O, A, BX, BY, (0, 0, 15, 3), lo, s)
        assert dist == min(cheb_floor(O, lo, s), 65535)
