"""The numeric limits of the ray model against the oracle: a world at the
maximum extent (32768 voxels along x), camera origins at the ends of the
accepted range (-32768, 65536) voxels, and direction components up to just
below 2^31.  The kernels' code runs on the host (CPU test) and on the GPU
(GPU test); both must equal the oracle bit for bit."""
import os

import numpy as np
import pytest

import oracle
from gpu_util import compare
from paper_2505_02017_amd import scenes
import test_gpu_parity as gp

F = 1 << 16
CL, GRID, NL, THR = 7, (256, 1, 1), 2, (3000, 0, 0)
NT = min(8, os.cpu_count() or 1)
LIM = (1 << 31) - 1


def _world_content(seed=2):
    rng = np.random.default_rng(seed)
    S = 1 << CL
    dense = {}
    for ci in range(GRID[0]):
        if ci in (0, 1, 100, 127, 128, 200, 254, 255) or rng.random() < 0.03:
            dense[ci] = scenes.random_grid(rng, S, 0.03)
        else:
            dense[ci] = np.zeros((S, S, S), np.uint8)
    return dense


def _frames(seed=5, n=48, W=24, H=12):
    """Origins at the ends of the range and inside; directions along +-x at
    the largest magnitude the corner rays allow, and steep diagonals."""
    rng = np.random.default_rng(seed)
    ext = [g << CL for g in GRID]
    xs = [-(32768 * F) + 1, -(32768 * F) + F, 0, (32768 * F) - 1, 32768 * F, 65536 * F - 1]
    out = []
    for i in range(n):
        O = [xs[i % len(xs)] if rng.random() < 0.7 else int(rng.integers(-(32768 * F) + 1, 65536 * F)),
             int(rng.integers(-2 * F, (ext[1] + 2) * F)), int(rng.integers(-2 * F, (ext[2] + 2) * F))]
        sx = 1 if rng.random() < 0.5 else -1
        kind = i % 3
        if kind == 0:    # along x, as long as the corner rays allow
            bx, by = int(rng.integers(0, 1 << 20)), int(rng.integers(0, 1 << 20))
            A = [sx * (LIM - (W - 1) * bx - (H - 1) * by - 4), -by * (H // 2), -bx * (W // 2)]
            BX, BY = [sx * bx, 0, bx], [sx * by, by, 0]
        elif kind == 1:  # steep diagonals with large components on every axis
            A = [sx * int(rng.integers(1 << 29, 1 << 30)), int(rng.integers(-(1 << 30), 1 << 30)),
                 int(rng.integers(-(1 << 30), 1 << 30))]
            BX = [int(v) for v in rng.integers(-(1 << 22), 1 << 22, 3)]
            BY = [int(v) for v in rng.integers(-(1 << 22), 1 << 22, 3)]
        else:            # tiny directions (long parameter ranges)
            A = [sx * int(rng.integers(1, 64)), int(rng.integers(-8, 9)), int(rng.integers(-8, 9))]
            BX, BY = [1, 0, 0], [0, 1, 1]
        out.append((O, A, BX, BY, W, H))
    return out


@pytest.fixture(scope="module")
def content():
    from paper_2505_02017_amd import svdag
    svdag.lib()
    dense = _world_content()
    blobs = {ci: svdag.svd_chunk_build(g, CL, NL) for ci, g in dense.items()}
    ow = oracle.World(CL, GRID, NL)
    for ci, g in dense.items():
        ow.add_chunk(ci, g)
    return svdag, blobs, ow


def _check(svdag, trace, ow, frames, label):
    hits = 0
    for i, (O, A, BX, BY, W, H) in enumerate(frames):
        fr = svdag.make_frame(O, A, BX, BY, W, H)
        raw = trace(fr)
        lods = ow.lod_pick(np.array(O, np.int64), THR)
        ref = ow.trace_frame(lods, gp._oracle_frame(fr), mode=1, threads=NT)
        hits += compare(svdag, raw, ref, label=f"{label} frame {i}")
    return hits


def test_extremes_host_kernels(content):
    import host_kernels as hk
    if not os.path.exists(hk.LIB):
        pytest.skip("host kernel build missing: run __graft_entry__.build()")
    svdag, blobs, ow = content
    hw = hk.HostWorld(svdag, CL, GRID, NL, THR, blobs)
    hits = _check(svdag, lambda fr: hw.trace(fr, threads=NT)[0], ow, _frames(), "host")
    assert hits > 0


@pytest.mark.gpu
def test_extremes_gpu(content):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from gpu_util import gpu_world, trace_gpu
    svdag, blobs, ow = content
    w = gpu_world(svdag, torch, CL, GRID, NL, blobs, THR)
    hits = _check(svdag, lambda fr: trace_gpu(svdag, torch, w, fr), ow, _frames(), "gpu")
    hits += _check(svdag, lambda fr: trace_gpu(svdag, torch, w, fr, svdag.SVD_BEAM), ow, _frames(), "gpu beam")
    assert hits > 0
