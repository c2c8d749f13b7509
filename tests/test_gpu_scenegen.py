"""The GPU copy of the terrain generator: every chunk it writes into device
memory equals, byte for byte, the host generator's chunk.  It is what makes
the 32x32-chunk map of 1024^3 chunks practical to build, so the check covers
that map and the single 1024^3 terrain chunk as well as small worlds with
several z layers, chunks smaller than a cave wavelength, and chunks where
boxes overlap."""
import os

import numpy as np
import pytest

from gpu_util import note
from paper_2505_02017_amd import scenes

pytestmark = pytest.mark.gpu
NT = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _check(torch, sw, chunks, work=None):
    S = sw.S
    out = torch.empty(S ** 3, dtype=torch.uint8, device="cuda")
    for c in chunks:
        note(f"scenegen {sw.kind} seed {sw.seed} S {S} chunk {c}")
        out.fill_(0xEE)
        work = sw.chunk_device(c, out, work)
        host = sw.chunk(c, threads=NT)
        dev = out.cpu().numpy()
        bad = np.flatnonzero(dev != host)
        assert bad.size == 0, (f"{sw.kind} {c}: {bad.size} bytes differ, first at {bad[0]} "
                               f"(gpu {dev[bad[0]]}, host {host[bad[0]]})")
    return work


def test_small_worlds_equal_host(torch):
    work = None
    sw = scenes.SceneWorld("custom", 7, chunk_log2=5, grid=(2, 2, 2))
    work = _check(torch, sw, list(sw.chunks()), work)
    sw = scenes.SceneWorld("custom", 3, chunk_log2=3, grid=(4, 4, 2))  # chunk edge below the cave wavelength
    work = _check(torch, sw, [(0, 0, 0), (3, 2, 1), (1, 3, 0), (2, 2, 1)], work)
    sw = scenes.SceneWorld("custom", 11, chunk_log2=6, grid=(3, 2, 1))
    _check(torch, sw, list(sw.chunks()), work)


def test_map512_chunks_with_boxes_equal_host(torch):
    sw = scenes.SceneWorld("map512", 2025)
    ip, dp, boxes = sw._terrain_params()
    assert len(boxes) == sw.nbox > 0
    _check(torch, sw, [(3, 5, 0), (0, 0, 0), (15, 15, 0), (8, 2, 0)])


def test_1024_chunks_equal_host(torch):
    sw = scenes.SceneWorld("map1024", 2025)
    work = _check(torch, sw, [(5, 7, 0), (31, 0, 0)])
    sw = scenes.SceneWorld("terrain1024", 2025)
    _check(torch, sw, [(0, 0, 0)], work)


def test_errors(torch):
    sw = scenes.SceneWorld("noise64", 1)
    out = torch.empty(sw.S ** 3, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        sw.chunk_device((0, 0, 0), out)
    sw = scenes.SceneWorld("custom", 7, chunk_log2=5, grid=(2, 2, 1))
    out = torch.empty(sw.S ** 3, dtype=torch.uint8, device="cuda")
    with pytest.raises(ValueError):
        sw.chunk_device((2, 0, 0), out)
    with pytest.raises(ValueError):
        sw.chunk_device((0, 0, 1), out)
    with pytest.raises(ValueError):
        sw.chunk_device((0, 0, 0), out[:-1])
    with pytest.raises(ValueError):
        sw.chunk_device((0, 0, 0), out.cpu())
