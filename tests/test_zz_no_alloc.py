"""The allocation-free batch (svd_batch_trace_frames_static): its records
equal those of svd_batch_trace_frames on the same frames, on two calls in a
row (the second smaller, over the scratch the first left behind), with and
without the beam pass; sizes beyond its static scratch are refused before
anything runs."""
import numpy as np
import pytest

import oracle
from gpu_util import build_blobs, compare, gpu_world, note, oracle_world
from paper_2505_02017_amd import scenes

pytestmark = pytest.mark.gpu
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
    sw = scenes.SceneWorld("custom", 43, chunk_log2=6, grid=(4, 4, 2))
    dense = {ci: sw.chunk(c) for ci, c in enumerate(sw.chunks())}
    note("static batch world: 4x4x2 x 64^3, 4 LODs")
    w = gpu_world(svdag, torch, 6, sw.grid, 4, build_blobs(svdag, 6, 4, dense), THR, extra_bytes=1 << 22)
    return sw, w, dense


def _cams(sw, seed, n):
    rng = np.random.default_rng(seed)
    sizes = [(1, 1), (7, 5), (64, 48), (33, 17), (160, 90), (96, 96), (250, 3), (2, 130)]
    out = []
    for i in range(n):
        W, H = sizes[int(rng.integers(0, len(sizes)))]
        out.append(sw.views(1, seed * 100 + i, W, H)[0])
    return out


def _frames(svdag, sw, seed, n):
    return [svdag.svd_camera_frame(c) for c in _cams(sw, seed, n)]


def _records(frames):
    return sum(f.width * f.height for f in frames)


def test_static_batch_equals_batch(env, world):
    svdag, torch = env
    sw, w, dense = world
    b = svdag.svd_batch_create(w, 24)
    for call, (seed, n, flags) in enumerate([(7, 19, 0), (8, 6, 0), (9, 11, svdag.SVD_BEAM), (10, 3, 0)]):
        cams = _cams(sw, seed, n)
        frames = [svdag.svd_camera_frame(c) for c in cams]
        recs = _records(frames)
        note(f"static batch call {call}: {n} views, {recs} records, flags {flags}")
        ref = torch.full((recs, 4), -1, dtype=torch.int32, device="cuda")
        svdag.svd_batch_trace_frames(b, frames, ref, flags)
        out = torch.full((recs + 5, 4), -7, dtype=torch.int32, device="cuda")
        svdag.svd_batch_trace_frames_static(w, frames, out, flags)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got[:recs], ref.cpu().numpy()), f"call {call}: records differ from the batch's"
        assert np.all(got[recs:] == -7), f"call {call}: wrote past the views' records"
    svdag.svd_batch_destroy(b)
    # the last call's views also agree with the oracle
    ow = oracle_world(6, sw.grid, 4, dense)
    off = 0
    for v, c in enumerate(cams):
        n = c.width * c.height
        of = oracle.camera_frame(c)
        compare(svdag, got[off:off + n], ow.trace_frame(ow.lod_pick(of.O, THR), of), label=f"static view {v}")
        off += n


def test_static_batch_refuses_oversize(env, world):
    svdag, torch = env
    sw, w, _ = world
    f = svdag.svd_camera_frame(sw.views(1, 11, 2, 2)[0])
    out = torch.empty((3000 * 4, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(svdag.SvdError) as e:       # 2304 + 3000 * (256 + 4 * 32) bytes > 1 MiB
        svdag.svd_batch_trace_frames_static(w, [f] * 3000, out)
    assert e.value.code == svdag.SVD_ENOMEM and "1048576" in str(e.value)
    with pytest.raises(svdag.SvdError) as e:       # output smaller than the view
        svdag.svd_batch_trace_frames_static(w, [f], out[:3])
    assert e.value.code == svdag.SVD_EINVAL
    with pytest.raises(svdag.SvdError) as e:       # unknown flag
        svdag.svd_batch_trace_frames_static(w, [f], out, 0x80)
    assert e.value.code == svdag.SVD_EINVAL
    # the largest batch that fits still runs: 2304 + n * 384 <= 1 MiB
    n = (1048576 - 2304) // 384
    svdag.svd_batch_trace_frames_static(w, [f] * n, out.new_empty((4 * n, 4)))
    torch.cuda.synchronize()
