"""GPU parity: libsvdag (through its C ABI) against the CPU oracle.

Bit-exact on hit flag, hit voxel, LOD, entry face, material and chunk;
t within 1e-4 relative (exactly 0 stays 0).  Every input is seeded."""
import os

import numpy as np
import pytest

import oracle
from gpu_util import build_blobs, compare, gpu_world, note, oracle_world, trace_gpu
from paper_2505_02017_amd import scenes

pytestmark = pytest.mark.gpu
F = 1 << 16
NT = min(16, os.cpu_count() or 1)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_02017_amd import svdag
    svdag.lib()
    return svdag, torch


def _frames(rng, ext, n, W=8, H=8):
    dirs = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, 0, -1), (1, 1, 0), (1, -1, 0), (-1, -1, -1),
            (1, 1, 1), (1, 2, 0), (2, -1, 1), (0, 1, -1), (3, 0, -2)]
    axes = [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (0, -1, 1)]
    out = []
    for i in range(n):
        kind = i % 4
        if kind == 0:
            O = [int(rng.integers(-2, e + 2)) * F for e in ext]
        elif kind == 1:
            O = [int(rng.integers(-2, e + 2)) * F + F // 2 for e in ext]
        elif kind == 2:
            O = [int(rng.integers(-3 * F, (e + 3) * F)) for e in ext]
        else:
            O = [int(rng.integers(0, 3)) * (e // 2) * F for e in ext]
        if rng.random() < 0.5:
            s = int(rng.integers(1, 1 << 12)) * 64
            A = [d * s for d in dirs[rng.integers(0, len(dirs))]]
            BX = [v * int(rng.integers(0, 3)) * s // 4 for v in axes[rng.integers(0, len(axes))]]
            BY = [v * int(rng.integers(0, 3)) * s // 4 for v in axes[rng.integers(0, len(axes))]]
        else:
            A = [int(v) for v in rng.integers(-(1 << 29), 1 << 29, 3)]
            BX = [int(v) for v in rng.integers(-(1 << 24), 1 << 24, 3)]
            BY = [int(v) for v in rng.integers(-(1 << 24), 1 << 24, 3)]
        out.append((O, A, BX, BY, W, H))
    return out


def _oracle_frame(svdag_frame):
    f = oracle._Frame()
    f.O[:] = list(svdag_frame.O)
    f.A[:] = list(svdag_frame.A)
    f.BX[:] = list(svdag_frame.BX)
    f.BY[:] = list(svdag_frame.BY)
    f.G = svdag_frame.G
    f.W = svdag_frame.width
    f.H = svdag_frame.height
    return oracle.Frame(f)


@pytest.mark.parametrize("cfg", [
    (3, (1, 1, 1), 1, 0.3, (256, 1024, 4096)),
    (3, (2, 2, 1), 1, 0.15, (256, 1024, 4096)),
    (4, (2, 1, 1), 2, 0.25, (12, 0, 0)),
    (5, (2, 2, 2), 3, 0.1, (16, 40, 0)),
    (6, (2, 1, 1), 4, 0.05, (20, 50, 90)),
])
def test_tiny_worlds_adversarial_frames(env, cfg):
    svdag, torch = env
    chunk_log2, grid, lod_count, fill, thr = cfg
    rng = np.random.default_rng(sum(grid) * 1000 + chunk_log2 * 10 + lod_count)
    S = 1 << chunk_log2
    nch = grid[0] * grid[1] * grid[2]
    dense = {ci: scenes.random_grid(rng, S, fill) for ci in range(nch)}
    note(f"tiny world {cfg}")
    w = gpu_world(svdag, torch, chunk_log2, grid, lod_count,
                  build_blobs(svdag, chunk_log2, lod_count, dense), thr)
    ow = oracle_world(chunk_log2, grid, lod_count, dense)
    ext = [g * S for g in grid]
    hits = 0
    for i, (O, A, BX, BY, W, H) in enumerate(_frames(rng, ext, 40)):
        fr = svdag.make_frame(O, A, BX, BY, W, H)
        raw = trace_gpu(svdag, torch, w, fr)
        vt = svdag.svd_view_table(w)
        raw_nb = trace_gpu(svdag, torch, w, fr, flags=svdag.SVD_BEAM)
        assert np.array_equal(raw, raw_nb), f"frame {i}: the beam pass changed a record"
        lods = ow.lod_pick(np.array(O, np.int64), thr)
        assert np.array_equal(vt & 3, lods), f"frame {i}: LOD pick differs"
        ref = ow.trace_frame(lods, _oracle_frame(fr), mode=1, threads=NT)
        hits += compare(svdag, raw, ref, label=f"{cfg} frame {i}")
    assert hits > 0


def test_noise64_full_frames(env):
    svdag, torch = env
    sw = scenes.SceneWorld("noise64", 1)
    dense = {0: sw.chunk((0, 0, 0))}
    note("noise64 64^3, 256x256 views")
    w = gpu_world(svdag, torch, 6, (1, 1, 1), 1, build_blobs(svdag, 6, 1, dense))
    ow = oracle_world(6, (1, 1, 1), 1, dense)
    for v, cam in enumerate(sw.views(3, 11)):
        raw = trace_gpu(svdag, torch, w, svdag.to_camera(cam))
        fr = oracle.camera_frame(cam)
        ref = ow.trace_frame(np.zeros(1, np.uint8), fr, mode=1, threads=NT)
        n = compare(svdag, raw, ref, label=f"noise64 view {v}")
        assert n > 0.2 * ref.size


@pytest.fixture(scope="module")
def terrain(env):
    """A 4x4x2 world of 64^3 terrain chunks with boxes, 4 LODs."""
    svdag, torch = env
    sw = scenes.SceneWorld("custom", 23, chunk_log2=6, grid=(4, 4, 2))
    dense = {sw_ci: sw.chunk(c) for sw_ci, c in enumerate(sw.chunks())}
    thr = (48, 96, 160)
    note("terrain 4x4x2 x 64^3, 4 LODs")
    w = gpu_world(svdag, torch, 6, sw.grid, 4, build_blobs(svdag, 6, 4, dense), thr)
    ow = oracle_world(6, sw.grid, 4, dense)
    return sw, w, ow, thr


def test_terrain_lods_full_frames_cull_invariant(env, terrain):
    svdag, torch = env
    sw, w, ow, thr = terrain
    seen_lods, culled = set(), 0
    for v, cam in enumerate(sw.views(4, 5, 160, 120)):
        note(f"terrain view {v}")
        raw = trace_gpu(svdag, torch, w, svdag.to_camera(cam))
        vt = svdag.svd_view_table(w)
        raw_nc = trace_gpu(svdag, torch, w, svdag.to_camera(cam), flags=svdag.SVD_NO_CULL)
        assert np.array_equal(raw, raw_nc), f"view {v}: culling changed the image"
        raw_nb = trace_gpu(svdag, torch, w, svdag.to_camera(cam), flags=svdag.SVD_NO_CULL | svdag.SVD_BEAM)
        assert np.array_equal(raw, raw_nb), f"view {v}: the beam pass changed the image"
        culled += int(np.count_nonzero(vt & 4))
        fr = oracle.camera_frame(cam)
        lods = ow.lod_pick(fr.O, thr)
        assert np.array_equal(vt & 3, lods)
        ref = ow.trace_frame(lods, fr, mode=1, threads=NT)
        compare(svdag, raw, ref, label=f"terrain view {v}")
        seen_lods |= set(ref["lod"][ref["hit"] == 1].tolist())
    assert len(seen_lods) >= 3 and culled > 0


def test_ragged_and_tiny_images(env, terrain):
    svdag, torch = env
    sw, w, ow, thr = terrain
    for (W, H) in [(1, 1), (1, 37), (29, 1), (17, 23), (250, 3)]:
        cam = sw.views(1, W * 7 + H, W, H)[0]
        note(f"image {W}x{H}")
        raw = trace_gpu(svdag, torch, w, svdag.to_camera(cam))
        fr = oracle.camera_frame(cam)
        ref = ow.trace_frame(ow.lod_pick(fr.O, thr), fr, mode=1, threads=NT)
        compare(svdag, raw, ref, label=f"{W}x{H}")


def test_stage_once_trace_repeatedly(env, terrain):
    """The persistent trace leaves its work queue at zero: tracing one staged
    view several times gives the same records every time; a trace whose
    frame differs from the staged one is refused."""
    svdag, torch = env
    sw, w, ow, thr = terrain
    cams = sw.views(2, 77, 97, 61)
    f0, f1 = (svdag.svd_camera_frame(c) for c in cams)
    outs = [torch.full((97 * 61, 4), -1, dtype=torch.int32, device="cuda") for _ in range(3)]
    svdag.svd_view_stage(w, f0)
    for o in outs:
        svdag.svd_view_trace(w, f0, o)
    torch.cuda.synchronize()
    ref = outs[0].cpu().numpy()
    for o in outs[1:]:
        assert np.array_equal(o.cpu().numpy(), ref)
    fr = oracle.camera_frame(cams[0])
    compare(svdag, ref, ow.trace_frame(ow.lod_pick(fr.O, thr), fr, threads=NT), label="staged once")
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_view_trace(w, f1, outs[0])
    assert e.value.code == svdag.SVD_EINVAL


def test_upload_replace_evict(env):
    svdag, torch = env
    rng = np.random.default_rng(77)
    S, grid = 16, (2, 1, 1)
    a = {0: scenes.random_grid(rng, S, 0.2), 1: scenes.random_grid(rng, S, 0.2)}
    b0 = scenes.random_grid(rng, S, 0.35)
    blobs = build_blobs(svdag, 4, 2, a)
    w = gpu_world(svdag, torch, 4, grid, 2, blobs, (10, 0, 0), extra_bytes=1 << 16)
    cam = scenes.Camera((-6.0, 7.5, 9.0), (16.0, 8.0, 8.0), (0.0, 0.0, 1.0), 60.0, 24, 16)
    fr = oracle.camera_frame(cam)
    # replace chunk 0
    svdag.svd_chunk_upload(w, (0, 0, 0), svdag.svd_chunk_build(b0, 4, 2))
    ow = oracle_world(4, grid, 2, {0: b0, 1: a[1]})
    compare(svdag, trace_gpu(svdag, torch, w, svdag.to_camera(cam)),
            ow.trace_frame(ow.lod_pick(fr.O, (10, 0, 0)), fr), label="replaced")
    # evicted chunks make the trace refuse before enqueueing anything
    svdag.svd_chunk_evict(w, (1, 0, 0))
    out = torch.empty((cam.width * cam.height, 4), dtype=torch.int32, device="cuda")
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_trace_view(w, svdag.to_camera(cam), out)
    assert e.value.code == svdag.SVD_ENOTFOUND
    svdag.svd_chunk_upload(w, (1, 0, 0), svdag.svd_chunk_build(a[1], 4, 2))
    compare(svdag, trace_gpu(svdag, torch, w, svdag.to_camera(cam)),
            ow.trace_frame(ow.lod_pick(fr.O, (10, 0, 0)), fr), label="re-uploaded")


def test_errors_before_enqueue(env):
    svdag, torch = env
    rng = np.random.default_rng(3)
    g = scenes.random_grid(rng, 8, 0.3)
    blob = svdag.svd_chunk_build(g, 3, 1)
    desc = svdag.make_desc(3, (1, 1, 1), 1)
    small = torch.empty(svdag.table_bytes((1, 1, 1)) + 256, dtype=torch.uint8, device="cuda")
    w = svdag.svd_world_create(desc, small)
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_chunk_upload(w, (0, 0, 0), blob)
    assert e.value.code == svdag.SVD_ENOMEM
    out = torch.empty((64, 4), dtype=torch.int32, device="cuda")
    cam = scenes.Camera((-3.0, 4.0, 4.0), (4.0, 4.0, 4.0), (0.0, 0.0, 1.0), 60.0, 8, 8)
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_trace_view(w, svdag.to_camera(cam), out)
    assert e.value.code == svdag.SVD_ENOTFOUND
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_world_create(desc, small[:100])
    assert e.value.code == svdag.SVD_ENOMEM
    big = torch.empty(svdag.table_bytes((1, 1, 1)) + (1 << 16), dtype=torch.uint8, device="cuda")
    w = svdag.svd_world_create(desc, big)
    svdag.svd_chunk_upload(w, (0, 0, 0), blob)
    for bad, code in [(scenes.Camera((1e5, 0, 0), (0, 0, 0), (0, 0, 1), 60, 8, 8), svdag.SVD_ERANGE),
                      (scenes.Camera((0, 0, 0), (0, 0, 0), (0, 0, 1), 60, 8, 8), svdag.SVD_EINVAL),
                      (scenes.Camera((0, 0, 0), (1, 0, 0), (0, 0, 1), 200, 8, 8), svdag.SVD_EINVAL)]:
        with pytest.raises(svdag.SvdError) as e:
            svdag.svd_trace_view(w, svdag.to_camera(bad), out)
        assert e.value.code == code


def test_zero_direction_rays(env):
    """Pixels whose direction is exactly zero never move: a hit at the
    origin's cell when it is solid at the picked LOD, else a miss; equal to
    the oracle on the GPU too (per-view and batched)."""
    svdag, torch = env
    chunk_log2, grid, lod_count, thr = 4, (2, 2, 1), 2, (20, 0, 0)
    rng = np.random.default_rng(77)
    S = 1 << chunk_log2
    dense = {ci: scenes.random_grid(rng, S, 0.5) for ci in range(4)}
    w = gpu_world(svdag, torch, chunk_log2, grid, lod_count, build_blobs(svdag, chunk_log2, lod_count, dense), thr,
                  extra_bytes=1 << 20)
    ow = oracle_world(chunk_log2, grid, lod_count, dense)
    hits = misses = 0
    frames = []
    for i in range(90):
        # pixel (0, 0) has D = A = 0; a third of the origins lie in the
        # world's low corner, where cell and chunk coordinates coincide
        hi = [2, 2, 2] if i % 3 == 0 else [2 * S, 2 * S, S]
        O = [int(rng.integers(-F if i % 3 else 0, hi[a] * F + (F if i % 3 else 0))) for a in range(3)]
        O = [min(max(o, -F), (2 * S + 1) * F) for o in O]
        sx = 1 if i % 2 else -1
        fr = svdag.make_frame(O, [0, 0, 0], [sx * 977, 31, -17], [0, 0, 0], 5, 1)
        frames.append(fr)
        raw = trace_gpu(svdag, torch, w, fr)
        ref = ow.trace_frame(ow.lod_pick(np.array(O, np.int64), thr), _oracle_frame(fr), mode=1, threads=NT)
        compare(svdag, raw, ref, label=f"zero-direction frame {i}")
        h = svdag.decode_hits(raw[:1])["hit"][0]
        hits += int(h == 1)
        misses += int(h == 0)
    assert hits > 5 and misses > 5
    # the same frames as one batch
    out = torch.empty((5 * len(frames), 4), dtype=torch.int32, device="cuda")
    b = svdag.svd_batch_create(w, len(frames))
    svdag.svd_batch_trace_frames(b, frames, out)
    torch.cuda.synchronize()
    raw_b = out.cpu().numpy()
    for i, fr in enumerate(frames):
        ref = ow.trace_frame(ow.lod_pick(np.array(list(fr.O), np.int64), thr), _oracle_frame(fr), mode=1,
                             threads=NT)
        compare(svdag, raw_b[5 * i:5 * i + 5], ref, label=f"zero-direction batch view {i}")
    svdag.svd_batch_destroy(b)
