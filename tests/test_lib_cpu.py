"""Host-side checks of libsvdag (no GPU needed): exported symbols, the
host builder against the oracle, blob serialisation and validation, and the
camera frame against the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2505_02017_amd import scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _svdag():
    from paper_2505_02017_amd import svdag
    if not os.path.exists(svdag.LIB_PATH):
        from paper_2505_02017_amd import build
        build.build_lib()
    return svdag


def test_exports_match_header():
    svdag = _svdag()
    hdr = open(os.path.join(ROOT, "include", "svdag.h")).read()
    declared = set(re.findall(r"\b(svd_[a-z_]+)\s*\(", hdr))
    declared -= {"svd_hit"}
    L = ctypes.CDLL(svdag.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(svdag.EXPORTS)


def test_header_constants_match_binding():
    """Every numeric #define of the C header has the same value in the binding."""
    svdag = _svdag()
    hdr = open(os.path.join(ROOT, "include", "svdag.h")).read()
    consts = re.findall(r"^#define\s+(SVD_[A-Z0-9_]+)\s+\(?(-?(?:0x[0-9A-Fa-f]+|\d+))u?\)?", hdr, re.M)
    assert len(consts) >= 12
    for name, val in consts:
        if hasattr(svdag, name):
            assert getattr(svdag, name) == int(val, 0), name
    for name in ("SVD_OK", "SVD_EINVAL", "SVD_EIO", "SVD_NO_CULL", "SVD_BEAM", "SVD_MAX_TIMED_PASSES"):
        assert hasattr(svdag, name), name


def _compare_blob(svdag, g, R, lod_count):
    b = svdag.svd_chunk_build(g, R.bit_length() - 1, lod_count)
    pyr = oracle.pyramid(g, R, lod_count)
    for k in range(lod_count):
        d = oracle.Dag(pyr[k], R >> k)
        w, l, rs, rm = svdag.svd_blob_canonical(b, k)
        assert np.array_equal(w, d.words), k
        assert np.array_equal(l, d.leaves), k
        assert np.array_equal(rs, d.rle_start), k
        assert np.array_equal(rm, d.rle_mat), k
        st = svdag.svd_blob_stats_get(b, k)
        assert st["n_solid"] == d.n_solid
        assert st["level_nodes"][2:d.R.bit_length()] == d.level_nodes[2:d.R.bit_length()]
        if d.n_solid:
            G = pyr[k].reshape(R >> k, R >> k, R >> k)
            zs, ys, xs = np.nonzero(G)
            assert st["aabb_lo"] == [xs.min(), ys.min(), zs.min()]
            assert st["aabb_hi"] == [xs.max(), ys.max(), zs.max()]
    return b


@pytest.mark.parametrize("R,fill,lods", [(8, 0.3, 1), (16, 0.02, 2), (32, 0.2, 3), (32, 0.9, 3),
                                          (64, 0.05, 4)])
def test_builder_matches_oracle_random(R, fill, lods):
    svdag = _svdag()
    rng = np.random.default_rng(R * 100 + int(fill * 100))
    for structured in (True, False):
        _compare_blob(svdag, scenes.random_grid(rng, R, fill, structured=structured), R, lods)


def test_builder_matches_oracle_generated():
    svdag = _svdag()
    _compare_blob(svdag, scenes.SceneWorld("noise64", 3).chunk((0, 0, 0)), 64, 4)
    sw = scenes.SceneWorld("custom", 9, chunk_log2=7, grid=(2, 2, 1))
    _compare_blob(svdag, sw.chunk((1, 0, 0)), 128, 4)


def test_builder_matches_oracle_uniform_regions():
    """Large regions of one material (the builder's uniform fast paths),
    with single voxels and rows that break them at every alignment: a
    different material, an empty voxel, a run that starts mid-block."""
    svdag = _svdag()
    rng = np.random.default_rng(12)
    R = 64
    z = np.arange(R)[:, None, None]
    g = np.broadcast_to(np.where(z < 40, 1 + z // 8, 0), (R, R, R)).astype(np.uint8).copy()
    g[20:28, 8:40, 16:48] = 0                                   # a cave
    g[8:12, 4:8, 0:64] = 9                                      # a row of another material
    for _ in range(60):                                         # isolated breaks
        x, y, zz = (int(v) for v in rng.integers(0, R, 3))
        g[zz, y, x] = int(rng.integers(0, 16))
    _compare_blob(svdag, g.reshape(-1), R, 4)
    g2 = np.full((R, R, R), 7, np.uint8)
    g2[:, :, 1::4] = 5                                          # breaks every 4-voxel row
    _compare_blob(svdag, g2.reshape(-1), R, 3)


def test_builder_empty_and_full():
    svdag = _svdag()
    b = _compare_blob(svdag, np.zeros(32 ** 3, np.uint8), 32, 3)
    assert svdag.svd_blob_stats_get(b, 0)["n_words"] == 0
    _compare_blob(svdag, np.full(32 ** 3, 200, np.uint8), 32, 3)


def test_blob_bytes_roundtrip_and_rejects():
    svdag = _svdag()
    rng = np.random.default_rng(7)
    g = scenes.random_grid(rng, 32, 0.2)
    b = svdag.svd_chunk_build(g, 5, 3)
    data = svdag.svd_blob_to_bytes(b)
    b2 = svdag.svd_blob_from_bytes(data)
    assert svdag.svd_blob_to_bytes(b2) == data
    for k in range(3):
        assert svdag.svd_blob_stats_get(b, k) == svdag.svd_blob_stats_get(b2, k)
    # truncations and trailing bytes are rejected
    for n in (0, 3, 16, len(data) // 2, len(data) - 1):
        with pytest.raises(svdag.SvdError) as e:
            svdag.svd_blob_from_bytes(data[:n])
        assert e.value.code == svdag.SVD_EFORMAT
    with pytest.raises(svdag.SvdError):
        svdag.svd_blob_from_bytes(data + b"\0" * 8)
    # single-word corruptions: rejected, or accepted only if still consistent
    arr = np.frombuffer(data, np.uint32).copy()
    for _ in range(300):
        bad = arr.copy()
        i = int(rng.integers(4, bad.size))
        bad[i] ^= np.uint32(1 << int(rng.integers(0, 32)))
        try:
            b3 = svdag.svd_blob_from_bytes(bad.tobytes())
        except svdag.SvdError as e:
            assert e.code in (svdag.SVD_EFORMAT, svdag.SVD_ERANGE)
            continue
        # accepted: it must re-serialise to itself (a consistent blob)
        assert svdag.svd_blob_to_bytes(b3) == bad.tobytes()


def test_build_rejects_bad_arguments():
    svdag = _svdag()
    with pytest.raises(svdag.SvdError):
        svdag.svd_chunk_build(np.zeros(8 ** 3, np.uint8), 3, 2)   # coarsest grid < 8^3
    with pytest.raises(svdag.SvdError):
        svdag.svd_chunk_build(np.zeros(4 ** 3, np.uint8), 2, 1)   # chunk too small


def test_camera_frame_matches_oracle():
    svdag = _svdag()
    rng = np.random.default_rng(12)
    cams = []
    for kind in ("noise64", "custom"):
        sw = scenes.SceneWorld(kind, 4, chunk_log2=6, grid=(3, 3, 1))
        cams += sw.views(20, 2)
    for _ in range(200):
        pos = rng.uniform(-30000, 60000, 3)
        cams.append(scenes.Camera(tuple(pos), tuple(pos + rng.normal(size=3) * rng.uniform(0.01, 1e4)),
                                  tuple(rng.normal(size=3)), float(rng.uniform(0.5, 170)),
                                  int(rng.integers(1, 5000)), int(rng.integers(1, 3000))).as_f32())
    n_ok = 0
    for cam in cams:
        try:
            fo = oracle.camera_frame(cam)
        except ValueError:
            with pytest.raises(svdag.SvdError):
                svdag.svd_camera_frame(cam)
            continue
        fl = svdag.svd_camera_frame(cam)
        assert list(fl.O) == fo.O.tolist()
        assert list(fl.A) == fo.A.tolist()
        assert list(fl.BX) == fo.BX.tolist()
        assert list(fl.BY) == fo.BY.tolist()
        assert fl.G == fo.G
        n_ok += 1
    assert n_ok > 150


def test_gpu_scene_generator_host_contract():
    """The GPU copy of the terrain generator loads and exports its two entry
    points; the world parameters it is given decode to the host world's boxes;
    its workspace is the stated layout (int32 column heights, then the two
    cave lattice tables of doubles, each 256-byte aligned); bad arguments are
    refused before anything reaches a device.  Its bytes are compared with the
    host generator's on the GPU."""
    sw = scenes.SceneWorld("map1024", 2025)
    ip, dp, boxes = sw._terrain_params()
    assert list(ip) == [1, 512, 1024, 512, 64, sw.nbox] and list(dp) == [400.0, 0.6803]
    X = sw.extent[0]
    assert boxes.shape == (sw.nbox, 8) and (boxes[:, 7] == 0).all()
    assert ((boxes[:, 6] >= 9) & (boxes[:, 6] <= 15)).all()
    assert (boxes[:, 0] >= 0).all() and (boxes[:, 3] <= X).all() and (boxes[:, 3] > boxes[:, 0]).all()
    assert (boxes[:, 2] >= 0).all() and (boxes[:, 5] <= 1024).all() and (boxes[:, 5] >= boxes[:, 2]).all()
    L = scenes._gpu_lib()
    a256 = lambda v: (v + 255) // 256 * 256
    # cave octaves: wavelengths 64 and 32, lattice ((S-1) >> log2(lam)) + 3 per axis
    assert L.sgg_work_bytes(ip, dp, 10) == a256(4 << 20) + a256(8 * 18 ** 3) + a256(8 * 34 ** 3)
    ipn = (ctypes.c_int64 * 6)(*ip)
    ipn[0] = 0  # not a terrain world
    assert L.sgg_work_bytes(ipn, dp, 10) == 0
    assert L.sgg_gen_chunk(ipn, dp, 1, 10, 0, 0, 0, None, 0, None, None, 0, None) == -1
    assert L.sgg_gen_chunk(ip, dp, 1, 10, 0, 0, 0, None, 0, None, None, 0, None) == -1
    assert L.sgg_gen_chunk(ip, dp, 1, 11, 0, 0, 0, None, 0, None, None, 0, None) == -1


def test_kernel_hash_is_the_built_sources():
    """The library reports the hash of the kernel sources it was built from;
    the tuning cache and the kernel profiles are keyed by it."""
    svdag = _svdag()
    from paper_2505_02017_amd import build
    h = svdag.svd_kernel_hash()
    assert re.fullmatch(r"[0-9a-f]{16}", h)
    assert h == build.kernel_source_hash(), "library older than its kernel sources: rebuild"


def test_tune_cache_file(tmp_path):
    svdag = _svdag()
    path = str(tmp_path / "tune.txt")
    k1 = "dev=gfx950:sramecc+:xnack-/256cu/2400mhz kernel=0123456789abcdef kind=view cl=9 grid=16x16x2 lods=4 flags=0 views=4 res=2560x1440*4"
    k2 = k1.replace("kind=view", "kind=batch")
    assert svdag.svd_tune_cache_lookup(path, k1) is None          # no file yet
    svdag.svd_tune_cache_store(path, k1, 16, 1, 6, 0.5)
    svdag.svd_tune_cache_store(path, k2, 8, 2, 5, 1.25)
    r = svdag.svd_tune_cache_lookup(path, k1)
    assert (r.tile_w, r.claim, r.blocks_per_cu, r.from_cache, r.configs_timed) == (16, 1, 6, 1, 0)
    assert abs(r.ms - 0.5) < 1e-6 and r.key.decode() == k1
    assert svdag.svd_tune_cache_lookup(path, k2).as_dict()["tile"] == "8x8"
    # a prefix of a key is another key
    assert svdag.svd_tune_cache_lookup(path, k1[:-1]) is None
    # replacing an entry keeps the others, and one line per key
    svdag.svd_tune_cache_store(path, k1, 32, 1, 4, 0.4)
    assert svdag.svd_tune_cache_lookup(path, k1).tile_w == 32
    assert svdag.svd_tune_cache_lookup(path, k2).tile_w == 8
    lines = open(path).read().splitlines()
    assert lines[0].startswith("#") and len(lines) == 3
    assert lines[-1] == k1 + "\t32 1 4 0.4000"
    # hand-written and malformed lines are kept and skipped
    with open(path, "a") as f:
        f.write("garbage line\n" + k2 + "\tnot numbers\n")
    assert svdag.svd_tune_cache_lookup(path, k2).tile_w == 8
    svdag.svd_tune_cache_store(path, k1, 64, 1, 2)
    assert "garbage line" in open(path).read()
    # bad entries are refused and leave the file alone
    before = open(path).read()
    for bad in ((k1, 12, 1, 6), (k1, 16, 0, 6), (k1, 16, 17, 6), (k1, 16, 1, 0), ("a\tb", 16, 1, 6),
                ("", 16, 1, 6)):
        with pytest.raises(svdag.SvdError) as e:
            svdag.svd_tune_cache_store(path, *bad)
        assert e.value.code == svdag.SVD_EINVAL
    assert open(path).read() == before
    # a directory that does not exist cannot be written
    with pytest.raises(svdag.SvdError) as e:
        svdag.svd_tune_cache_store(str(tmp_path / "no" / "tune.txt"), k1, 16, 1, 6)
    assert e.value.code == svdag.SVD_EIO
    assert not [p for p in os.listdir(tmp_path) if ".tmp." in p]


def test_plain_c_caller(tmp_path):
    """The boundary is a C ABI: a C99 program (pedantic, warnings as errors)
    includes svdag.h, links libsvdag.so and uses entry points that need no
    GPU (the kernel hash, the tuning cache, the camera frame, an error
    message)."""
    import shutil
    import subprocess
    svdag = _svdag()
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    src = tmp_path / "caller.c"
    src.write_text(r'''
#include <stdio.h>
#include <string.h>
#include "svdag.h"
int main(int argc, char** argv) {
  (void)argc;
  svd_tune_result r;
  memset(&r, 0, sizeof(r));
  strcpy(r.key, "dev=test kind=view");
  r.tile_w = 8; r.claim = 1; r.blocks_per_cu = 5; r.ms = 0.25f;
  if (svd_tune_cache_store(argv[1], &r) != SVD_OK) return 1;
  svd_tune_result back;
  if (svd_tune_cache_lookup(argv[1], "dev=test kind=view", &back) != SVD_OK) return 2;
  if (back.tile_w != 8 || back.blocks_per_cu != 5 || !back.from_cache) return 3;
  if (svd_tune_cache_lookup(argv[1], "dev=other", &back) != SVD_ENOTFOUND) return 4;
  svd_camera cam = {{100.0f, 100.0f, 50.0f}, {200.0f, 150.0f, 20.0f}, {0.0f, 0.0f, 1.0f}, 60.0f, 64, 32};
  svd_ray_frame f;
  if (svd_camera_frame(&cam, &f) != SVD_OK || f.width != 64) return 5;
  cam.vfov_deg = 0.0f;
  if (svd_camera_frame(&cam, &f) == SVD_OK || strlen(svd_last_error()) == 0) return 6;
  printf("%s\n", svd_kernel_hash());
  return 0;
}
''')
    exe = tmp_path / "caller"
    libdir = os.path.dirname(svdag.LIB_PATH)
    r = subprocess.run(["gcc", "-std=c99", "-pedantic", "-Wall", "-Wextra", "-Werror", f"-I{ROOT}/include",
                        str(src), "-o", str(exe), f"-L{libdir}", "-lsvdag", f"-Wl,-rpath,{libdir}"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe), str(tmp_path / "tune.txt")], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, (r.returncode, r.stderr)
    from paper_2505_02017_amd import build
    assert r.stdout.strip() == build.kernel_source_hash()
