"""Host-side pieces of bench.py: the one-GPU contract and the byte model of
the roofline (no GPU needed)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_unknown_other_workload_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--other-workloads", "terrain1024,nope"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "unknown workload 'nope'" in r.stderr and r.stdout == ""


def _counts_and_hits():
    cnt = np.zeros(3, dtype=[("chunk_visits", np.int32), ("chunk_entries", np.int32),
                             ("node_cubes", np.int32), ("leaf_cubes", np.int32),
                             ("preceding_siblings", np.int32), ("run_probes", np.int32)])
    cnt["chunk_visits"] = [1, 3, 2]
    cnt["chunk_entries"] = [0, 2, 1]
    cnt["node_cubes"] = [0, 10, 4]
    cnt["leaf_cubes"] = [0, 3, 1]
    cnt["preceding_siblings"] = [0, 9, 2]
    cnt["run_probes"] = [0, 10, 3]
    hits = np.zeros(3, dtype=[("hit", np.int32), ("lod", np.int32), ("chunk", np.int32)])
    hits["hit"] = [0, 1, 1]
    hits["lod"] = [0, 0, 2]
    hits["chunk"] = [0, 1, 1]
    return cnt, hits


def test_bytes_per_ray_model():
    """The paper-format model: 8 B per internal node descended (root
    included), 8 B per leaf bitmap, at a hit 4 B per preceding-sibling count,
    4 B per run probe and 1 B material, and the 16-B record."""
    import bench
    cnt, hits = _counts_and_hits()
    b = bench.bytes_per_ray(cnt, hits)
    assert b[0] == 16                                   # a miss that entered no DAG
    assert b[1] == 8 * (2 + 10) + 8 * 3 + 4 * 9 + 4 * 10 + 1 + 16
    assert b[2] == 8 * (1 + 4) + 8 * 1 + 4 * 2 + 4 * 3 + 1 + 16


def test_layout_bytes_per_ray_model():
    import bench
    cnt, hits = _counts_and_hits()
    cl = 9
    b = bench.layout_bytes_per_ray(cnt, hits, cl)
    # a miss: one view word and the record
    assert b[0] == 4 + 16
    # hit at LOD 0 after 10 run probes, 7 prefix levels
    assert b[1] == 4 * 3 + 20 * 2 + 4 * 10 + 12 * 3 + 16 + 28 + 4 * (cl - 0 - 2) + 4 * 10 + 1
    # hit at LOD 2 after 3 run probes, 5 prefix levels
    assert b[2] == 4 * 2 + 20 * 1 + 4 * 4 + 12 * 1 + 16 + 28 + 4 * (cl - 2 - 2) + 4 * 3 + 1
    s = bench.layout_bytes_per_ray(cnt, hits, cl, sector=64)
    # every read a whole sector (two for a leaf: word and bitmap); the record stays 16 B
    assert s[0] == 64 + 16
    assert s[1] == 64 * (3 + 2 + 10 + 2 * 3) + 16 + 64 * (1 + (cl - 2) + 10 + 1)


def test_host_cores_reports_the_usable_cpus():
    import bench
    cores, nproc, limit = bench.host_cores()
    assert 1 <= cores <= nproc
    assert nproc == len(os.sched_getaffinity(0))
    if limit is None:
        assert cores == nproc


def test_tune_cache_path(tmp_path):
    """The bench's tuning cache: its directory is created; 'none' turns it
    off; a directory that cannot be created turns it off instead of failing
    the run."""
    import types
    import bench
    p = tmp_path / "a" / "b" / "tune.txt"
    assert bench.tune_cache_path(types.SimpleNamespace(tune_cache=str(p))) == str(p)
    assert p.parent.is_dir()
    assert bench.tune_cache_path(types.SimpleNamespace(tune_cache="none")) is None
    assert bench.tune_cache_path(types.SimpleNamespace(tune_cache="/proc/no-such-dir/tune.txt")) is None
