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


def test_bytes_per_ray_model():
    import bench
    cnt = np.zeros(3, dtype=[("chunk_visits", np.int32), ("chunk_entries", np.int32),
                             ("node_cubes", np.int32), ("leaf_cubes", np.int32)])
    cnt["chunk_visits"] = [1, 3, 2]
    cnt["chunk_entries"] = [0, 2, 1]
    cnt["node_cubes"] = [0, 10, 4]
    cnt["leaf_cubes"] = [0, 3, 1]
    hits = np.zeros(3, dtype=[("hit", np.int32), ("lod", np.int32), ("chunk", np.int32)])
    hits["hit"] = [0, 1, 1]
    hits["lod"] = [0, 0, 2]
    hits["chunk"] = [0, 1, 1]
    n_rle = np.array([[1, 1, 1, 1], [1000, 1, 5, 1]])
    cl = 9
    b = bench.bytes_per_ray(cnt, hits, None, cl, n_rle)
    # a miss: one view word and the record
    assert b[0] == 4 + 16
    # hit at LOD 0 in a chunk of 1000 runs: 10 search steps, 7 prefix levels
    assert b[1] == 4 * 3 + 20 * 2 + 4 * 10 + 12 * 3 + 16 + 28 + 4 * (cl - 0 - 2) + 4 * 10 + 1
    # hit at LOD 2 with 5 runs: 3 search steps, 5 prefix levels
    assert b[2] == 4 * 2 + 20 * 1 + 4 * 4 + 12 * 1 + 16 + 28 + 4 * (cl - 2 - 2) + 4 * 3 + 1
    s = bench.bytes_per_ray(cnt, hits, None, cl, n_rle, sector=64)
    # every read a whole sector (two for a leaf: word and bitmap); the record stays 16 B
    assert s[0] == 64 + 16
    assert s[1] == 64 * (3 + 2 + 10 + 2 * 3) + 16 + 64 * (1 + (cl - 2) + 10 + 1)
