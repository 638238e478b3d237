"""Host-side parts of bench.py: the one-GPU refusal and the byte accounting."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_construct_bytes():
    import bench
    # n = m = 5000: m (n-1) (4n + 8)
    assert bench.construct_bytes(5000, 5000) == 5000 * 4999 * 20008


def test_sorted_walk_bytes():
    import bench
    n, m = 100, 10
    steps = m * (n - 1)
    # 64 entries per step, no fallback, over two launches
    assert bench.sorted_walk_bytes((2 * 64 * steps, 0, 0), 2, n, m) == steps * 384 + steps * 8
    # every step falls back and scans all 25 blocks after 256 entries
    got = bench.sorted_walk_bytes((256 * steps, steps, 25 * steps), 1, n, m)
    assert got == steps * (256 * 6 + 25 * 16 + 8)
