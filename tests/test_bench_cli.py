"""bench.py's command line on the CPU: it refuses more than one GPU and bad
serving options before touching a device, and its integer cube root (used
to report alpha = y / icbrt(x)) is exact."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bad_serving_options_are_refused():
    r = run("--serve-modes", "fast")
    assert r.returncode != 0 and "--serve-modes" in r.stderr
    r = run("--x", str(2**72 + 1))
    assert r.returncode != 0 and "--x" in r.stderr


def test_icbrt():
    sys.path.insert(0, ROOT)
    import bench
    for n in (1, 7, 8, 26, 27, 10**18 - 1, 10**18, 2**63 + 2**61, 2**64 - 1):
        r = bench.icbrt(n)
        assert r**3 <= n < (r + 1)**3, n
