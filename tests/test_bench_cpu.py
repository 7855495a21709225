"""Host logic of bench.py (no GPU): the roofline flop count with and without
the coarse-grid start, and the one-GPU guard."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_xc_flops_counts_each_iteration_at_its_grid():
    nbf, ngrid, niter = [10, 20], [1000, 3000], [5, 7]
    # main grid only: 4 G N^2 per iteration
    assert bench.xc_flops(nbf, ngrid, niter) == 4.0 * (1000 * 100 * 5 + 3000 * 400 * 7)
    # two (three) of the iterations on a coarse grid of 200 (600) points
    got = bench.xc_flops(nbf, ngrid, niter, [200, 600], [2, 3])
    assert got == 4.0 * (100 * (1000 * 3 + 200 * 2) + 400 * (3000 * 4 + 600 * 3))
    assert bench.xc_flops(nbf, ngrid, niter, [200, 600], [0, 0]) == bench.xc_flops(nbf, ngrid, niter)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
