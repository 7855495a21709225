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


def test_screened_flops_scale_each_grid():
    nbf, ngrid, niter = [10, 20], [1000, 3000], [5, 7]
    got = bench.xc_flops(nbf, ngrid, niter, [200, 600], [2, 3], 0.5, 0.25)
    assert got == 4.0 * (100 * (0.5 * 1000 * 3 + 0.25 * 200 * 2) + 400 * (0.5 * 3000 * 4 + 0.25 * 600 * 3))


def test_parallel_generation_equals_serial():
    from paper_2311_01135_amd import molgen
    got = bench.gen_batch(40, 5, (3, 6), workers=3)
    ref = molgen.batch(40, 5, (3, 6))
    assert len(got) == len(ref)
    for (z1, x1), (z2, x2) in zip(got, ref):
        assert list(z1) == list(z2) and (x1 == x2).all()


def test_screening_ratios_committed():
    import argparse
    a = argparse.Namespace(seed=2, heavy="9-11", basis="sto-3g", grid="50,12,24", coarse_grid="25,8,16")
    r = bench.screened_ratio(a)
    assert r is not None and 0.3 < r["main"] < 1.0 and 0.3 < r["coarse"] < 1.0
    a.seed = 3
    assert bench.screened_ratio(a) is None
