"""ks_get_eri_window (the entry point for callers that cannot allocate
device memory) against ks_get_eri on the same batch: bit-identical values,
on two calls in a row with the second smaller (a window, then a smaller
molecule's whole list read window by window), plus its argument checks."""
import ctypes as C

import numpy as np
import pytest

from paper_2311_01135_amd import molgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_01135_amd import ks as K
    K.load()
    return K


@pytest.mark.parametrize("prec", [0, 1])
def test_window_equals_get_eri(ks, prec):
    mols = molgen.batch(2, 2, (9, 11)) + [molgen.water(0)]
    with ks.Batch(mols, prec=prec) as b:
        b.eri_build()
        full0, full2 = b.eri(0), b.eri(2)
        n0 = b.n_eri[0]
        assert n0 > ks.ERI_WINDOW_MAX              # the large molecule needs several windows
        # first call: a full-size window in the middle of molecule 0's list
        lo = n0 // 3
        w = b.eri_window(0, lo, ks.ERI_WINDOW_MAX)
        assert np.array_equal(w, full0[lo:lo + ks.ERI_WINDOW_MAX])
        # second call, smaller: water's whole list (406 integrals) in one window
        w2 = b.eri_window(2, 0, b.n_eri[2])
        assert np.array_equal(w2, full2)
        # molecule 0 read back window by window, the last one ragged
        got = np.empty(n0)
        for s in range(0, n0, ks.ERI_WINDOW_MAX):
            c = min(ks.ERI_WINDOW_MAX, n0 - s)
            got[s:s + c] = b.eri_window(0, s, c)
        assert np.array_equal(got, full0)


def test_window_argument_checks(ks):
    with ks.Batch([molgen.water(0)]) as b:
        L = ks.load()
        out = np.zeros(8)
        dp = out.ctypes.data_as(C.POINTER(C.c_double))
        assert L.ks_get_eri_window(b.h, 0, 0, 8, dp) == -6          # before eri_build
        b.eri_build()
        n = b.n_eri[0]
        assert L.ks_get_eri_window(b.h, 0, 0, 8, dp) == 0
        assert L.ks_get_eri_window(b.h, 0, 0, ks.ERI_WINDOW_MAX + 1, dp) == -1
        assert L.ks_get_eri_window(b.h, 0, n - 4, 8, dp) == -1      # past the end
        assert L.ks_get_eri_window(b.h, 0, -1, 8, dp) == -1
        assert L.ks_get_eri_window(b.h, 1, 0, 8, dp) == -1          # no such molecule
        assert L.ks_get_eri_window(b.h, 0, 0, 8, None) == -1
        assert L.ks_get_eri_window(b.h, 0, n, 0, None) == 0         # empty window
