"""The C ABI library loads, exports every declared entry point, and rejects
bad input before touching the GPU (runs without a GPU)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ks.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:ks_status|void|int|const char\s*\*)\s+(\w+)\s*\(", txt, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2311_01135_amd import ks
    if not os.path.exists(ks.LIB_PATH):
        pytest.fail("libks.so is not built; run __graft_entry__.build()")
    return ks.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    from paper_2311_01135_amd import ks
    assert set(ks.EXPORTS) <= set(names)


def test_default_options(lib):
    from paper_2311_01135_amd import ks
    o = ks.default_options()
    assert o.xc == 1 and o.prec == 0 and (o.n_rad, o.n_theta, o.n_phi) == (50, 12, 24)
    assert o.e_tol == 1e-9 and o.comm_tol == 1e-7 and o.max_iter == 100 and o.diis_space == 8


def _create(lib, Z, xyz, n_atoms=None, **kw):
    from paper_2311_01135_amd import ks
    o = ks.default_options(**kw)
    Z = np.ascontiguousarray(Z, dtype=np.int32)
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1))
    na = np.array([len(Z)] if n_atoms is None else n_atoms, dtype=np.int32)
    h = C.c_void_p()
    st = lib.ks_batch_create(C.byref(o), len(na), na.ctypes.data_as(C.POINTER(C.c_int)),
                             Z.ctypes.data_as(C.POINTER(C.c_int)), xyz.ctypes.data_as(C.POINTER(C.c_double)),
                             None, None, C.byref(h))
    return st, h, lib.ks_last_error().decode()


@pytest.mark.parametrize("Z,xyz,msg", [
    ([1], [[0, 0, 0]], "electrons"),                             # odd electron count
    ([2, 2], [[0, 0, 0], [1, 0, 0]], "element"),                 # He unsupported
    ([1, 1], [[0, 0, 0], [0, 0, 0.01]], "closer"),               # coincident atoms
    ([1, 1], [[0, 0, 0], [0, 0, float("nan")]], "non-finite"),
])
def test_rejects_bad_molecules(lib, Z, xyz, msg):
    st, h, err = _create(lib, Z, xyz)
    assert st == -1 and not h.value and msg in err


def test_rejects_bad_options(lib):
    st, h, err = _create(lib, [1, 1], [[0, 0, 0], [0, 0, 0.74]], diis_space=9)
    assert st == -1 and "diis_space" in err
    st, h, err = _create(lib, [1, 1], [[0, 0, 0], [0, 0, 0.74]], prec=7)
    assert st == -1
    st, h, err = _create(lib, [1, 1], [[0, 0, 0], [0, 0, 0.74]], direct=2)
    assert st == -1 and "direct" in err
    st, h, err = _create(lib, [1, 1], [[0, 0, 0], [0, 0, 0.74]], schwarz_tol=-1.0)
    assert st == -1 and "schwarz_tol" in err
    st, h, err = _create(lib, [1, 1], [[0, 0, 0], [0, 0, 0.74]], graphs=3)
    assert st == -1 and "graphs" in err
    st, h, err = _create(lib, [1, 1], [[0, 0, 0], [0, 0, 0.74]], basis=2)
    assert st == -1 and "basis" in err
    # coarse start grid: all three counts or none, each within the main grid
    st, h, err = _create(lib, [1, 1], [[0, 0, 0], [0, 0, 0.74]], coarse_rad=25)
    assert st == -1 and "coarse grid" in err
    st, h, err = _create(lib, [1, 1], [[0, 0, 0], [0, 0, 0.74]], coarse_rad=60, coarse_theta=8, coarse_phi=16)
    assert st == -1 and "coarse grid" in err
    st, h, err = _create(lib, [1, 1], [[0, 0, 0], [0, 0, 0.74]], coarse_rad=25, coarse_theta=8, coarse_phi=-1)
    assert st == -1 and "coarse grid" in err
    # 6-31G covers H, C, N, O: fluorine is rejected before any device work
    st, h, err = _create(lib, [9, 1], [[0, 0, 0], [0, 0, 0.92]], basis=1)
    assert st == -1 and "6-31G" in err


def test_rejects_too_large_fp64(lib):
    from paper_2311_01135_amd import molgen
    z, x = molgen.tree(12, 3, 0)        # 7*12+2 = 86 > 82 basis functions in FP64
    assert molgen.nbf_sto3g(z) > 82
    st, h, err = _create(lib, z, x)
    assert st == -5 and "basis functions" in err


def test_rejects_beyond_mixed_limit(lib):
    # 45 carbon atoms on a line: 225 basis functions, one past the mixed
    # path's 224 (in 6-31G, 9 per atom: 405); molecules of exactly 224 run
    # in the GPU tests
    z = [6] * 45
    x = [[1.5 * k, 0.0, 0.0] for k in range(45)]
    st, h, err = _create(lib, z, x, prec=1)
    assert st == -5 and "225 basis functions" in err
    st, h, err = _create(lib, z, x, prec=1, basis=1)
    assert st == -5 and "405 basis functions" in err


def test_null_handle_calls(lib):
    assert lib.eri_build(None) == -1
    assert lib.scf_solve(None) == -1
    assert lib.scf_solve_many(None, 1) == -1
    arr = (C.c_void_p * 2)(None, None)
    assert lib.scf_solve_many(arr, 2) == -1
    assert lib.ks_get_results(None, None, None, None, None, None, None, None, None, None) == -1
    n, c = C.c_int(), C.c_int()
    assert lib.ks_get_iterations(None, 0, C.byref(n), C.byref(c)) == -1
    lib.ks_batch_destroy(None)


def test_server_host_paths(lib):
    """Submission validation and polling of a queued ticket need no device."""
    from paper_2311_01135_amd import ks, molgen
    with ks.Server(hbm_budget=1 << 30) as s:
        with pytest.raises(ks.KsError) as e:
            s.submit([1], [[0, 0, 0]])                          # odd electron count
        assert e.value.status == -1
        with pytest.raises(ks.KsError):
            s.submit([2, 2], [[0, 0, 0], [1, 0, 0]])            # unsupported element
        z, x = molgen.water(0)
        t0 = s.submit(z, x)
        t1 = s.submit(z, x + 0.01)
        assert (t0, t1) == (0, 1)
        assert s.poll(t0) is None                               # queued, not run
        st = s.stats()
        assert st["queued"] == 2 and st["resident"] == 0 and st["done"] == 0
        with pytest.raises(ks.KsError):
            s.poll(7)
