"""Molecules beyond the LDS-resident kernels (mixed path, N > 96 functions):
a batch that holds one 20-heavy-atom molecule (N = 130) runs every kernel in
its large-molecule mode (global-memory J/K accumulation, XC with the
density in L2 and grouped tiles, global-memory eigensolver and N x N
products).  The small molecules of the same batch are checked against the
oracle (J/K and V_XC from random densities, SCF energies), the large one
against the oracle SCF result written by tests/golden/make_golden_large.py;
the integral-direct build in the same mode against the oracle (small
molecules) and the stored build (large one).

Tolerances (mixed path): J, K, V_XC elements 1e-5; E_XC 1e-5 Ha; SCF
|dE|, |d gap| <= 1e-4 Ha.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_01135_amd import molgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_scf_large.json")


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_01135_amd import ks as K
    K.load()
    return K


def _mols():
    return [molgen.water(0), molgen.tree(3, 7, 3), molgen.tree(20, 4, 0)]


def _rand_density(o, seed):
    rng = np.random.default_rng(seed)
    S, _, _ = o.int1e()
    w, U = np.linalg.eigh(S)
    X = U @ np.diag(w ** -0.5) @ U.T
    Q, _ = np.linalg.qr(rng.standard_normal((o.nbf, o.nbf)))
    C = X @ Q[:, :o.nocc]
    return 2 * C @ C.T


@pytest.fixture(scope="module")
def batch(ks):
    mols = _mols()
    b = ks.Batch(mols, prec=ks.KS_MIXED)
    assert max(b.nbf) > 96
    b.setup()
    b.eri_build()
    yield mols, b
    b.close()


def test_large_batch_kernels_vs_oracle(batch):
    mols, b = batch
    orc = [O.Mol(z, x) for z, x in mols[:2]]
    Ps = [_rand_density(o, 50 + m) for m, o in enumerate(orc)]
    # the large molecule gets its own random density; only its shape matters here
    ol = O.Mol(*mols[2])
    Ps.append(_rand_density(ol, 52))
    P = b.pack(Ps)
    J, K, V = b.empty(), b.empty(), b.empty()
    b.jk_build(P, J, K)
    exc = b.xc_build(P, V)
    Js, Ks, Vs = b.unpack(J), b.unpack(K), b.unpack(V)
    for m, o in enumerate(orc):
        Jr, Kr = o.jk(o.eri(), Ps[m])
        er, Vr = o.xc(O.XC_B3LYP, o.grid(), Ps[m])
        assert np.abs(Js[m] - Jr).max() < 1e-5, m
        assert np.abs(Ks[m] - Kr).max() < 1e-5, m
        assert abs(exc[m] - er) < 1e-5, (m, exc[m], er)
        assert np.abs(Vs[m] - Vr).max() < 1e-5, m
    for M in (Js[2], Ks[2], Vs[2]):
        assert np.isfinite(M).all() and np.abs(M - M.T).max() < 1e-9


def test_large_batch_scf(ks):
    mols = _mols() + [molgen.tree(20, 4, 1)]
    refs = [O.Mol(z, x).scf(xc=O.XC_B3LYP) for z, x in mols[:2]]
    with open(GOLD) as f:
        gold = {x["index"]: x for x in json.load(f)["molecules"]}
    with ks.Batch(mols, prec=ks.KS_MIXED) as b:
        b.scf_solve()
        for m, ref in enumerate(refs):
            r = b.result(m)
            assert r["status"] == 1
            assert abs(r["E"] - ref["E"]) <= 1e-4 and abs(r["gap"] - ref["gap"]) <= 1e-4, m
        for m, idx in ((2, 0), (3, 1)):
            r, g = b.result(m), gold[idx]
            assert r["status"] == 1 and g["nbf"] == b.nbf[m]
            assert abs(r["E"] - g["E"]) <= 1e-4 and abs(r["gap"] - g["gap"]) <= 1e-4, (idx, r["E"], g["E"])


def test_large_batch_direct_jk(ks, batch):
    # Integral-direct J/K in the large-molecule mode (bra-major digestion with
    # per-class launches): FP64 integrals and accumulation, so with the
    # Schwarz threshold at 1e-14 the small molecules match the oracle to
    # 1e-9 and the large one the stored (FP32-integral) build to 1e-5.
    mols, bs = batch
    orc = [O.Mol(z, x) for z, x in mols[:2]]
    Ps = [_rand_density(o, 60 + m) for m, o in enumerate(orc)]
    Ps.append(_rand_density(O.Mol(*mols[2]), 62))
    with ks.Batch(mols, prec=ks.KS_MIXED, direct=1, schwarz_tol=1e-14) as b:
        assert max(b.nbf) > 96
        b.setup()
        b.eri_build()
        P = b.pack(Ps)
        J, K = b.empty(), b.empty()
        b.jk_build(P, J, K)
        Js, Ks = b.unpack(J), b.unpack(K)
    Ps_ = bs.pack(Ps)
    J0, K0 = bs.empty(), bs.empty()
    bs.jk_build(Ps_, J0, K0)
    J0s, K0s = bs.unpack(J0), bs.unpack(K0)
    for m, o in enumerate(orc):
        Jr, Kr = o.jk(o.eri(), Ps[m])
        assert np.abs(Js[m] - Jr).max() < 1e-9, m
        assert np.abs(Ks[m] - Kr).max() < 1e-9, m
    assert np.abs(Js[2] - J0s[2]).max() < 1e-5
    assert np.abs(Ks[2] - K0s[2]).max() < 1e-5
    assert np.abs(Js[2] - Js[2].T).max() < 1e-12 and np.abs(Ks[2] - Ks[2].T).max() < 1e-12


def test_large_direct_scf(ks):
    # direct mixed SCF with the default screening on a batch holding both
    # 20-heavy-atom molecules against their oracle SCF results
    mols = [molgen.water(0), molgen.tree(20, 4, 0), molgen.tree(20, 4, 1)]
    with open(GOLD) as f:
        gold = {x["index"]: x for x in json.load(f)["molecules"]}
    ref = O.Mol(*mols[0]).scf(xc=O.XC_B3LYP)
    with ks.Batch(mols, prec=ks.KS_MIXED, direct=1, schwarz_tol=1e-10) as b:
        b.scf_solve()
        r = b.result(0)
        assert r["status"] == 1 and abs(r["E"] - ref["E"]) <= 1e-4
        for m, idx in ((1, 0), (2, 1)):
            r, g = b.result(m), gold[idx]
            assert r["status"] == 1 and g["nbf"] == b.nbf[m]
            assert abs(r["E"] - g["E"]) <= 1e-4 and abs(r["gap"] - g["gap"]) <= 1e-4, (idx, r["E"], g["E"])
