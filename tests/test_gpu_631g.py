"""6-31G (H, C, N, O) on the HIP path against the FP64 oracle, through the
C ABI: the six-primitive core shell, the 3 + 1 split valence and the padded
36-entry primitive-pair tables.

Tolerances as for STO-3G: FP64 one-electron integrals and ERIs 1e-12
absolute, J/K 1e-11, V_xc and E_xc 1e-10, SCF |dE|, |d gap| <= 1e-8 Ha with
iterations within 1; mixed SCF |dE|, |d gap| <= 1e-4 Ha.
"""
import concurrent.futures as cf

import numpy as np
import pytest

from oracle import oracle as O
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


def _mols():
    # water; CH4-like, C-N, N-O-C and N-O-C-C trees (seed 13): every 6-31G
    # element, shells of every primitive count, several sizes in one batch
    out = [molgen.water(0)]
    for n, idx in ((1, 0), (2, 4), (3, 5), (4, 5)):
        z, x, k = molgen.tree_without(n, 13, idx)
        assert k == 0
        out.append((z, x))
    return out


def _rand_density(o, seed):
    rng = np.random.default_rng(seed)
    S, _, _ = o.int1e()
    w, U = np.linalg.eigh(S)
    X = U @ np.diag(w ** -0.5) @ U.T
    Q, _ = np.linalg.qr(rng.standard_normal((o.nbf, o.nbf)))
    C = X @ Q[:, :o.nocc]
    return 2 * C @ C.T


@pytest.fixture(scope="module")
def small(ks):
    mols = _mols()
    orc = [O.Mol(z, x, basis=O.BASIS_631G) for z, x in mols]
    b = ks.Batch(mols, basis=ks.KS_BASIS_631G)
    b.setup()
    b.eri_build()
    yield mols, orc, b
    b.close()


def test_sizes_and_integrals(small):
    mols, orc, b = small
    for m, o in enumerate(orc):
        assert b.nbf[m] == o.nbf == molgen.nbf_631g(mols[m][0]) and b.nocc[m] == o.nocc
        S, T, V = o.int1e()
        for name, ref in (("S", S), ("T", T), ("V", V)):
            assert np.abs(b.matrix(m, name) - ref).max() < 1e-12, (m, name)
        assert np.abs(b.eri(m) - o.eri()).max() < 1e-12, m


def test_jk_xc(small):
    mols, orc, b = small
    Ps = [_rand_density(o, 40 + m) for m, o in enumerate(orc)]
    P = b.pack(Ps)
    J, K, V = b.empty(), b.empty(), b.empty()
    b.jk_build(P, J, K)
    exc = b.xc_build(P, V)
    Js, Ks, Vs = b.unpack(J), b.unpack(K), b.unpack(V)
    for m, o in enumerate(orc):
        Jr, Kr = o.jk(o.eri(), Ps[m])
        er, Vr = o.xc(O.XC_B3LYP, o.grid(), Ps[m])
        assert np.abs(Js[m] - Jr).max() < 1e-11, m
        assert np.abs(Ks[m] - Kr).max() < 1e-11, m
        assert abs(exc[m] - er) < 1e-10, (m, exc[m], er)
        assert np.abs(Vs[m] - Vr).max() < 1e-10, m


def _oracle_scf(args):
    z, x = args
    return O.Mol(z, x, basis=O.BASIS_631G).scf(xc=O.XC_B3LYP)


@pytest.fixture(scope="module")
def refs():
    mols = _mols()
    with cf.ThreadPoolExecutor(len(mols)) as ex:
        return list(ex.map(_oracle_scf, mols))


@pytest.mark.parametrize("prec", [0, 1])
def test_scf_vs_oracle(ks, refs, prec):
    mols = _mols()
    tol = 1e-8 if prec == 0 else 1e-4
    with ks.Batch(mols, prec=prec, basis=ks.KS_BASIS_631G) as b:
        b.scf_solve()
        for m, ref in enumerate(refs):
            r = b.result(m)
            assert r["status"] == 1 and ref["status"] == 1
            assert abs(r["E"] - ref["E"]) <= tol, (m, r["E"], ref["E"])
            assert abs(r["gap"] - ref["gap"]) <= tol, (m, r["gap"], ref["gap"])
            if prec == 0:
                assert abs(r["n_iter"] - ref["n_iter"]) <= 1
                assert np.abs(r["P"] - ref["P"]).max() <= 1e-6


def test_direct_631g(ks, refs):
    # integral-direct FP64 over the padded primitive-pair tables
    mols = _mols()
    with ks.Batch(mols, basis=ks.KS_BASIS_631G, direct=1) as b:
        b.scf_solve()
        for m, ref in enumerate(refs):
            r = b.result(m)
            assert r["status"] == 1 and abs(r["E"] - ref["E"]) <= 1e-8, (m, r["E"], ref["E"])


def test_631g_rejects_fluorine(ks):
    with pytest.raises(ks.KsError):
        ks.Batch([(np.array([9, 1]), np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.92]]))], basis=ks.KS_BASIS_631G)


def test_631g_server_equals_batch(ks):
    # the continuous-batching server with the 6-31G basis: each result equals
    # the molecule solved alone in a batch (FP64, same kernels)
    mols = _mols()
    alone = []
    for z, x in mols:
        with ks.Batch([(z, x)], basis=ks.KS_BASIS_631G, jk_chunks=8, xc_chunks=16) as b:
            b.scf_solve()
            alone.append(b.result(0))
    with ks.Server(max_batch=2, basis=ks.KS_BASIS_631G) as s:
        tickets = [s.submit(z, x) for z, x in mols]
        for _ in range(400):
            s.progress()
            if s.stats()["done"] == len(mols):
                break
        served = [s.poll(t) for t in tickets]
    for a, r in zip(alone, served):
        assert r is not None
        assert abs(r["E"] - a["E"]) <= 1e-10 and abs(r["gap"] - a["gap"]) <= 1e-10


def test_631g_graphs(ks, refs):
    # graph-replayed iterations with the 36-entry pair tables
    mols = _mols()
    s = torch.cuda.Stream()
    with ks.Batch(mols, basis=ks.KS_BASIS_631G, graphs=1, stream=s.cuda_stream) as b:
        b.scf_solve()
        for m, ref in enumerate(refs):
            r = b.result(m)
            assert r["status"] == 1 and abs(r["E"] - ref["E"]) <= 1e-8, (m, r["E"], ref["E"])
