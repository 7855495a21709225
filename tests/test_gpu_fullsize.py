"""Full-size parity: the benchmark's own batch (4096 molecules, 9-11 heavy
atoms, seed 2) in the launch configuration bench.py times, compared with
oracle SCF results for its first 64 molecules (written by
tests/golden/make_golden_subset.py) and two later samples (written by
tests/golden/make_golden.py), plus properties that hold for every molecule;
and full-grid kernel parity for one 9-heavy-atom molecule.

Tolerances: FP64 |dE|, |d gap| <= 1e-8 Ha, iterations within 1 and, for
molecules 0-2 (oracle densities written by make_golden_density.py),
max|dP| <= 1e-6; mixed
|dE|, |d gap| <= 1e-4 Ha; tr(PS) = N_e to 1e-8 (FP64) / 1e-6 (mixed).
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_01135_amd import autotune, molgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
GOLD = os.path.join(GOLDEN, "oracle_scf_samples.json")
SUBSET = os.path.join(GOLDEN, "oracle_scf_seed2_first64.json")
N_BENCH = 4096


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_01135_amd import ks as K
    K.load()
    return K


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def bench_refs(gold):
    with open(SUBSET) as f:
        sub = json.load(f)["molecules"]
    seen = {g["index"] for g in sub}
    extra = [g for g in gold["molecules"] if g["set"] == "bench_9-11_seed2" and g["index"] not in seen]
    return sub + extra


@pytest.fixture(scope="module")
def bench_mols():
    return molgen.batch(N_BENCH, 2, (9, 11))


@pytest.mark.parametrize("prec", [1, 0])
def test_bench_batch_vs_oracle_samples(ks, bench_refs, bench_mols, prec):
    tol = 1e-4 if prec == 1 else 1e-8
    opts = autotune.tuned_options(prec, [molgen.nbf_sto3g(z) for z, _ in bench_mols])
    print("batch %d molecules, prec %d, options %s" % (len(bench_mols), prec, opts), flush=True)
    assert len(bench_refs) >= 64
    with ks.Batch(bench_mols, prec=prec, **opts) as b:
        b.scf_solve()
        for g in bench_refs:
            r = b.result(g["index"])
            assert r["status"] == 1
            assert abs(r["E"] - g["E"]) <= tol, (g["index"], r["E"], g["E"])
            assert abs(r["gap"] - g["gap"]) <= tol, (g["index"], r["gap"], g["gap"])
            if prec == 0:
                assert abs(r["n_iter"] - g["n_iter"]) <= 1
        if prec == 0:
            # full-size densities (FP64: max|dP| <= 1e-6)
            dens = np.load(os.path.join(GOLDEN, "oracle_density_seed2.npz"))
            for m in range(3):
                dP = np.abs(b.result(m)["P"] - dens["P_default_%d" % m]).max()
                print("molecule %d: max|dP| vs oracle %.2e" % (m, dP), flush=True)
                assert dP <= 1e-6, (m, dP)
        # properties of every molecule of the batch
        trtol = 1e-6 if prec == 1 else 1e-8
        for m in range(b.n_mol):
            r = b.result(m)
            assert r["status"] == 1, m
            S = b.matrix(m, "S")
            P = r["P"]
            ne = 2 * b.nocc[m]
            assert abs(np.sum(P * S) - ne) <= trtol * ne, m
            assert np.abs(P - P.T).max() <= 1e-12
            assert r["gap"] > 0 and r["homo"] < r["lumo"]


def test_c1_molecules_fp64(ks, gold):
    mols = [g for g in gold["molecules"] if g["set"] == "c1_9_seed1"]
    geo = [molgen.batch(1, 1, 9, start=g["index"])[0] for g in mols]
    with ks.Batch(geo) as b:
        b.scf_solve()
        for m, g in enumerate(mols):
            r = b.result(m)
            assert r["status"] == 1
            assert abs(r["E"] - g["E"]) <= 1e-8 and abs(r["gap"] - g["gap"]) <= 1e-8


def test_water_fp64(ks, gold):
    with ks.Batch([molgen.water(0)]) as b:
        b.scf_solve()
        r = b.result(0)
    w = gold["water_seed0"]
    assert abs(r["E"] - w["E"]) <= 1e-8 and abs(r["gap"] - w["gap"]) <= 1e-8 and r["n_iter"] == w["n_iter"]


@pytest.fixture(scope="module")
def big(ks):
    z, x = molgen.tree(9, 1, 0)
    o = O.Mol(z, x)
    b = ks.Batch([(z, x)])
    b.setup()
    b.eri_build()
    yield o, b
    b.close()


def _density(o, seed):
    rng = np.random.default_rng(seed)
    S, _, _ = o.int1e()
    w, U = np.linalg.eigh(S)
    X = U @ np.diag(w ** -0.5) @ U.T
    Q, _ = np.linalg.qr(rng.standard_normal((o.nbf, o.nbf)))
    C = X @ Q[:, :o.nocc]
    return 2 * C @ C.T


def test_fullsize_grid(big):
    o, b = big
    ref = o.grid()
    got = b.grid(0)
    assert np.abs(got[:, :3] - ref[:, :3]).max() < 1e-12
    assert np.abs(got[:, 3] - ref[:, 3]).max() <= 1e-12 * np.abs(ref[:, 3]).max()


def test_fullsize_jk_xc(big):
    o, b = big
    P = _density(o, 3)
    Pt = b.pack([P])
    J, K, V = b.empty(), b.empty(), b.empty()
    b.jk_build(Pt, J, K)
    exc = b.xc_build(Pt, V)
    Jr, Kr = o.jk(o.eri(), P)
    er, Vr = o.xc(O.XC_B3LYP, o.grid(), P)
    assert np.abs(b.unpack(J)[0] - Jr).max() < 1e-10
    assert np.abs(b.unpack(K)[0] - Kr).max() < 1e-10
    assert abs(exc[0] - er) < 1e-9
    assert np.abs(b.unpack(V)[0] - Vr).max() < 1e-10
