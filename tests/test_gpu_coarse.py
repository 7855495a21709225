"""SCF started on a coarse grid (options coarse_rad/theta/phi): molecules
move to the main grid once |dE| < 1e-4 Ha and the commutator < 1e-3 on the
coarse one, and convergence is only tested on the main grid, so the results
are those of the main grid.

- FP64: the first 8 molecules of the 9-11-heavy-atom benchmark set (seed 2)
  against their stored oracle SCF results (tests/golden, written by
  make_golden_subset.py): |dE| <= 1e-8 Ha and max|dP| <= 1e-6 (molecules
  0-2, make_golden_density.py).  The gap is held to 1e-6 Ha here, not the
  1e-8 of a run without the coarse start: with it the iterates differ from
  the oracle's, so the two runs stop at different points inside the
  stopping rule (commutator max-norm < 1e-7), and orbital energies, unlike
  the energy, move to first order with that residual.  The fixed point
  itself is the oracle's: converged tightly (dE < 1e-12 Ha, commutator
  < 1e-10) on both sides, E and the gap agree to 1e-8 Ha and P to 1e-6.
  Against the same batch without the coarse start, max|dP| <= 1e-6.
- Mixed path, same molecules, stored and integral-direct J/K: |dE|,
  |d gap| <= 1e-4 Ha against the oracle.
- Iteration accounting: 1 <= coarse iterations <= 12, at least two
  main-grid iterations after them.
- Direct xc_build calls use the main grid whatever the SCF stage.
- Graph-replayed iterations (the stage switch happens inside the replays)
  equal plain launches.
- The bulk getter (ks_get_results) returns exactly what the per-molecule
  getters return.
"""
import json
import os

import numpy as np
import pytest

from paper_2311_01135_amd import molgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_scf_seed2_first64.json")
DENS = os.path.join(os.path.dirname(__file__), "golden", "oracle_density_seed2")
COARSE = dict(coarse_rad=25, coarse_theta=8, coarse_phi=16)
NMOL = 8


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_01135_amd import ks as K
    K.load()
    return K


@pytest.fixture(scope="module")
def mols_gold():
    with open(GOLD) as f:
        gold = {m["index"]: m for m in json.load(f)["molecules"]}
    return molgen.batch(NMOL, 2, (9, 11)), [gold[i] for i in range(NMOL)]


def _solve(ks, mols, **kw):
    with ks.Batch(mols, **kw) as b:
        b.scf_solve()
        return [b.result(m) for m in range(len(mols))], [b.iterations(m) for m in range(len(mols))]


@pytest.mark.parametrize("prec,direct", [(0, 0), (1, 0), (1, 1)])
def test_coarse_start_matches_oracle(ks, mols_gold, prec, direct):
    mols, gold = mols_gold
    tol_e, tol_g = (1e-8, 1e-6) if prec == 0 else (1e-4, 1e-4)
    print("coarse start, prec %d, direct %d, %d molecules" % (prec, direct, len(mols)), flush=True)
    res, its = _solve(ks, mols, prec=prec, direct=direct, **COARSE)
    for m, (r, g, (n, nc)) in enumerate(zip(res, gold, its)):
        assert r["status"] == 1, m
        assert abs(r["E"] - g["E"]) <= tol_e, (m, r["E"], g["E"])
        assert abs(r["gap"] - g["gap"]) <= tol_g, (m, r["gap"], g["gap"])
        assert 1 <= nc <= 12 and n >= nc + 2, (m, n, nc)
        assert r["n_iter"] == n
    if prec == 0:
        dens = np.load(DENS + ".npz")
        for m in range(3):
            dP = np.abs(res[m]["P"] - dens["P_default_%d" % m]).max()
            print("molecule %d: max|dP| vs oracle %.2e" % (m, dP), flush=True)
            assert dP <= 1e-6, (m, dP)
        ref, its0 = _solve(ks, mols, prec=prec)
        for m in range(len(mols)):
            assert its0[m][1] == 0
            assert np.abs(res[m]["P"] - ref[m]["P"]).max() <= 1e-6, m
            assert abs(res[m]["E"] - ref[m]["E"]) <= 1e-8, m


def test_coarse_start_tight_fixed_point(ks, mols_gold):
    """Both sides converged to dE < 1e-12 Ha and commutator < 1e-10: the
    coarse-start FP64 path reaches the oracle's fixed point (E and gap to
    1e-8 Ha, P to 1e-6)."""
    mols, _ = mols_gold
    with open(DENS + ".json") as f:
        tight = {t["index"]: t for t in json.load(f)["tight"]}
    dens = np.load(DENS + ".npz")
    res, its = _solve(ks, mols, prec=0, e_tol=1e-12, comm_tol=1e-10, max_iter=200, **COARSE)
    for m, r in enumerate(res):
        g = tight[m]
        assert r["status"] == 1 and g["status"] == 1, m
        print("molecule %d: tight |dE| %.2e |dgap| %.2e, %d iterations (%d coarse), oracle %d"
              % (m, abs(r["E"] - g["E"]), abs(r["gap"] - g["gap"]), its[m][0], its[m][1], g["n_iter"]), flush=True)
        assert abs(r["E"] - g["E"]) <= 1e-8, (m, r["E"], g["E"])
        assert abs(r["gap"] - g["gap"]) <= 1e-8, (m, r["gap"], g["gap"])
        if m < 3:
            assert np.abs(r["P"] - dens["P_tight_%d" % m]).max() <= 1e-6, m


def test_xc_build_uses_main_grid(ks, mols_gold):
    mols, _ = mols_gold
    mols = mols[:3]
    out = []
    for kw in ({}, COARSE):
        with ks.Batch(mols, prec=0, **kw) as b:
            b.setup()                        # P holds the initial guess, the same in both batches
            P = b.pack([b.matrix(m, "P") for m in range(len(mols))])
            V = b.empty()
            e = b.xc_build(P, V)
            out.append((np.asarray(e), b.unpack(V)))
    (e0, V0), (e1, V1) = out
    assert np.abs(e0 - e1).max() <= 1e-12
    for a, c in zip(V0, V1):
        assert np.abs(a - c).max() <= 1e-12


@pytest.mark.parametrize("prec", [0, 1])
def test_coarse_start_graph_replay(ks, mols_gold, prec):
    mols, _ = mols_gold
    mols = mols[:4]
    tol = 1e-9 if prec == 0 else 1e-6
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    with ks.Batch(mols, prec=prec, graphs=1, stream=s1.cuda_stream, **COARSE) as bg, \
            ks.Batch(mols, prec=prec, graphs=0, stream=s2.cuda_stream, **COARSE) as bp:
        steps = 0
        while True:
            ng = bg.scf_step()
            torch.cuda.synchronize()
            npl = bp.scf_step()
            steps += 1
            assert ng == npl, (steps, ng, npl)
            for m in range(len(mols)):
                assert bg.iterations(m) == bp.iterations(m), (steps, m)
                assert abs(bg.convergence(m)[0] - bp.convergence(m)[0]) <= tol, (steps, m)
            if ng == 0:
                break
            assert steps < 60
        for m in range(len(mols)):
            rg, rp = bg.result(m), bp.result(m)
            assert rg["status"] == rp["status"] == 1
            assert abs(rg["E"] - rp["E"]) <= tol and bg.iterations(m)[1] >= 1


def test_bulk_results_equal_per_molecule(ks, mols_gold):
    mols, _ = mols_gold
    mols = mols[:5] + [molgen.water(0)]
    with ks.Batch(mols, prec=1, **COARSE) as b:
        b.scf_solve()
        bulk = b.results()
        for m in range(len(mols)):
            r, q = b.result(m), bulk[m]
            for k in ("E", "homo", "lumo", "gap", "status", "n_iter"):
                assert r[k] == q[k], (m, k)
            assert np.array_equal(r["eps"], q["eps"]) and np.array_equal(r["P"], q["P"])
            assert b.iterations(m) == (q["n_iter"], q["n_coarse"])
