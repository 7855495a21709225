"""Molecules at the size limits: 82 basis functions in FP64 (the largest the
LDS-resident kernels take) and 224 in the mixed path (global-memory J/K,
L2-resident density in XC, global-memory eigensolver), plus a ragged
223-function 6-31G molecule.

The SCF checks rest on size consistency of the restricted KS energy
(section 2): fragments with stored or live oracle results are placed
100 angstrom apart, so the energy of the assembly is the sum of fragment
energies and its HOMO (LUMO) is the highest (lowest) fragment HOMO (LUMO),
up to the fragments' multipole interactions.  The oracle's own SCF of the
82-function assembly differs from its fragment sum by 4.7e-8 Ha in the
energy and 2e-7 Ha in HOMO and LUMO.  Tolerances: FP64 energy 1e-6 Ha and
orbital energies 1e-5 Ha; mixed path energy 2e-4 Ha (twice the
per-fragment 1e-4) and orbital energies 1e-4 Ha.

The J/K checks sample elements against sums over oracle integrals taken
one by one (oracle eri_one) for a random density: integral-direct J/K
(FP64 integrals) to 1e-9; stored mixed J/K (FP32 integrals, each rounded
to 2^-24 relative) to 2^-21 sum |P_kl (ij|kl)|, a worst-case bound on
rounding the integrals and the FP32 sum.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_01135_amd import molgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(__file__)
SEP = 100.0                                 # angstrom between fragment centroids


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_01135_amd import ks as K
    K.load()
    return K


def _gold(name):
    with open(os.path.join(HERE, "golden", name)) as f:
        return {m["index"]: m for m in json.load(f)["molecules"]}


def _assemble(frags):
    """Fragments on a line, centroids SEP apart and centred on the origin."""
    zs, xs = [], []
    for k, (z, x) in enumerate(frags):
        x = np.asarray(x, dtype=float)
        shift = np.array([(k - (len(frags) - 1) / 2) * SEP, 0.0, 0.0])
        zs.append(np.asarray(z))
        xs.append(x - x.mean(axis=0) + shift)
    return np.concatenate(zs), np.concatenate(xs)


def _small_fragments():
    """Water and methane with their live oracle SCF results."""
    out = []
    for z, x in (molgen.water(0), molgen.tree(1, 0, 0)):
        r = O.Mol(z, x).scf(xc=O.XC_B3LYP)
        assert r["status"] == 1
        out.append(((z, x), dict(E=r["E"], homo=r["homo"], lumo=r["lumo"])))
    return out


def _check_additive(res, refs, e_tol, orb_tol):
    E = sum(r["E"] for r in refs)
    homo = max(r["homo"] for r in refs)
    lumo = min(r["lumo"] for r in refs)
    assert res["status"] == 1
    assert abs(res["E"] - E) <= e_tol, (res["E"], E)
    assert abs(res["homo"] - homo) <= orb_tol, (res["homo"], homo)
    assert abs(res["lumo"] - lumo) <= orb_tol, (res["lumo"], lumo)
    assert abs(res["gap"] - (lumo - homo)) <= 2 * orb_tol


def _rand_density(N, nocc, seed, S):
    rng = np.random.default_rng(seed)
    w, U = np.linalg.eigh(S)
    X = U @ np.diag(w ** -0.5) @ U.T
    Q, _ = np.linalg.qr(rng.standard_normal((N, N)))
    C = X @ Q[:, :nocc]
    return 2 * C @ C.T


def _jk_samples(o, P, elems):
    """J_ij, K_ij and sum |P_kl (ij|kl)|, sum |P_kl (ik|jl)| from single oracle integrals."""
    N = o.nbf
    out = []
    for i, j in elems:
        J = K = aJ = aK = 0.0
        for k in range(N):
            for l in range(N):
                g = o.eri_one(i, j, k, l)
                h = o.eri_one(i, k, j, l)
                J += P[k, l] * g
                K += P[k, l] * h
                aJ += abs(P[k, l] * g)
                aK += abs(P[k, l] * h)
        out.append((J, K, aJ, aK))
    return out


def test_fp64_at_82_functions(ks):
    # a 66-function molecule of the 9-11-heavy-atom set + water + methane
    sub = _gold("oracle_scf_seed2_first64.json")[37]
    frags = [molgen.batch(1, 2, (9, 11), start=37)[0]]
    refs = [sub]
    for mol, r in _small_fragments():
        frags.append(mol)
        refs.append(r)
    z, x = _assemble(frags)
    print("FP64 limit: %d atoms" % len(z), flush=True)
    with ks.Batch([(z, x)], prec=ks.KS_FP64) as b:
        assert b.nbf[0] == 82
        b.scf_solve()
        _check_additive(b.result(0), refs, 1e-6, 1e-5)


@pytest.fixture(scope="module")
def limit_mol():
    # 130 + 78 + 7 + 9 = 224 functions
    big = _gold("oracle_scf_large.json")[0]
    sub = _gold("oracle_scf_seed2_first64.json")[42]
    frags = [molgen.tree(20, 4, 0), molgen.batch(1, 2, (9, 11), start=42)[0]]
    refs = [big, sub]
    for mol, r in _small_fragments():
        frags.append(mol)
        refs.append(r)
    return _assemble(frags), refs


@pytest.mark.parametrize("direct", [0, 1])
def test_mixed_at_224_functions_scf(ks, limit_mol, direct):
    (z, x), refs = limit_mol
    print("mixed limit SCF, direct=%d, %d atoms" % (direct, len(z)), flush=True)
    with ks.Batch([(z, x)], prec=ks.KS_MIXED, direct=direct) as b:
        assert b.nbf[0] == 224
        b.scf_solve()
        _check_additive(b.result(0), refs, 2e-4, 1e-4)


def test_mixed_at_224_functions_jk(ks, limit_mol):
    (z, x), _ = limit_mol
    o = O.Mol(z, x)
    N = o.nbf
    assert N == 224
    S, _, _ = o.int1e()
    P = _rand_density(N, o.nocc, 90, S)
    # corners, the ragged tail, a cross-fragment pair and the middle
    elems = [(0, 0), (223, 223), (223, 0), (200, 131), (100, 37)]
    ref = _jk_samples(o, P, elems)
    got = {}
    for direct in (0, 1):
        print("mixed limit J/K, direct=%d" % direct, flush=True)
        with ks.Batch([(z, x)], prec=ks.KS_MIXED, direct=direct, schwarz_tol=1e-14) as b:
            b.setup()
            b.eri_build()
            Pd = b.pack([P])
            J, K = b.empty(), b.empty()
            b.jk_build(Pd, J, K)
            got[direct] = (b.unpack(J)[0], b.unpack(K)[0])
    for (i, j), (Jr, Kr, aJ, aK) in zip(elems, ref):
        Jd, Kd = got[1]
        assert abs(Jd[i, j] - Jr) < 1e-9 and abs(Kd[i, j] - Kr) < 1e-9, (i, j)
        Js, Ks = got[0]
        assert abs(Js[i, j] - Jr) <= 2.0 ** -21 * aJ + 1e-12, (i, j, Js[i, j] - Jr, aJ)
        assert abs(Ks[i, j] - Kr) <= 2.0 ** -21 * aK + 1e-12, (i, j, Ks[i, j] - Kr, aK)
    for Jm, Km in got.values():
        assert np.abs(Jm - Jm.T).max() < 1e-12 and np.abs(Km - Km.T).max() < 1e-12


def test_631g_ragged_223_functions_jk(ks):
    z, x = molgen.tree(19, 4, 1)
    o = O.Mol(z, x, basis=O.BASIS_631G)
    N = o.nbf
    assert N == 223
    S, _, _ = o.int1e()
    P = _rand_density(N, o.nocc, 91, S)
    elems = [(0, 0), (222, 222), (222, 3), (150, 77)]
    ref = _jk_samples(o, P, elems)
    print("6-31G 223 functions, direct J/K", flush=True)
    with ks.Batch([(z, x)], prec=ks.KS_MIXED, direct=1, schwarz_tol=1e-14, basis=ks.KS_BASIS_631G) as b:
        assert b.nbf[0] == N
        b.setup()
        b.eri_build()
        Pd = b.pack([P])
        J, K = b.empty(), b.empty()
        b.jk_build(Pd, J, K)
        Jd, Kd = b.unpack(J)[0], b.unpack(K)[0]
    for (i, j), (Jr, Kr, _, _) in zip(elems, ref):
        assert abs(Jd[i, j] - Jr) < 1e-9 and abs(Kd[i, j] - Kr) < 1e-9, (i, j, Jd[i, j] - Jr, Kd[i, j] - Kr)
