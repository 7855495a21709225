"""Element-wise parity of the Fock-build kernels that the benchmark times,
at full size: the first two molecules of the 9-11-heavy-atom benchmark batch
(seed 2; 71 and 65 functions) in a batch with the benchmark's tuned launch
shape, digested against the oracle's converged density (tests/golden,
written by make_golden_density.py), compared with the oracle's J, K, V_XC
and E_XC (paper section 3.1) element by element.

Tolerances follow from the roundings of the mixed path, as bounds scaled by
sums of absolute values (computed from the oracle's own quantities):
- J, K: each integral is evaluated in FP32 and stored in FP32; its error is
  held to 2^-19 Q_mn Q_ls (16 units u = 2^-24 of FP32 rounding on the
  quartet's Schwarz product Q_mn = sqrt((mn|mn)), from the oracle's
  integrals; the same bound the integral test checks), the density and the
  accumulation stay FP64, so |dJ_mn| <= 2^-19 Q_mn sum_ls Q_ls |P_ls| and
  |dK_ml| <= 2^-19 sum_ns Q_mn |P_ns| Q_ls, plus 1e-12 per term.
- V_XC: the Phi^T W product multiplies bf16 pairs (each operand within
  2^-17 relative, so 2^-16 per product term); the FP32 AO values carry
  |x| 1e-7 <= 4e-6 relative from the exponential at |x| <= 40 (2^-18 on
  each of the two factors, 2^-17 together), and the FP32 density and
  functional ~1e-6; in all eps = 2^-16 + 2^-17 + 2^-18 of
  A_mn + A_nm, A_mn = sum_g |phi_m| w (|v_rho|/2 |phi_n|
  + 2 |v_sigma| |grad rho| |grad phi_n|), which bounds sum_g |phi_m| |W_n|.
- E_XC: the FP32 density (through X = Phi P on FP32 MFMAs) and functional:
  eps_E = 2^-17 of sum_g w (|e| + |v_rho| rho + 2 |v_sigma| sigma), the
  first-order change of E_XC under a relative perturbation of rho, sigma
  and e.
Also checked: the FP64 kernels of the FP64 benchmark launch shape on the
same molecules to 1e-10.
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
NMOL = 2


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_01135_amd import ks as K
    K.load()
    return K


@pytest.fixture(scope="module")
def case():
    """Molecules, oracle densities and the oracle's J, K, V_XC, E_XC with
    their error scales."""
    dens = np.load(os.path.join(GOLDEN, "oracle_density_seed2.npz"))
    mols = molgen.batch(NMOL, 2, (9, 11))
    out = []
    for m, (z, x) in enumerate(mols):
        print("oracle J/K/XC of molecule %d" % m, flush=True)
        o = O.Mol(z, x)
        P = dens["P_default_%d" % m]
        eri = o.eri()
        J, K = o.jk(eri, P)
        N = o.nbf
        npair = N * (N + 1) // 2
        qp = np.sqrt(np.abs(eri[[q * (q + 1) // 2 + q for q in range(npair)]]))
        Q = np.zeros((N, N))
        iu, ju = np.tril_indices(N)
        Q[iu, ju] = qp
        Q[ju, iu] = qp
        BJ = Q * np.sum(Q * np.abs(P))
        BK = Q @ np.abs(P) @ Q
        grid = o.grid()
        exc, V = o.xc(O.XC_B3LYP, grid, P)
        A, SE = _xc_scales(o, grid, P)
        out.append(dict(P=P, J=J, K=K, BJ=BJ, BK=BK, Psum=np.abs(P).sum(), V=V, exc=exc, A=A, SE=SE))
    return mols, out


def _xc_scales(o, grid, P, chunk=20000):
    N = o.nbf
    A = np.zeros((N, N))
    se = 0.0
    for c0 in range(0, len(grid), chunk):
        g = grid[c0:c0 + chunk]
        ao = o.ao(g[:, :3])
        phi, dphi = ao[:, 0, :], ao[:, 1:, :]
        X = phi @ P
        rho = np.einsum("gi,gi->g", X, phi)
        grad = 2.0 * np.einsum("gi,gdi->gd", X, dphi)
        sigma = (grad ** 2).sum(1)
        e, vr, vs = O.functional(O.XC_B3LYP, rho, sigma)
        w = np.where(rho >= 1e-12, g[:, 3], 0.0)
        wabs = w[:, None] * (0.5 * np.abs(vr)[:, None] * np.abs(phi)
                             + 2.0 * (np.abs(vs) * np.sqrt(sigma))[:, None] * np.linalg.norm(dphi, axis=1))
        A += np.abs(phi).T @ wabs
        se += float(np.sum(w * (np.abs(e) + np.abs(vr) * rho + 2.0 * np.abs(vs) * sigma)))
    return A + A.T, se


def _bench_options(prec):
    return autotune.tuned_options(prec, [molgen.nbf_sto3g(z) for z, _ in molgen.batch(4096, 2, (9, 11))])


@pytest.mark.parametrize("prec", [1, 0])
def test_bench_kernels_vs_oracle(ks, case, prec):
    mols, ref = case
    opts = _bench_options(prec)
    print("prec %d, options %s" % (prec, opts), flush=True)
    with ks.Batch(mols, prec=prec, **opts) as b:
        b.setup()
        b.eri_build()
        Pt = b.pack([r["P"] for r in ref])
        J, K, V = b.empty(), b.empty(), b.empty()
        b.jk_build(Pt, J, K)
        exc = b.xc_build(Pt, V)
        J, K, V = b.unpack(J), b.unpack(K), b.unpack(V)
    u = 2.0 ** -24
    eps_v = 2.0 ** -16 + 2.0 ** -17 + 2.0 ** -18
    eps_e = 2.0 ** -17
    for m, r in enumerate(ref):
        dJ, dK, dV = np.abs(J[m] - r["J"]), np.abs(K[m] - r["K"]), np.abs(V[m] - r["V"])
        dE = abs(exc[m] - r["exc"])
        if prec == 1:
            tJ = 2.0 ** -19 * r["BJ"] + 1e-12 * r["Psum"]
            tK = 2.0 ** -19 * r["BK"] + 1e-12 * r["Psum"]
            tV = eps_v * r["A"] + 1e-14
            tE = eps_e * r["SE"]
        else:
            tJ = tK = tV = np.full_like(dJ, 1e-10)
            tE = 1e-9
        print("molecule %d: max |dJ| %.2e (%.3f of bound) |dK| %.2e (%.3f) |dV| %.2e (%.3f) |dExc| %.2e (%.3f)"
              % (m, dJ.max(), (dJ / tJ).max(), dK.max(), (dK / tK).max(), dV.max(), (dV / tV).max(),
                 dE, dE / tE), flush=True)
        assert np.all(dJ <= tJ), (m, np.unravel_index(np.argmax(dJ / tJ), dJ.shape))
        assert np.all(dK <= tK), (m, np.unravel_index(np.argmax(dK / tK), dK.shape))
        assert np.all(dV <= tV), (m, np.unravel_index(np.argmax(dV / tV), dV.shape))
        assert dE <= tE, (m, dE, tE)
