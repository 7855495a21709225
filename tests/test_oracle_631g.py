"""Pins of the oracle's 6-31G basis (H, C, N, O; the next basis after
STO-3G, with a six-primitive core shell, a 3 + 1 split valence and sp
shells sharing exponents).

- H2 at R = 1.4 bohr, Hartree-Fock: H is the same 31G contraction in 4-31G
  and 6-31G, and the textbook table of H2 energies (Szabo and Ostlund,
  "Modern Quantum Chemistry", chapter 3) gives -1.127 Ha for 4-31G.
- Variable primitive counts: overlap and (ss|ss) integrals of contracted
  s functions with 6, 3 and 1 primitives against the Gaussian-product
  closed forms summed by hand over primitive pairs (mpmath).
- Normalisation (S_mu,mu = 1), Tr(P S) = N_e and P S P = 2 P for a 6-31G
  SCF, and the function count (H 2, C/N/O 9).
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import oracle as O
from paper_2311_01135_amd import molgen

BOHR = 0.52917721092


def _h2(r_bohr):
    return np.array([1, 1]), np.array([[0.0, 0.0, 0.0], [0.0, 0.0, r_bohr * BOHR]])


def test_h2_hf_energy_textbook():
    z, x = _h2(1.4)
    m = O.Mol(z, x, basis=O.BASIS_631G)
    assert (m.nbf, m.nocc) == (4, 1)
    r = m.scf(xc=O.XC_HF)
    assert r["status"] == 1
    assert abs(r["E"] - (-1.127)) < 5e-4, r["E"]
    # the split valence lowers the energy below STO-3G's -1.1167
    assert r["E"] < O.Mol(z, x).scf(xc=O.XC_HF)["E"] - 5e-3


def test_function_counts():
    z = np.array([8, 6, 7, 1, 1, 1])
    x = np.array([[0, 0, 0], [1.4, 0, 0], [0, 1.4, 0], [0, 0, 1.0], [2.4, 0, 0], [0, 2.4, 0]], dtype=float)
    m = O.Mol(z, x, basis=O.BASIS_631G)
    assert m.nbf == 3 * 9 + 3 * 2
    # fluorine is not part of this 6-31G table
    with pytest.raises(ValueError):
        O.Mol(np.array([9, 1]), np.array([[0, 0, 0], [0, 0, 0.92]]), basis=O.BASIS_631G)


def _s_contraction(m, s):
    L, at, b0, a, c = m.shell(s)
    assert L == 0
    return a, c


def _overlap_ss(a1, c1, A, a2, c2, B):
    tot = mp.mpf(0)
    AB2 = sum((mp.mpf(A[k]) - mp.mpf(B[k])) ** 2 for k in range(3))
    for i in range(len(a1)):
        for j in range(len(a2)):
            p = mp.mpf(a1[i]) + mp.mpf(a2[j])
            mu = mp.mpf(a1[i]) * mp.mpf(a2[j]) / p
            tot += mp.mpf(c1[i]) * mp.mpf(c2[j]) * (mp.pi / p) ** 1.5 * mp.exp(-mu * AB2)
    return tot


def _eri_ssss(sh, centres):
    # (ab|cd) for contracted s functions: sum over primitive quartets of
    # 2 pi^(5/2) / (p q sqrt(p+q)) K_ab K_cd F0(pq/(p+q) |P-Q|^2)
    (a1, c1), (a2, c2), (a3, c3), (a4, c4) = sh
    A, B, C, D = [[mp.mpf(v) for v in r] for r in centres]
    tot = mp.mpf(0)
    for i in range(len(a1)):
        for j in range(len(a2)):
            p = mp.mpf(a1[i]) + mp.mpf(a2[j])
            P = [(mp.mpf(a1[i]) * A[k] + mp.mpf(a2[j]) * B[k]) / p for k in range(3)]
            Kab = mp.exp(-mp.mpf(a1[i]) * mp.mpf(a2[j]) / p * sum((A[k] - B[k]) ** 2 for k in range(3)))
            for k_ in range(len(a3)):
                for l_ in range(len(a4)):
                    q = mp.mpf(a3[k_]) + mp.mpf(a4[l_])
                    Q = [(mp.mpf(a3[k_]) * C[k] + mp.mpf(a4[l_]) * D[k]) / q for k in range(3)]
                    Kcd = mp.exp(-mp.mpf(a3[k_]) * mp.mpf(a4[l_]) / q * sum((C[k] - D[k]) ** 2 for k in range(3)))
                    T = p * q / (p + q) * sum((P[k] - Q[k]) ** 2 for k in range(3))
                    F0 = mp.mpf(1) if T == 0 else mp.sqrt(mp.pi / T) / 2 * mp.erf(mp.sqrt(T))
                    tot += (mp.mpf(c1[i]) * mp.mpf(c2[j]) * mp.mpf(c3[k_]) * mp.mpf(c4[l_]) * 2 * mp.pi ** 2.5
                            / (p * q * mp.sqrt(p + q)) * Kab * Kcd * F0)
    return tot


def test_variable_primitive_integrals_vs_closed_form():
    mp.mp.dps = 25
    z, x = molgen.water(0)
    m = O.Mol(z, x, basis=O.BASIS_631G)
    R = np.asarray(x, dtype=float) / BOHR
    S, _, _ = m.int1e()
    # shells: O 1s (6), 2s (3), 2p, 3s (1), 3p; H 1s (3), H 2s (1), ...
    sh_o1s, sh_o2s, sh_o3s = (_s_contraction(m, s) for s in (0, 1, 3))
    sh_h1s, sh_h2s = (_s_contraction(m, s) for s in (5, 6))
    assert len(sh_o1s[0]) == 6 and len(sh_o2s[0]) == 3 and len(sh_o3s[0]) == 1
    assert len(sh_h1s[0]) == 3 and len(sh_h2s[0]) == 1
    ao = {"o1s": 0, "o2s": 1, "o3s": 5, "h1s": 9, "h2s": 10}
    shells = {"o1s": (sh_o1s, R[0]), "o2s": (sh_o2s, R[0]), "o3s": (sh_o3s, R[0]),
              "h1s": (sh_h1s, R[1]), "h2s": (sh_h2s, R[1])}
    for u in shells:
        for v in shells:
            (a1, c1), A = shells[u]
            (a2, c2), B = shells[v]
            ref = _overlap_ss(a1, c1, A, a2, c2, B)
            assert abs(S[ao[u], ao[v]] - float(ref)) < 1e-13, (u, v)
    eri = m.eri()

    def idx(i, j, k, l):
        ij = i * (i + 1) // 2 + j if i >= j else j * (j + 1) // 2 + i
        kl = k * (k + 1) // 2 + l if k >= l else l * (l + 1) // 2 + k
        return ij * (ij + 1) // 2 + kl if ij >= kl else kl * (kl + 1) // 2 + ij

    for q in (("o1s", "o1s", "o1s", "o1s"), ("o1s", "h1s", "o3s", "h2s"), ("h2s", "h2s", "o2s", "o1s"),
              ("o3s", "o3s", "h1s", "h1s")):
        sh = [shells[t][0] for t in q]
        cen = [shells[t][1] for t in q]
        ref = float(_eri_ssss(sh, cen))
        got = eri[idx(*(ao[t] for t in q))]
        assert abs(got - ref) < 1e-12 * max(1.0, abs(ref)), (q, got, ref)


def test_water_scf_invariants():
    z, x = molgen.water(0)
    m = O.Mol(z, x, basis=O.BASIS_631G)
    assert (m.nbf, m.nocc) == (13, 5)
    S, _, _ = m.int1e()
    assert np.abs(np.diag(S) - 1.0).max() < 1e-13
    r = m.scf(xc=O.XC_B3LYP, nrad=30, nth=10, nph=20)
    assert r["status"] == 1
    P = r["P"]
    assert abs(np.sum(P * S) - 10.0) < 1e-9
    assert np.abs(P @ S @ P - 2 * P).max() < 1e-8
    # the larger basis lowers the energy against STO-3G on the same grid
    assert r["E"] < O.Mol(z, x).scf(xc=O.XC_B3LYP, nrad=30, nth=10, nph=20)["E"] - 0.3
