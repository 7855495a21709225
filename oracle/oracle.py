"""ctypes wrapper over the FP64 CPU oracle (oracle/ks_oracle.c).

Test infrastructure only: the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.
It imports nothing from the HIP package.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ks_oracle.c")
_LIB = os.path.join(_HERE, "libks_oracle.so")

XC_HF, XC_B3LYP, XC_B3LYP5 = 0, 1, 2
ST_CONVERGED, ST_MAXITER, ST_DIVERGED, ST_INVALID = 1, 2, 3, 4
GUESS_ATOM, GUESS_CORE = 0, 1
BASIS_STO3G, BASIS_631G = 0, 1

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc -O2 (no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        L.orc_mol_new.restype = C.c_void_p
        L.orc_mol_new.argtypes = [C.c_int, _ip, _dp, C.c_int]
        L.orc_mol_new_basis.restype = C.c_void_p
        L.orc_mol_new_basis.argtypes = [C.c_int, _ip, _dp, C.c_int, C.c_int]
        L.orc_mol_free.argtypes = [C.c_void_p]
        L.orc_mol_info.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.orc_shell.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                C.POINTER(C.c_int), C.POINTER(C.c_int), _dp, _dp]
        L.orc_enuc.restype = C.c_double
        L.orc_enuc.argtypes = [C.c_void_p]
        L.orc_int1e.argtypes = [C.c_void_p, _dp, _dp, _dp]
        L.orc_n_eri.restype = C.c_long
        L.orc_n_eri.argtypes = [C.c_void_p]
        L.orc_eri.argtypes = [C.c_void_p, _dp]
        L.orc_eri_one.restype = C.c_double
        L.orc_eri_one.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int]
        L.orc_jk.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp]
        L.orc_boys.argtypes = [C.c_int, C.c_double, _dp]
        L.orc_gauss_legendre.argtypes = [C.c_int, _dp, _dp]
        L.orc_radial.argtypes = [C.c_int, _dp, _dp]
        L.orc_grid_size.restype = C.c_long
        L.orc_grid_size.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.orc_grid.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, _dp]
        L.orc_ao.argtypes = [C.c_void_p, C.c_long, _dp, _dp]
        L.orc_functional.argtypes = [C.c_int, C.c_long, _dp, _dp, _dp, _dp, _dp]
        L.orc_xc.restype = C.c_double
        L.orc_xc.argtypes = [C.c_void_p, C.c_int, C.c_long, _dp, _dp, _dp]
        L.orc_eigh.argtypes = [C.c_int, _dp, _dp, _dp]
        L.orc_scf.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                              C.c_int, C.c_int, C.c_int, C.POINTER(C.c_double), _dp, _dp,
                              C.POINTER(C.c_int), C.POINTER(C.c_int), _dp]
        _lib = L
    return _lib


def boys(mmax: int, T: float) -> np.ndarray:
    out = np.zeros(mmax + 1)
    lib().orc_boys(mmax, float(T), out)
    return out


def gauss_legendre(n: int):
    x, w = np.zeros(n), np.zeros(n)
    lib().orc_gauss_legendre(n, x, w)
    return x, w


def radial(n: int):
    r, w = np.zeros(n), np.zeros(n)
    lib().orc_radial(n, r, w)
    return r, w


def functional(xc: int, rho, sigma):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    n = rho.size
    e, vr, vs = np.zeros(n), np.zeros(n), np.zeros(n)
    lib().orc_functional(xc, n, rho, sigma, e, vr, vs)
    return e, vr, vs


def eigh(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    n = A.shape[0]
    w, V = np.zeros(n), np.zeros((n, n))
    lib().orc_eigh(n, A, w, V)
    return w, V


class Mol:
    """One molecule in the oracle: Z (ints), xyz in Angstrom."""

    def __init__(self, Z, xyz_ang, charge: int = 0, basis: int = 0):
        Z = np.ascontiguousarray(Z, dtype=np.int32)
        xyz = np.ascontiguousarray(np.asarray(xyz_ang, dtype=np.float64).reshape(-1))
        self.h = lib().orc_mol_new_basis(len(Z), Z, xyz, charge, basis)
        if not self.h:
            raise ValueError("oracle rejected the molecule (element, charge or geometry)")
        nbf, nocc, nsh = C.c_int(), C.c_int(), C.c_int()
        lib().orc_mol_info(self.h, C.byref(nbf), C.byref(nocc), C.byref(nsh))
        self.nbf, self.nocc, self.nshell = nbf.value, nocc.value, nsh.value
        self.natom = len(Z)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_mol_free(self.h)
            self.h = None

    def shell(self, s):
        """(L, atom, first AO, exponents, coefficients) of shell s."""
        L, at, b0, n = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        a, c = np.zeros(6), np.zeros(6)
        lib().orc_shell(self.h, s, C.byref(L), C.byref(at), C.byref(b0), C.byref(n), a, c)
        return L.value, at.value, b0.value, a[:n.value].copy(), c[:n.value].copy()

    def enuc(self) -> float:
        return lib().orc_enuc(self.h)

    def int1e(self):
        N = self.nbf
        S, T, V = np.zeros((N, N)), np.zeros((N, N)), np.zeros((N, N))
        lib().orc_int1e(self.h, S, T, V)
        return S, T, V

    def n_eri(self) -> int:
        return lib().orc_n_eri(self.h)

    def eri(self) -> np.ndarray:
        out = np.zeros(self.n_eri())
        lib().orc_eri(self.h, out)
        return out

    def eri_one(self, i, j, k, l) -> float:
        return lib().orc_eri_one(self.h, int(i), int(j), int(k), int(l))

    def jk(self, eri, P):
        N = self.nbf
        J, K = np.zeros((N, N)), np.zeros((N, N))
        lib().orc_jk(self.h, np.ascontiguousarray(eri), np.ascontiguousarray(P, dtype=np.float64), J, K)
        return J, K

    def grid(self, nrad=50, nth=12, nph=24) -> np.ndarray:
        G = lib().orc_grid_size(self.h, nrad, nth, nph)
        out = np.zeros((G, 4))
        lib().orc_grid(self.h, nrad, nth, nph, out)
        return out

    def ao(self, xyz) -> np.ndarray:
        xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, 3))
        out = np.zeros((xyz.shape[0], 4, self.nbf))
        lib().orc_ao(self.h, xyz.shape[0], xyz, out)
        return out

    def xc(self, xc: int, grid, P):
        N = self.nbf
        V = np.zeros((N, N))
        g = np.ascontiguousarray(grid, dtype=np.float64)
        e = lib().orc_xc(self.h, xc, g.shape[0], g, np.ascontiguousarray(P, dtype=np.float64), V)
        return e, V

    def scf(self, xc: int = XC_B3LYP, nrad=50, nth=12, nph=24, e_tol=1e-9, comm_tol=1e-7,
            max_iter=100, diis_space=8, guess=GUESS_ATOM):
        N = self.nbf
        E = C.c_double()
        eps, P, terms = np.zeros(N), np.zeros((N, N)), np.zeros(6)
        nit, st = C.c_int(), C.c_int()
        rc = lib().orc_scf(self.h, xc, nrad, nth, nph, e_tol, comm_tol, max_iter, diis_space, guess,
                           C.byref(E), eps, P, C.byref(nit), C.byref(st), terms)
        if rc != 0:
            raise ValueError("oracle SCF failed: near-singular overlap")
        no = self.nocc
        homo, lumo = eps[no - 1], (eps[no] if no < N else float("nan"))
        return dict(E=E.value, eps=eps, P=P, n_iter=nit.value, status=st.value,
                    homo=homo, lumo=lumo, gap=lumo - homo, terms=terms)
