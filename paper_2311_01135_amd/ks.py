"""Thin ctypes binding of libks.so (argument marshalling only).

Every step of the Kohn-Sham path runs in the library's HIP kernels; this
module converts arguments, owns nothing on the device except through the
library handle, and raises KsError on any non-zero status.  Device buffers
are torch CUDA (HIP) tensors; torch is used for memory and streams only.
Importing this module on a machine without the built library raises an
ImportError: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libks.so")

KS_XC_HF, KS_XC_B3LYP, KS_XC_B3LYP5 = 0, 1, 2
KS_FP64, KS_MIXED = 0, 1
KS_GUESS_ATOM, KS_GUESS_CORE = 0, 1
KS_BASIS_STO3G, KS_BASIS_631G = 0, 1
ERI_WINDOW_MAX = 1048576          # KS_ERI_WINDOW_MAX of ks.h
MOL_ACTIVE, MOL_CONVERGED, MOL_MAXITER, MOL_DIVERGED = 0, 1, 2, 3
MATRIX = {"S": 0, "T": 1, "V": 2, "X": 3, "F": 4, "P": 5, "J": 6, "K": 7, "Vxc": 8}
STATUS_NAMES = {0: "KS_OK", -1: "KS_EINVAL", -2: "KS_ENOMEM", -3: "KS_EDEVICE", -4: "KS_ENOCONV",
                -5: "KS_EUNSUPPORTED", -6: "KS_ESTATE"}

EXPORTS = ["ks_default_options", "ks_batch_create", "ks_batch_sizes", "ks_batch_quartets", "ks_setup",
           "eri_build", "jk_build", "xc_build", "fock_build", "scf_step", "scf_solve", "scf_solve_many",
           "ks_get_result", "ks_get_eri", "ks_get_eri_window", "ks_get_matrix", "ks_get_grid", "ks_get_convergence",
           "ks_get_iterations", "ks_get_results", "ks_kernel_times",
           "ks_kernel_counts", "ks_set_timing",
           "ks_batch_destroy", "ks_last_error", "ks_server_create", "ks_server_submit",
           "ks_server_progress", "ks_server_poll", "ks_server_stats", "ks_server_fail_admissions",
           "ks_server_destroy"]


class KsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


class Options(C.Structure):
    _fields_ = [("xc", C.c_int), ("prec", C.c_int), ("n_rad", C.c_int), ("n_theta", C.c_int),
                ("n_phi", C.c_int), ("e_tol", C.c_double), ("comm_tol", C.c_double),
                ("max_iter", C.c_int), ("diis_space", C.c_int), ("jk_chunks", C.c_int),
                ("xc_chunks", C.c_int), ("guess", C.c_int), ("xc_points", C.c_int),
                ("xc_waves", C.c_int), ("direct", C.c_int), ("schwarz_tol", C.c_double),
                ("basis", C.c_int), ("graphs", C.c_int), ("coarse_rad", C.c_int),
                ("coarse_theta", C.c_int), ("coarse_phi", C.c_int), ("eri_threads", C.c_int * 6),
                ("eri_unroll", C.c_int * 6)]


_lib = None


def load():
    """Load libks.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libks.so not built (run paper_2311_01135_amd/build.py): %s" % LIB_PATH)
    L = C.CDLL(LIB_PATH)
    vp, ip, dp, lp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_long)
    L.ks_default_options.argtypes = [C.POINTER(Options)]
    L.ks_batch_create.argtypes = [C.POINTER(Options), C.c_int, ip, ip, dp, ip, vp, C.POINTER(vp)]
    L.ks_batch_sizes.argtypes = [vp, C.c_int, ip, ip, lp, lp]
    L.ks_batch_quartets.argtypes = [vp, lp, lp]
    for f in ("ks_setup", "eri_build", "scf_solve"):
        getattr(L, f).argtypes = [vp]
    L.jk_build.argtypes = [vp, vp, vp, vp]
    L.xc_build.argtypes = [vp, vp, vp, dp]
    L.fock_build.argtypes = [vp, vp, vp, dp]
    L.scf_step.argtypes = [vp, ip]
    L.scf_solve_many.argtypes = [C.POINTER(vp), C.c_int]
    L.ks_get_result.argtypes = [vp, C.c_int, dp, dp, dp, dp, dp, dp, ip, ip]
    L.ks_get_eri.argtypes = [vp, C.c_int, dp]
    L.ks_get_eri_window.argtypes = [vp, C.c_int, C.c_long, C.c_long, dp]
    L.ks_get_eri_window.restype = C.c_int
    L.ks_get_matrix.argtypes = [vp, C.c_int, C.c_int, dp]
    L.ks_get_grid.argtypes = [vp, C.c_int, dp]
    L.ks_kernel_times.argtypes = [vp, C.POINTER(C.c_char_p), dp, C.c_int]
    L.ks_kernel_times.restype = C.c_int
    L.ks_set_timing.argtypes = [vp, C.c_int]
    L.ks_kernel_counts.argtypes = [vp, dp, C.c_int]
    L.ks_kernel_counts.restype = C.c_int
    L.ks_get_convergence.argtypes = [vp, C.c_int, dp, dp, dp]
    L.ks_get_convergence.restype = C.c_int
    L.ks_get_iterations.argtypes = [vp, C.c_int, ip, ip]
    L.ks_get_iterations.restype = C.c_int
    L.ks_get_results.argtypes = [vp, dp, dp, dp, dp, ip, ip, ip, dp, dp]
    L.ks_get_results.restype = C.c_int
    L.ks_batch_destroy.argtypes = [vp]
    L.ks_batch_destroy.restype = None
    L.ks_server_create.argtypes = [C.POINTER(Options), C.c_size_t, C.c_int, C.POINTER(vp)]
    L.ks_server_submit.argtypes = [vp, C.c_int, ip, dp, C.c_int, lp]
    L.ks_server_progress.argtypes = [vp, ip]
    L.ks_server_poll.argtypes = [vp, C.c_long, dp, dp, dp, dp, ip, ip, dp]
    L.ks_server_stats.argtypes = [vp, ip, ip, lp, C.POINTER(C.c_size_t)]
    L.ks_server_fail_admissions.argtypes = [vp, C.c_int]
    L.ks_server_destroy.argtypes = [vp]
    L.ks_server_destroy.restype = None
    for name in ("ks_server_create", "ks_server_submit", "ks_server_progress", "ks_server_poll", "ks_server_stats",
                 "ks_server_fail_admissions"):
        getattr(L, name).restype = C.c_int
    L.ks_last_error.restype = C.c_char_p
    for name in ("ks_batch_create", "ks_batch_sizes", "ks_batch_quartets", "ks_setup", "eri_build",
                 "jk_build", "xc_build", "fock_build", "scf_step", "scf_solve", "scf_solve_many", "ks_get_result",
                 "ks_get_eri", "ks_get_matrix", "ks_get_grid"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(st):
    if st != 0:
        raise KsError(st, load().ks_last_error().decode())


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def default_options(**kw) -> Options:
    o = Options()
    load().ks_default_options(C.byref(o))
    for k, v in kw.items():
        if isinstance(v, (list, tuple)):
            v = (C.c_int * len(v))(*v)
        setattr(o, k, v)
    return o


def solve_many(batches):
    """scf_solve over several batches at once (each on its own stream, so their
    kernels overlap); same results as solving each alone."""
    arr = (C.c_void_p * len(batches))(*[b.h for b in batches])
    _check(load().scf_solve_many(arr, len(batches)))


class Batch:
    """A batch of molecules resident on the GPU.  mols: list of (Z, xyz_angstrom)."""

    def __init__(self, mols, charges=None, stream=None, **options):
        L = load()
        self.opt = default_options(**options)
        n_atoms = np.array([len(z) for z, _ in mols], dtype=np.int32)
        Z = np.ascontiguousarray(np.concatenate([np.asarray(z, dtype=np.int32) for z, _ in mols]))
        xyz = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float64).reshape(-1) for _, x in mols]))
        ch = None if charges is None else np.ascontiguousarray(np.asarray(charges, dtype=np.int32))
        h = C.c_void_p()
        sp = None if stream is None else C.c_void_p(stream)
        _check(L.ks_batch_create(C.byref(self.opt), len(mols), _iptr(n_atoms), _iptr(Z), _dptr(xyz),
                                 None if ch is None else _iptr(ch), sp, C.byref(h)))
        self.h = h
        self.n_mol = len(mols)
        self.nbf, self.nocc, self.n_eri, self.n_grid = [], [], [], []
        for m in range(self.n_mol):
            nb, no, ne, ng = C.c_int(), C.c_int(), C.c_long(), C.c_long()
            _check(L.ks_batch_sizes(self.h, m, C.byref(nb), C.byref(no), C.byref(ne), C.byref(ng)))
            self.nbf.append(nb.value)
            self.nocc.append(no.value)
            self.n_eri.append(ne.value)
            self.n_grid.append(ng.value)
        self.mat_off = np.concatenate([[0], np.cumsum([n * n for n in self.nbf])]).astype(np.int64)

    # -- lifetime ---------------------------------------------------------
    def close(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.ks_batch_destroy(h)
        self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- entry points -----------------------------------------------------
    def quartets(self):
        a, b = C.c_long(), C.c_long()
        _check(load().ks_batch_quartets(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def setup(self):
        _check(load().ks_setup(self.h))

    def eri_build(self):
        _check(load().eri_build(self.h))

    def jk_build(self, P, J, K):
        _check(load().jk_build(self.h, C.c_void_p(P.data_ptr()), C.c_void_p(J.data_ptr()), C.c_void_p(K.data_ptr())))

    def xc_build(self, P, V):
        exc = np.zeros(self.n_mol)
        _check(load().xc_build(self.h, C.c_void_p(P.data_ptr()), C.c_void_p(V.data_ptr()), _dptr(exc)))
        return exc

    def fock_build(self, P=None, F=None):
        et = np.zeros((self.n_mol, 6))
        _check(load().fock_build(self.h, None if P is None else C.c_void_p(P.data_ptr()),
                                 None if F is None else C.c_void_p(F.data_ptr()), _dptr(et)))
        return et

    def scf_step(self) -> int:
        n = C.c_int()
        _check(load().scf_step(self.h, C.byref(n)))
        return n.value

    def scf_solve(self):
        _check(load().scf_solve(self.h))

    def set_timing(self, on: bool):
        load().ks_set_timing(self.h, 1 if on else 0)

    def kernel_times(self):
        names = (C.c_char_p * 64)()
        ms = (C.c_double * 64)()
        n = load().ks_kernel_times(self.h, names, ms, 64)
        cnt = (C.c_double * 64)()
        load().ks_kernel_counts(self.h, cnt, 64)
        return {names[i].decode(): (ms[i], int(cnt[i])) for i in range(min(n, 64))}

    def convergence(self, m):
        E, dE, err = C.c_double(), C.c_double(), C.c_double()
        _check(load().ks_get_convergence(self.h, m, C.byref(E), C.byref(dE), C.byref(err)))
        return E.value, dE.value, err.value

    def results(self, density=True):
        """Every molecule's result in one call (ks_get_results): a list of
        dicts with the keys of result() plus n_coarse; eps and P are views
        into one array each (P omitted with density=False)."""
        n = self.n_mol
        E, homo, lumo, gap = (np.zeros(n) for _ in range(4))
        st, it, nc = (np.zeros(n, dtype=np.int32) for _ in range(3))
        eps = np.zeros(int(sum(self.nbf)))
        P = np.zeros(int(sum(N * N for N in self.nbf))) if density else None
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int))
        _check(load().ks_get_results(self.h, _dptr(E), _dptr(homo), _dptr(lumo), _dptr(gap), ip(st), ip(it), ip(nc),
                                     _dptr(eps), _dptr(P) if density else None))
        out, a0, m0 = [], 0, 0
        for m, N in enumerate(self.nbf):
            r = dict(E=float(E[m]), eps=eps[a0:a0 + N], homo=float(homo[m]), lumo=float(lumo[m]), gap=float(gap[m]),
                     status=int(st[m]), n_iter=int(it[m]), n_coarse=int(nc[m]))
            if density:
                r["P"] = P[m0:m0 + N * N].reshape(N, N)
            out.append(r)
            a0 += N
            m0 += N * N
        return out

    def iterations(self, m):
        """(iterations so far, of which on the coarse start grid)."""
        n, c = C.c_int(), C.c_int()
        _check(load().ks_get_iterations(self.h, m, C.byref(n), C.byref(c)))
        return n.value, c.value

    # -- results ----------------------------------------------------------
    def result(self, m):
        N = self.nbf[m]
        E, homo, lumo, gap = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        st, it = C.c_int(), C.c_int()
        eps, P = np.zeros(N), np.zeros((N, N))
        _check(load().ks_get_result(self.h, m, C.byref(E), _dptr(eps), _dptr(P), C.byref(homo), C.byref(lumo),
                                    C.byref(gap), C.byref(st), C.byref(it)))
        return dict(E=E.value, eps=eps, P=P, homo=homo.value, lumo=lumo.value, gap=gap.value,
                    status=st.value, n_iter=it.value)

    def eri(self, m):
        out = np.zeros(self.n_eri[m])
        _check(load().ks_get_eri(self.h, m, _dptr(out)))
        return out

    def eri_window(self, m, lo, count, out=None):
        """Packed ERIs lo .. lo+count-1 of molecule m (ks_get_eri_window: no
        device allocation, at most ERI_WINDOW_MAX per call)."""
        if out is None:
            out = np.zeros(max(0, count))
        _check(load().ks_get_eri_window(self.h, m, lo, count, _dptr(out) if count > 0 else None))
        return out

    def matrix(self, m, which):
        N = self.nbf[m]
        out = np.zeros((N, N))
        _check(load().ks_get_matrix(self.h, m, MATRIX[which] if isinstance(which, str) else which, _dptr(out)))
        return out

    def grid(self, m):
        out = np.zeros((self.n_grid[m], 4))
        _check(load().ks_get_grid(self.h, m, _dptr(out)))
        return out

    # -- helpers for concatenated device matrices -------------------------
    def pack(self, mats, device="cuda"):
        import torch
        flat = np.concatenate([np.ascontiguousarray(a, dtype=np.float64).reshape(-1) for a in mats])
        return torch.from_numpy(flat).to(device)

    def empty(self, device="cuda"):
        import torch
        return torch.zeros(int(self.mat_off[-1]), dtype=torch.float64, device=device)

    def unpack(self, t):
        a = t.detach().cpu().numpy()
        return [a[self.mat_off[m]:self.mat_off[m + 1]].reshape(self.nbf[m], self.nbf[m]) for m in range(self.n_mol)]


class Server:
    """Continuous-batching SCF server (ks_server_*)."""

    def __init__(self, hbm_budget: int = 0, max_batch: int = 64, **options):
        L = load()
        self.opt = default_options(**options)
        h = C.c_void_p()
        _check(L.ks_server_create(C.byref(self.opt), C.c_size_t(hbm_budget), max_batch, C.byref(h)))
        self.h = h

    def close(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.ks_server_destroy(h)
        self.h = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, Z, xyz, charge: int = 0) -> int:
        Z = np.ascontiguousarray(np.asarray(Z, dtype=np.int32))
        xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1))
        t = C.c_long()
        _check(load().ks_server_submit(self.h, len(Z), _iptr(Z), _dptr(xyz), charge, C.byref(t)))
        return t.value

    def progress(self) -> int:
        n = C.c_int()
        _check(load().ks_server_progress(self.h, C.byref(n)))
        return n.value

    def poll(self, ticket):
        """dict of results when finished, None while pending."""
        E, homo, lumo, gap, lat = (C.c_double() for _ in range(5))
        st, it = C.c_int(), C.c_int()
        rc = load().ks_server_poll(self.h, ticket, C.byref(E), C.byref(homo), C.byref(lumo), C.byref(gap),
                                   C.byref(st), C.byref(it), C.byref(lat))
        if rc == -6:
            return None
        _check(rc)
        return dict(E=E.value, homo=homo.value, lumo=lumo.value, gap=gap.value, status=st.value,
                    n_iter=it.value, latency=lat.value)

    def fail_admissions(self, n: int):
        """Testing hook: the next n admissions fail as if out of device memory."""
        _check(load().ks_server_fail_admissions(self.h, n))

    def stats(self):
        q, r, d, by = C.c_int(), C.c_int(), C.c_long(), C.c_size_t()
        _check(load().ks_server_stats(self.h, C.byref(q), C.byref(r), C.byref(d), C.byref(by)))
        return dict(queued=q.value, resident=r.value, done=d.value, bytes=by.value)
