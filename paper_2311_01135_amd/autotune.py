"""Tile / chunk autotuner for the Fock-build kernels.

For a workload (number of molecules, heavy-atom range, precision) it times,
with HIP events on the batch stream, the XC kernel over its launch shapes
(grid points per sub-block x wavefronts per work group) and work-group counts
per molecule, the J/K digestion over its work-group counts per molecule, on
the molecules' initial densities, and the ERI class kernels over their
work-group size and ket-loop unroll (each quartet class separately).  The best settings are stored in a JSON
table keyed by precision, basis-size bucket (largest N rounded up to 16) and
batch-size bucket; `tuned_options` returns the entry closest to a batch.

    python -m paper_2311_01135_amd.autotune --n-mol 256 --heavy 9-11 --prec mixed
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")

XC_SHAPES = [(64, 8), (64, 16), (32, 8), (32, 16), (16, 8), (64, 4), (32, 4)]
XC_CHUNKS = [16, 32, 64]
JK_CHUNKS = [2, 4, 8, 16]
ERI_THREADS = [64, 128, 256]
ERI_UNROLL = [3, 9]
ERI_CLASSES = ["ssss", "psss", "psps", "ppss", "ppps", "pppp"]


def _bucket_np(nbf_max: int) -> int:
    return (nbf_max + 15) // 16 * 16


def _bucket_batch(n_mol: int) -> int:
    b = 1
    while b < n_mol:
        b *= 4
    return b


def key(prec: int, nbf_max: int, n_mol: int) -> str:
    return "%s/np%d/b%d" % ("mixed" if prec == 1 else "fp64", _bucket_np(nbf_max), _bucket_batch(n_mol))


def load_table(path: str = TABLE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def tuned_options(prec: int, nbf, path: str = TABLE) -> dict:
    """Options (xc_points, xc_waves, xc_chunks, jk_chunks) for a batch with
    basis sizes nbf, from the nearest tuned entry of the same precision and
    basis bucket (by batch size); {} when nothing is tuned."""
    table = load_table(path)
    want_np = _bucket_np(max(nbf))
    best, dist = None, None
    for k, v in table.items():
        p, np_s, b_s = k.split("/")
        if p != ("mixed" if prec == 1 else "fp64") or int(np_s[2:]) != want_np:
            continue
        d = abs(int(b_s[1:]).bit_length() - _bucket_batch(len(nbf)).bit_length())
        if dist is None or d < dist:
            best, dist = v, d
    if not best:
        return {}
    keys = ("xc_points", "xc_waves", "xc_chunks", "jk_chunks", "eri_threads", "eri_unroll")
    return {k: best[k] for k in keys if k in best}


def _time_xc(ks, mols, prec, pts, waves, chunks, reps):
    b = ks.Batch(mols, prec=prec, xc_points=pts, xc_waves=waves, xc_chunks=chunks)
    b.setup()
    P = b.pack([b.matrix(m, "P") for m in range(b.n_mol)])
    V = b.empty()
    b.xc_build(P, V)
    b.set_timing(True)
    for _ in range(reps):
        b.xc_build(P, V)
    ms = b.kernel_times()["xc"][0]
    b.close()
    return ms


def _time_jk(ks, mols, prec, chunks, reps):
    b = ks.Batch(mols, prec=prec, jk_chunks=chunks)
    b.eri_build()
    P = b.pack([b.matrix(m, "P") for m in range(b.n_mol)])
    J, K = b.empty(), b.empty()
    b.jk_build(P, J, K)
    b.set_timing(True)
    for _ in range(reps):
        b.jk_build(P, J, K)
    ms = b.kernel_times()["jk"][0]
    b.close()
    return ms


def _time_eri(ks, mols, prec, threads, unroll, reps):
    """Per-class ERI kernel times (ms) of eri_build with these launch shapes,
    the grid and one-electron set-up finished first; median of reps builds."""
    import torch
    runs = []
    for _ in range(reps):
        b = ks.Batch(mols, prec=prec, eri_threads=threads, eri_unroll=unroll)
        b.setup()
        torch.cuda.synchronize()
        b.set_timing(True)
        b.eri_build()
        kt = b.kernel_times()
        runs.append([kt["eri_" + c][0] if ("eri_" + c) in kt else 0.0 for c in ERI_CLASSES])
        b.close()
    runs.sort(key=sum)
    return runs[len(runs) // 2]


def tune_eri(ks, mols, prec, reps=3, log=print):
    """Work-group size and ket unroll per quartet class: every (threads,
    unroll) pair is timed for all classes at once (the classes are separate
    launches), and each class keeps its fastest pair."""
    res = []
    for t in ERI_THREADS:
        for u in ERI_UNROLL:
            ms = _time_eri(ks, mols, prec, [t] * 6, [u] * 6, reps)
            res.append((t, u, ms))
            log("eri threads %3d unroll %d: %s (sum %.2f ms)" % (t, u, " ".join("%.2f" % v for v in ms), sum(ms)))
    threads, unroll, best_ms = [], [], []
    for c in range(6):
        t, u, ms = min(res, key=lambda r: r[2][c])
        threads.append(t)
        unroll.append(u)
        best_ms.append(ms[c])
    base = next(r[2] for r in res if r[0] == 128 and r[1] == 3)
    return dict(eri_threads=threads, eri_unroll=unroll, eri_ms=sum(best_ms), eri_ms_default=sum(base)), res


def tune(ks, mols, prec, reps=3, log=print, shapes=None, xc_chunks=None, jk_chunks=None):
    res = {"xc": [], "jk": []}
    for pts, waves in shapes or XC_SHAPES:
        for ch in xc_chunks or XC_CHUNKS:
            ms = _time_xc(ks, mols, prec, pts, waves, ch, reps)
            res["xc"].append(dict(xc_points=pts, xc_waves=waves, xc_chunks=ch, ms=ms))
            log("xc points %2d waves %d chunks %2d: %.2f ms" % (pts, waves, ch, ms))
    for ch in jk_chunks or JK_CHUNKS:
        ms = _time_jk(ks, mols, prec, ch, reps)
        res["jk"].append(dict(jk_chunks=ch, ms=ms))
        log("jk chunks %2d: %.2f ms" % (ch, ms))
    bx = min(res["xc"], key=lambda r: r["ms"])
    bj = min(res["jk"], key=lambda r: r["ms"])
    best = dict(xc_points=bx["xc_points"], xc_waves=bx["xc_waves"], xc_chunks=bx["xc_chunks"],
                jk_chunks=bj["jk_chunks"], xc_ms=bx["ms"], jk_ms=bj["ms"])
    be, res["eri"] = tune_eri(ks, mols, prec, reps, log)
    best.update(be)
    return best, res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-mol", type=int, default=256)
    ap.add_argument("--heavy", default="9-11")
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--prec", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=TABLE)
    ap.add_argument("--xc-shapes", default="", help="points x waves list, e.g. 64x16,64x8 (default: all)")
    ap.add_argument("--xc-chunks", default="", help="work groups per molecule list, e.g. 32,64 (default: all)")
    ap.add_argument("--jk-chunks", default="", help="J/K work groups per molecule list (default: all)")
    ap.add_argument("--eri-only", action="store_true",
                    help="tune only the ERI launch shapes and merge them into the existing entry")
    a = ap.parse_args()
    sys.path.insert(0, ROOT)
    import torch
    from paper_2311_01135_amd import ks, molgen
    torch.cuda.set_device(0)
    lo, hi = (int(v) for v in a.heavy.split("-")) if "-" in a.heavy else (int(a.heavy),) * 2
    mols = molgen.batch(a.n_mol, a.seed, (lo, hi) if lo != hi else lo)
    prec = 1 if a.prec == "mixed" else 0
    shapes = [tuple(int(v) for v in t.split("x")) for t in a.xc_shapes.split(",")] if a.xc_shapes else None
    xcc = [int(v) for v in a.xc_chunks.split(",")] if a.xc_chunks else None
    jkc = [int(v) for v in a.jk_chunks.split(",")] if a.jk_chunks else None
    nbf = [molgen.nbf_sto3g(z) for z, _ in mols]
    table = load_table(a.out)
    k = key(prec, max(nbf), len(mols))
    if a.eri_only:
        best, _ = tune_eri(ks, mols, prec, a.reps, log=lambda s: print(s, flush=True))
        entry = dict(table.get(k, {}))
        entry.update(best)
        entry.setdefault("workload", "%d x %s heavy, seed %d" % (a.n_mol, a.heavy, a.seed))
        table[k] = entry
    else:
        best, res = tune(ks, mols, prec, a.reps, log=lambda s: print(s, flush=True), shapes=shapes, xc_chunks=xcc,
                         jk_chunks=jkc)
        table[k] = dict(best, workload="%d x %s heavy, seed %d" % (a.n_mol, a.heavy, a.seed))
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print("best", json.dumps(best))


if __name__ == "__main__":
    main()
