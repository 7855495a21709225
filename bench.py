"""Throughput benchmark: batched restricted B3LYP/STO-3G SCF solves on one GPU.

A step is one full pass of the hot path over one batch of synthetic molecules
(default 4096 molecules of 9-11 heavy C/N/O/F atoms plus H, the paper's
workload size, seed 2): batch creation
(host prep, uploads), one-electron integrals, Loewdin, grid and Becke
weights, ERIs, and SCF iterations (J/K, XC, Fock, DIIS, eigensolve, density)
until every molecule has converged, then the results (energies, orbital
energies, gaps, densities) copied to the host.

The headline value is the mixed-precision path (ERIs, J/K and XC in FP32);
the plain FP64 GPU path runs on the same inputs for the speed ratio and the
per-molecule energy/gap differences; for the default workload the first 64
molecules are also compared with stored oracle results.  The larger
integral-direct workload runs as
  --n-mol 64 --heavy 20-30 --seed 4 --direct --schwarz-tol 1e-10 --grid 75,18,36
The roofline entry is for the XC
kernel (the dominant one), timed live with HIP events on the batch stream.
The CPU baseline is the FP64 oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SCF solves/sec, 9–11 heavy atoms, FP32 vs FP64 (|ΔE|≤1e-4 Ha); p99 latency"
PEAK = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}   # MI355X dense MFMA TFLOP/s (FP64, FP32, bf16)
HBM_PEAK = 8000.0                      # GB/s
SCREENING = os.path.join(ROOT, "tests", "golden", "xc_screening_seed2.json")
COUNTERS = os.path.join(ROOT, "profiles", "counters_4096mol_9-11heavy_mixed.json")
CSRC = os.path.join(ROOT, "paper_2311_01135_amd", "csrc")
# kernel family -> (rocprofv3 kernel-name prefix, sources its code comes from)
COUNTER_KERNELS = {
    "xc": ("ks::xc_kernel<", ["k_xc.hip", "wave.h"]),
    "jk": ("ks::jk_class_kernel<", ["k_jk.hip", "jk_scatter.h", "wave.h"]),
    "eri": ("ks::eri_class_kernel<", ["k_ints.hip"]),
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n-mol", type=int, default=4096)
    p.add_argument("--heavy", type=str, default="9-11", help="n or lo-hi heavy atoms")
    p.add_argument("--seed", type=int, default=2)
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison pass")
    p.add_argument("--fp64-only", action="store_true", help="time the FP64 path as the main value")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample", type=int, default=0, help="molecules in the oracle sample (0 = one per thread)")
    p.add_argument("--jk-chunks", type=int, default=0)
    p.add_argument("--xc-chunks", type=int, default=0)
    p.add_argument("--serve-requests", type=int, default=20000, help="serving leg requests (0 = skip)")
    p.add_argument("--serve-saturation", type=int, default=4096,
                   help="requests of the saturated run that sets the Poisson arrival rate (first of the serving set)")
    p.add_argument("--no-configs", action="store_true", help="skip the water and 256 x 9-heavy-atom FP64 legs")
    p.add_argument("--grid", type=str, default="50,12,24", help="radial,theta,phi points per atom")
    p.add_argument("--coarse-grid", type=str, default="25,8,16",
                   help="radial,theta,phi of the coarse start grid (0,0,0 = none); results stay the main grid's")
    p.add_argument("--direct", action="store_true", help="integral-direct J/K (ERIs recomputed every iteration)")
    p.add_argument("--no-direct-leg", action="store_true",
                   help="skip the 64 x 20-30-heavy-atom integral-direct leg of the config legs")
    p.add_argument("--schwarz-tol", type=float, default=0.0, help="Schwarz screening threshold (0 = off)")
    p.add_argument("--basis", choices=["sto-3g", "6-31g"], default="sto-3g",
                   help="6-31G covers H, C, N, O: molecules with F are replaced by F-free trees of the same size")
    p.add_argument("--summarize-counters", default="",
                   help="no GPU: summarise the rocprofv3 counter directories under this path into the committed "
                        "profiles/ counter summary (workload from the other options)")
    p.add_argument("--summarize-command", default="", help="the profiling command, recorded in the summary")
    p.add_argument("--copy-calibration-mib", type=int, default=0,
                   help="run one plain streaming copy of this many MiB before the timed region (the reference "
                        "kernel that scales hardware byte counters)")
    return p.parse_args()


def _gen_chunk(job):
    from paper_2311_01135_amd import molgen
    n, seed, heavy, start, f_free = job
    if f_free:
        return molgen.batch_without(n, seed, heavy)
    return molgen.batch(n, seed, heavy, start=start)


def gen_batch(n, seed, heavy, f_free=False, workers=None):
    """molgen.batch(n, seed, heavy) generated in chunks on a process pool
    (each molecule has its own random stream, so the chunks give the same
    molecules); run before anything touches the GPU."""
    import concurrent.futures as cf
    import multiprocessing as mp
    if f_free:
        return _gen_chunk((n, seed, heavy, 0, True))
    workers = workers or max(1, min(16, os.cpu_count() or 1))
    step = max(64, (n + 4 * workers - 1) // (4 * workers))
    jobs = [(min(step, n - s0), seed, heavy, s0, False) for s0 in range(0, n, step)]
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
        out = []
        for part in ex.map(_gen_chunk, jobs):
            out += part
    return out


def heavy_range(s):
    if "-" in s:
        lo, hi = s.split("-")
        return (int(lo), int(hi))
    return int(s)


def xc_flops(nbf, ngrid, niter, ngridc=None, ncoarse=None, r_main=1.0, r_coarse=1.0):
    """Algorithmic XC GEMM flops: 2 G N^2 for X = Phi P plus 2 G N^2 for Phi^T W, per iteration
    (G of the coarse start grid for the iterations that ran on it); with r_main / r_coarse < 1 the
    screened count (the dense work of each grid scaled by its screened fraction)."""
    ngridc = ngridc or [0] * len(nbf)
    ncoarse = ncoarse or [0] * len(nbf)
    return float(sum(4.0 * n * n * (r_main * g * (it - ic) + r_coarse * gc * ic)
                     for n, g, it, gc, ic in zip(nbf, ngrid, niter, ngridc, ncoarse)))


def _sha(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def summarize_counters(d, out, workload):
    """Counter summary of a profiled benchmark run (rocprofv3 output
    directories under d: kt (kernel trace), pa/pb/pc (SQ counters), pf
    (FETCH_SIZE), pw (WRITE_SIZE), written with -o <name> --output-format
    csv): per kernel family its launches, average duration, HBM bytes per
    launch (each counter scaled by what it reads for the copy-calibration
    kernel), MFMA busy fraction, VALU floating-point operations and LDS
    statistics, with the hash of the sources the counters were taken on."""
    import csv
    import collections

    def rows(name):
        with open(os.path.join(d, name, name + "_counter_collection.csv")) as f:
            return list(csv.DictReader(f))

    agg = collections.defaultdict(lambda: collections.defaultdict(float))
    disp = collections.defaultdict(set)
    copy = {}
    owner = {}                 # a counter collected in several passes is taken from the first
    for pas in ("pa", "pb", "pc", "pf", "pw"):
        for r in rows(pas):
            k = r["Kernel_Name"]
            name = r["Counter_Name"]
            if owner.setdefault(name, pas) != pas:
                continue
            v = float(r["Counter_Value"])
            if "vectorized_elementwise_kernel" in k and "MulFunctor" in k:
                copy[name] = copy.get(name, 0.0) + v
                continue
            for fam, (prefix, _) in COUNTER_KERNELS.items():
                if k.startswith(prefix) or k.startswith("void " + prefix):
                    agg[fam][name] += v
                    disp[(fam, pas)].add(r["Dispatch_Id"])
    dur = collections.defaultdict(list)
    with open(os.path.join(d, "kt", "kt_kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            for fam, (prefix, _) in COUNTER_KERNELS.items():
                k = r["Kernel_Name"]
                if k.startswith(prefix) or k.startswith("void " + prefix):
                    dur[fam].append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    mib = workload.get("copy_calibration_mib", 1024)
    fetch_factor = mib * 1024.0 / copy["FETCH_SIZE"] if copy.get("FETCH_SIZE") else None
    write_factor = mib * 1024.0 / copy["WRITE_SIZE"] if copy.get("WRITE_SIZE") else None
    doc = dict(workload=workload, copy_calibration=dict(mib=mib, fetch_factor=fetch_factor, write_factor=write_factor),
               kernels={})
    n_iter = len(disp[("xc", "pa")]) or 1      # one XC launch per SCF iteration
    for fam, (prefix, srcs) in COUNTER_KERNELS.items():
        c = agg[fam]
        n = len(disp[(fam, "pa")]) or 1
        gui = c.get("GRBM_GUI_ACTIVE", 0.0) / 8.0           # summed over the 8 XCDs
        # launches per build: J/K runs two class-group kernels per iteration,
        # the ERIs six class kernels once
        per_build = n / n_iter if fam == "jk" else (n if fam == "eri" else 1)
        ent = dict(kernel=prefix, sources=srcs, source_sha256=_sha(srcs), launches_pmc=n, launches_per_build=per_build,
                   launches_trace=len(dur[fam]), avg_ms_trace=(sum(dur[fam]) / len(dur[fam]) / 1e6) if dur[fam] else None)
        if fetch_factor and "FETCH_SIZE" in c:
            ent["hbm_bytes_per_launch"] = (c["FETCH_SIZE"] * fetch_factor + c.get("WRITE_SIZE", 0.0) * write_factor) \
                * 1024.0 / max(1, len(disp[(fam, "pf")]))
        if gui:
            ent["mfma_busy_frac"] = c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (gui * 1024.0)
            ent["lds_busy_frac"] = c.get("SQ_LDS_IDX_ACTIVE", 0.0) / (gui * 256.0)
            ent["lds_bank_conflict_frac"] = c.get("SQ_LDS_BANK_CONFLICT", 0.0) / (gui * 256.0)
            ent["valu_issue_frac"] = 4.0 * c.get("SQ_INSTS_VALU", 0.0) / (gui * 1024.0)
        fl32 = 64.0 * (2 * c.get("SQ_INSTS_VALU_FMA_F32", 0.0) + c.get("SQ_INSTS_VALU_MUL_F32", 0.0)
                       + c.get("SQ_INSTS_VALU_ADD_F32", 0.0))
        fl64 = 64.0 * (2 * c.get("SQ_INSTS_VALU_FMA_F64", 0.0) + c.get("SQ_INSTS_VALU_MUL_F64", 0.0)
                       + c.get("SQ_INSTS_VALU_ADD_F64", 0.0))
        npc = max(1, len(disp[(fam, "pc")]))
        ent["valu_flops_per_launch"] = dict(f32=fl32 / npc, f64=fl64 / npc,
                                            transcendental_lane_ops=64.0 * (c.get("SQ_INSTS_VALU_TRANS_F32", 0.0)
                                                                            + c.get("SQ_INSTS_VALU_TRANS_F64", 0.0)) / npc)
        ent["mfma_flops_per_launch"] = 512.0 * (c.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0)
                                                + c.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0)
                                                + c.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0)) / n
        ent["counters_per_launch"] = {k: v / n for k, v in sorted(c.items())}
        doc["kernels"][fam] = ent
    with open(out, "w") as f:
        json.dump(doc, f, indent=1)
    return doc


def counters_for(args, fam):
    """The committed counter summary of a kernel family, when it was taken on
    this workload and the kernel's current sources; else None."""
    if not os.path.exists(COUNTERS):
        return None
    with open(COUNTERS) as f:
        doc = json.load(f)
    w = doc.get("workload", {})
    if (w.get("n_mol") != args.n_mol or w.get("seed") != args.seed or w.get("heavy") != args.heavy
            or w.get("coarse_grid") != args.coarse_grid or args.basis != "sto-3g" or args.direct
            or args.schwarz_tol > 0 or grid_shape(args) != (50, 12, 24) or args.fp64_only):
        return None
    ent = doc.get("kernels", {}).get(fam)
    if not ent or ent.get("source_sha256") != _sha(ent["sources"]):
        return None
    return ent


def screened_ratio(args):
    """Ratio of the screened XC GEMM work sum_b G_b N_b^2 (N_b: AOs above
    1e-10 in 64-point block b) to the dense 4 G N^2, from the committed
    oracle-based estimate for the benchmark molecules; None for other
    workloads.  The kernel itself does the dense work."""
    if (not os.path.exists(SCREENING) or args.seed != 2 or heavy_range(args.heavy) != (9, 11)
            or args.basis != "sto-3g" or grid_shape(args) != (50, 12, 24)):
        return None
    if args.coarse_grid not in ("0,0,0", "25,8,16"):
        return None
    with open(SCREENING) as f:
        d = json.load(f)
    return dict(main=d["ratio_main"], coarse=d["ratio_coarse"],
                source="tests/golden/xc_screening_seed2.json (molecules 0-%d, tau %g, %d-point blocks)"
                % (len(d["molecules"]) - 1, d["tau"], d["block_points"]))


def copy_calibration(torch, mib):
    """One elementwise copy of mib MiB (reads and writes mib MiB each)."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst


def grid_shape(args):
    r, t, f = (int(v) for v in args.grid.split(","))
    return r, t, f


def oracle_subset(args, res, res64):
    """|dE|, |dgap| of the GPU results against stored oracle SCF results for
    the first molecules of the workload (tests/golden, written by a script
    that calls only the oracle), when the stored set is this workload's."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "golden",
                        "oracle_scf_seed2_first64.json")
    if (not os.path.exists(path) or args.direct or args.schwarz_tol > 0 or grid_shape(args) != (50, 12, 24)
            or args.basis != "sto-3g"):
        return None
    with open(path) as f:
        doc = json.load(f)
    if doc["seed"] != args.seed or tuple(doc["heavy"]) != heavy_range(args.heavy):
        return None
    ref = [m for m in doc["molecules"] if m["index"] < len(res)]
    if not ref:
        return None
    out = dict(n=len(ref), source="tests/golden/oracle_scf_seed2_first64.json")
    for name, rr in (("main", res), ("fp64_gpu", res64)):
        if rr is None:
            continue
        dE = np.array([abs(rr[m["index"]]["E"] - m["E"]) for m in ref])
        dg = np.array([abs(rr[m["index"]]["gap"] - m["gap"]) for m in ref])
        out[name] = dict(max_abs_dE=float(dE.max()), max_abs_dgap=float(dg.max()),
                         per_molecule_dE=[float(v) for v in dE])
    return out


def solve_batch(ks, mols, prec, timing, args):
    from paper_2311_01135_amd import autotune, molgen
    kw = dict(prec=prec)
    if args.basis == "6-31g":
        kw["basis"] = ks.KS_BASIS_631G
    else:
        kw.update(autotune.tuned_options(prec, [molgen.nbf_sto3g(z) for z, _ in mols]))
    if args.jk_chunks:
        kw["jk_chunks"] = args.jk_chunks
    if args.xc_chunks:
        kw["xc_chunks"] = args.xc_chunks
    kw["n_rad"], kw["n_theta"], kw["n_phi"] = grid_shape(args)
    kw.update(coarse_options(args))
    if args.direct:
        kw["direct"] = 1
    if args.schwarz_tol > 0:
        kw["schwarz_tol"] = args.schwarz_tol
    b = ks.Batch(mols, **kw)
    if timing:
        b.set_timing(True)
    b.scf_solve()
    res = b.results()                  # every molecule's E, eps, HOMO/LUMO, gap, P, status, iterations
    return b, res


def run_path(ks, torch, mols, prec, args, steps, warmup):
    for _ in range(warmup):
        b, _ = solve_batch(ks, mols, prec, False, args)
        b.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    times, last = [], None
    for s in range(steps):
        ts = time.perf_counter()
        b, res = solve_batch(ks, mols, prec, True, args)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        kt = b.kernel_times()
        nq = b.quartets()
        info = dict(nbf=list(b.nbf), ngrid=list(b.n_grid), quartets=nq, n_eri=list(b.n_eri),
                    n_atoms=[len(z) for z, _ in mols])
        b.close()
        last = (res, kt, info)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return total, times, last


def coarse_options(args):
    r, t, f = (int(v) for v in args.coarse_grid.split(","))
    return dict(coarse_rad=r, coarse_theta=t, coarse_phi=f)


def serve_run(ks, reqs, arrivals, prec, **options):
    """Drive a ks.Server with requests arriving at the given times (s); returns
    (wall seconds, latencies from scheduled arrival to observed completion,
    NaN for a rejected request, number rejected, iterations per request)."""
    srv = ks.Server(prec=prec, **options)
    n = len(reqs)
    lat = np.full(n, np.nan)
    iters = np.zeros(n, dtype=np.int64)
    pending = {}
    nxt, done, rejected = 0, 0, 0

    def collect(now):
        nonlocal done, rejected
        for tk in list(pending):
            try:
                r = srv.poll(tk)
            except ks.KsError:              # rejected at admission: done, with an error
                pending.pop(tk)
                done += 1
                rejected += 1
                continue
            if r is not None:
                i = pending.pop(tk)
                lat[i] = now - arrivals[i]
                iters[i] = r["n_iter"]
                done += 1

    t0 = time.perf_counter()
    while done < n:
        t = time.perf_counter() - t0
        while nxt < n and arrivals[nxt] <= t:
            z, x = reqs[nxt]
            pending[srv.submit(z, x)] = nxt
            nxt += 1
        st = srv.stats()
        if st["queued"] == 0 and st["resident"] == 0:
            collect(time.perf_counter() - t0)   # requests rejected while nothing was resident
            if done < n and nxt < n:
                time.sleep(max(0.0, min(0.01, arrivals[nxt] - (time.perf_counter() - t0))))
            elif done < n and not pending:
                raise RuntimeError("serving: %d requests neither finished nor pending" % (n - done))
            continue
        if srv.progress() > 0:
            collect(time.perf_counter() - t0)
    wall = time.perf_counter() - t0
    srv.close()
    return wall, lat, rejected, iters


def serving_leg(ks, args, reqs):
    """Serving workload: 3-11 heavy atoms (seed 3), mixed precision; the
    saturated throughput of the first requests submitted at once sets the
    rate, then all requests arrive as a Poisson stream at 0.8 x that rate."""
    n = len(reqs)
    ns = min(n, args.serve_saturation)
    wall_sat, _, rej_sat, _ = serve_run(ks, reqs[:ns], np.zeros(ns), ks.KS_MIXED, **coarse_options(args))
    sat = (ns - rej_sat) / wall_sat
    lam = 0.8 * sat
    rng = np.random.default_rng(3)
    arrivals = np.cumsum(rng.exponential(1.0 / lam, n))
    wall, lat, rej, iters = serve_run(ks, reqs, arrivals, ks.KS_MIXED, **coarse_options(args))
    ok = lat[np.isfinite(lat)]
    return dict(requests=n, heavy_atoms="3-11", precision="mixed", saturation_requests=ns,
                saturated_solves_per_s=sat, arrival_rate_per_s=lam, solves_per_s=len(ok) / wall,
                wall_s=wall, p50_latency_s=float(np.percentile(ok, 50)), p99_latency_s=float(np.percentile(ok, 99)),
                max_latency_s=float(ok.max()), rejected=int(rej + rej_sat),
                mean_iterations=float(iters[np.isfinite(lat)].mean()))


def config_legs(ks, torch, water, c1, big, args):
    """The other workloads: one water molecule (FP64, seed 0) solved alone,
    its time per solve and |dE|, |d gap| against the stored oracle result; a
    batch of 256 nine-heavy-atom molecules (FP64, seed 1) with its solves/s
    and ERI rates (main grid only, no coarse start, default options); and,
    when given, 64 molecules of 20-30 heavy atoms (seed 4) solved
    integral-direct in mixed precision with Schwarz screening at 1e-10 on the
    75 x 18 x 36 grid (with the 25 x 8 x 16 coarse start), one timed solve."""
    out = {}
    gold = os.path.join(ROOT, "tests", "golden", "oracle_scf_samples.json")
    with ks.Batch(water) as b:             # warm-up
        b.scf_solve()
    torch.cuda.synchronize()
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        with ks.Batch(water) as b:
            b.scf_solve()
            r = b.result(0)
        ts.append(time.perf_counter() - t0)
    w = dict(workload="water, B3LYP/STO-3G, FP64, grid 50x12x24, seed 0", s_per_solve_median=float(np.median(ts)),
             E=r["E"], gap=r["gap"], n_iter=r["n_iter"])
    if os.path.exists(gold):
        with open(gold) as f:
            g = json.load(f)["water_seed0"]
        w.update(abs_dE_vs_oracle=abs(r["E"] - g["E"]), abs_dgap_vs_oracle=abs(r["gap"] - g["gap"]),
                 oracle_n_iter=g["n_iter"])
    out["water"] = w
    from paper_2311_01135_amd import autotune, molgen
    opts = autotune.tuned_options(ks.KS_FP64, [molgen.nbf_sto3g(z) for z, _ in c1])
    with ks.Batch(c1, **opts) as b:        # warm-up
        b.scf_solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with ks.Batch(c1, **opts) as b:
        b.set_timing(True)
        b.scf_solve()
        res = b.results(density=False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kt = b.kernel_times()
        nq, nprim = b.quartets()
        neri = float(sum(b.n_eri))
    eri_ms = kt.get("eri", (float("nan"), 1))[0]
    out["fp64_256x9"] = dict(workload="256 molecules, 9 heavy atoms, B3LYP/STO-3G, FP64, grid 50x12x24, seed 1",
                             solves_per_s=len(c1) / wall, s_per_batch=wall,
                             iterations_mean=float(np.mean([x["n_iter"] for x in res])),
                             unconverged=int(sum(x["status"] != 1 for x in res)),
                             eri_unique_shell_quartets_per_s=nq / (eri_ms * 1e-3),
                             eri_unique_integrals_per_s=neri / (eri_ms * 1e-3), eri_ms=eri_ms)
    print("configs: water %.1f ms/solve |dE| %.1e; 256x9 FP64 %.1f solves/s"
          % (w["s_per_solve_median"] * 1e3, w.get("abs_dE_vs_oracle", float("nan")),
             out["fp64_256x9"]["solves_per_s"]), file=sys.stderr, flush=True)
    if big:
        kw = dict(prec=ks.KS_MIXED, direct=1, schwarz_tol=1e-10, n_rad=75, n_theta=18, n_phi=36,
                  coarse_rad=25, coarse_theta=8, coarse_phi=16)
        kw.update(autotune.tuned_options(ks.KS_MIXED, [molgen.nbf_sto3g(z) for z, _ in big]))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with ks.Batch(big, **kw) as b:
            b.set_timing(True)
            b.scf_solve()
            res = b.results(density=False)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            kt = b.kernel_times()
            nbf = list(b.nbf)
            ngrid = float(sum(b.n_grid))
        ms = {k: round(v[0], 3) for k, v in kt.items() if k in ("jk_direct", "xc", "eigh", "diis", "grid", "lowdin")}
        out["direct_64x20-30"] = dict(
            workload="64 molecules, 20-30 heavy atoms, seed 4, B3LYP/STO-3G, mixed precision, integral-direct J/K "
                     "with Schwarz screening 1e-10, grid 75x18x36 per atom, SCF started on a 25x8x16 coarse grid; "
                     "one timed solve",
            solves_per_s=len(big) / wall, s_per_batch=wall, nbf_min=min(nbf), nbf_max=max(nbf), grid_points=ngrid,
            iterations_mean=float(np.mean([x["n_iter"] for x in res])), iterations_max=int(max(x["n_iter"] for x in res)),
            coarse_grid_mean=float(np.mean([x["n_coarse"] for x in res])),
            unconverged=int(sum(x["status"] != 1 for x in res)), kernel_ms_avg=ms)
        print("configs: 64x20-30 direct %.2f solves/s (%.1f s per batch, %.1f iterations)"
              % (len(big) / wall, wall, out["direct_64x20-30"]["iterations_mean"]), file=sys.stderr, flush=True)
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(mols, args):
    from oracle import oracle as O
    O.lib()
    nthreads = max(1, min(16, os.cpu_count() or 1))
    n = args.cpu_sample or nthreads
    sample = mols[:n]
    out = [None] * len(sample)
    per = [0.0] * len(sample)

    def work(i):
        z, x = sample[i]
        t = time.perf_counter()
        out[i] = O.Mol(z, x).scf(xc=O.XC_B3LYP)
        per[i] = time.perf_counter() - t

    t0 = time.perf_counter()
    idx = list(range(len(sample)))
    lock = threading.Lock()

    def worker():
        while True:
            with lock:
                if not idx:
                    return
                i = idx.pop(0)
            work(i)

    th = [threading.Thread(target=worker) for _ in range(min(nthreads, len(sample)))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    wall = time.perf_counter() - t0
    return dict(value=len(sample) / wall, unit="solves/s", cores=min(nthreads, len(sample)), kind="oracle",
                cpu_model=cpu_model(), host_cpus=os.cpu_count(),
                median_s_per_molecule_one_thread=float(np.median(per)),
                sample="first %d molecules of the batch, full FP64 SCF each (integrals, grid, every iteration), "
                       "one per thread, %.1f s wall" % (len(sample), wall)), out


def main():
    args = parse()
    if args.summarize_counters:
        doc = summarize_counters(args.summarize_counters, COUNTERS,
                                 dict(n_mol=args.n_mol, seed=args.seed, heavy=args.heavy, precision="mixed",
                                      coarse_grid=args.coarse_grid, copy_calibration_mib=args.copy_calibration_mib
                                      or 1024, command=args.summarize_command))
        print(json.dumps({k: {kk: v[kk] for kk in v if kk != "counters_per_launch"}
                          for k, v in doc["kernels"].items()}, indent=1))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)
    from paper_2311_01135_amd import molgen
    # every input is generated before anything touches the GPU (process pool)
    heavy = heavy_range(args.heavy)
    t_gen = time.perf_counter()
    mols = gen_batch(args.n_mol, args.seed, heavy, f_free=args.basis == "6-31g")
    reqs = gen_batch(args.serve_requests, 3, (3, 11)) if args.serve_requests > 0 else []
    legs = not args.no_configs and args.basis == "sto-3g"
    water = [molgen.water(0)] if legs else []
    c1 = gen_batch(256, 1, 9) if legs else []
    big = gen_batch(64, 4, (20, 30)) if legs and not args.no_direct_leg else []
    print("generated %d + %d + %d + %d molecules in %.1f s" % (len(mols), len(reqs), len(c1), len(big),
                                                               time.perf_counter() - t_gen), file=sys.stderr, flush=True)

    import torch
    from paper_2311_01135_amd import ks

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    ks.load()

    main_prec = ks.KS_FP64 if args.fp64_only else ks.KS_MIXED
    if args.copy_calibration_mib:
        copy_calibration(torch, args.copy_calibration_mib)
    total, times, (res, kt, info) = run_path(ks, torch, mols, main_prec, args, args.steps, args.warmup)
    value = args.n_mol * args.steps / total
    print("main path: %.2f solves/s, %.2f s/step" % (value, total / args.steps), file=sys.stderr, flush=True)
    niter = [r["n_iter"] for r in res]
    ncoarse = [r["n_coarse"] for r in res]
    cg = [int(v) for v in args.coarse_grid.split(",")]
    ngridc = [n * cg[0] * cg[1] * cg[2] for n in info["n_atoms"]]
    status = [r["status"] for r in res]

    fp64 = None
    acc = None
    res64 = None
    if not args.no_fp64 and not args.fp64_only:
        t64, times64, (res64, kt64, _) = run_path(ks, torch, mols, ks.KS_FP64, args, 1, 0)
        dE = np.array([abs(a["E"] - b["E"]) for a, b in zip(res, res64)])
        dg = np.array([abs(a["gap"] - b["gap"]) for a, b in zip(res, res64)])
        it64 = [r["n_iter"] for r in res64]
        fp64 = dict(value=args.n_mol / t64, unit="solves/s", s_per_batch=t64,
                    iterations={"mean": float(np.mean(it64)), "max": int(max(it64)),
                                "coarse_grid_mean": float(np.mean([r["n_coarse"] for r in res64]))},
                    stopping="dE < 1e-9 Ha and commutator < 1e-7 (the mixed path stops at 1e-6 Ha and 1e-5, "
                             "the resolution of its FP32 Fock matrix)",
                    kernel_ms={k: v[0] for k, v in kt64.items()})
        acc = dict(max_abs_dE_vs_fp64_gpu=float(dE.max()), p99_abs_dE=float(np.percentile(dE, 99)),
                   max_abs_dgap_vs_fp64_gpu=float(dg.max()), n_over_1e4=int(((dE > 1e-4) | (dg > 1e-4)).sum()),
                   fp64_unconverged=int(sum(r["status"] != 1 for r in res64)))
        print("fp64 path: %.2f solves/s; max|dE| %.2e max|dgap| %.2e" % (fp64["value"], dE.max(), dg.max()),
              file=sys.stderr, flush=True)

    vs_oracle = oracle_subset(args, res, res64)
    if vs_oracle:
        print("vs oracle (%d molecules): main max|dE| %.2e max|dgap| %.2e"
              % (vs_oracle["n"], vs_oracle["main"]["max_abs_dE"], vs_oracle["main"]["max_abs_dgap"]),
              file=sys.stderr, flush=True)

    # roofline of the XC kernel (dominant), from the last timed step
    xc_ms, xc_launches = kt.get("xc", (float("nan"), 0))
    fl = xc_flops(info["nbf"], info["ngrid"], niter, ngridc, ncoarse)
    achieved = fl / max(1, xc_launches) / (xc_ms * 1e-3) / 1e12 if xc_launches else float("nan")
    dtype = "f64" if main_prec == ks.KS_FP64 else "f32"
    # against each contraction's own peak: X = Phi P on FP32 MFMAs, Phi^T W on
    # bf16-pair MFMAs in the mixed path (both FP64 in the FP64 path); the
    # bound is the time both halves take at their peaks
    half = fl / max(1, xc_launches) / 2.0
    pk2 = PEAK["bf16"] if dtype == "f32" else PEAK["f64"]
    t_bound = half / (PEAK[dtype] * 1e12) + half / (pk2 * 1e12)
    per_dtype = dict(x_phi_p=dtype, phit_w="bf16 pairs" if dtype == "f32" else "f64",
                     bound_ms=t_bound * 1e3, frac=t_bound / (xc_ms * 1e-3) if xc_launches else float("nan"))
    scr = screened_ratio(args)
    fls = xc_flops(info["nbf"], info["ngrid"], niter, ngridc, ncoarse, scr["main"], scr["coarse"]) if scr else None
    roof = dict(bound="mfma", kernel="xc_kernel", achieved=achieved, peak=PEAK[dtype], unit="TFLOP/s",
                frac=achieved / PEAK[dtype], per_dtype=per_dtype,
                screened=(dict(flops_per_launch=fls / max(1, xc_launches), ratio=fls / fl,
                               frac=achieved * (fls / fl) / PEAK[dtype], source=scr["source"]) if scr else None),
                traffic=(counters_for(args, "xc") or {}).get("hbm_bytes_per_launch"),
                mfma_busy_frac=(counters_for(args, "xc") or {}).get("mfma_busy_frac"),
                flops_per_launch=fl / max(1, xc_launches), avg_launch_ms=xc_ms, launches=xc_launches)

    # work rates of the other kernels, from the same live HIP-event timings:
    # ERIs (once per molecule; the grid runs beside them on a second stream),
    # J/K against its HBM roofline (the unique integrals streamed once per
    # active molecule-iteration, FP32 in the mixed path), Becke pairs
    es = 8 if main_prec == ks.KS_FP64 else 4
    eri_ms = kt.get("eri", (float("nan"), 1))[0]
    jk_ms, jk_n = kt.get("jk", (float("nan"), 0))
    grid_ms = kt.get("grid", (float("nan"), 1))[0]
    nq, nprim = info["quartets"]
    jk_bytes = float(sum(e * es * it for e, it in zip(info["n_eri"], niter))) / max(1, jk_n)
    jk_gbs = jk_bytes / (jk_ms * 1e-3) / 1e9 if jk_n else float("nan")
    jkd_ms, jkd_n = kt.get("jk_direct", (float("nan"), 0))
    # ERI VALU work from the committed counters (floating-point lane operations
    # of the class kernels per build), against this run's build time; J/K HBM
    # bytes and LDS statistics likewise
    ce, cj = counters_for(args, "eri"), counters_for(args, "jk")
    eri_fl = ((ce["valu_flops_per_launch"]["f32"] + ce["valu_flops_per_launch"]["f64"]) * ce["launches_per_build"]
              if ce else None)
    vpk = PEAK["f32"] if main_prec == ks.KS_MIXED else PEAK["f64"]
    rates = {
        "eri": dict(bound="valu", unique_shell_quartets_per_s=nq / (eri_ms * 1e-3),
                    primitive_quartets_per_s=nprim / (eri_ms * 1e-3),
                    unique_integrals_per_s=float(sum(info["n_eri"])) / (eri_ms * 1e-3), avg_launch_ms=eri_ms,
                    class_ms={c: kt[k][0] for c, k in (("ssss", "eri_ssss"), ("psss", "eri_psss"),
                                                        ("psps", "eri_psps"), ("ppss", "eri_ppss"),
                                                        ("ppps", "eri_ppps"), ("pppp", "eri_pppp")) if k in kt},
                    flops_per_build=eri_fl, achieved_tflops=(eri_fl / (eri_ms * 1e-3) / 1e12) if eri_fl else None,
                    peak_tflops=vpk, frac=(eri_fl / (eri_ms * 1e-3) / 1e12 / vpk) if eri_fl else None,
                    note="flops: VALU floating-point lane operations counted by rocprofv3 (2 per FMA) in the "
                         "class kernels, committed profile; time: this run's build, beside the grid kernel"),
        "jk": dict(bound="hbm", achieved=jk_gbs, peak=HBM_PEAK, unit="GB/s", frac=jk_gbs / HBM_PEAK,
                   bytes_per_launch=jk_bytes, avg_launch_ms=jk_ms, launches=jk_n,
                   traffic=(cj["hbm_bytes_per_launch"] * cj["launches_per_build"]
                            if cj and "hbm_bytes_per_launch" in cj else None),
                   lds_busy_frac=cj.get("lds_busy_frac") if cj else None,
                   lds_bank_conflict_frac=cj.get("lds_bank_conflict_frac") if cj else None),
        "jk_direct": dict(bound="valu", avg_launch_ms=jkd_ms, launches=jkd_n,
                          note="integral-direct: ERIs recomputed inside the digestion, nothing streamed") if jkd_n else None,
        "grid": dict(bound="valu", becke_pairs_per_s=float(sum(g * n * (n - 1) / 2 for g, n in
                                                                 zip(info["ngrid"], info["n_atoms"]))) / (grid_ms * 1e-3),
                     avg_launch_ms=grid_ms),
    }

    legs_out = None
    if legs:
        legs_out = config_legs(ks, torch, water, c1, big, args)

    serving = None
    if args.serve_requests > 0:
        serving = serving_leg(ks, args, reqs)
        print("serving: %.1f solves/s saturated, lambda %.1f/s, p50 %.3f s p99 %.3f s"
              % (serving["saturated_solves_per_s"], serving["arrival_rate_per_s"], serving["p50_latency_s"],
                 serving["p99_latency_s"]), file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu, _ = cpu_baseline(mols, args)

    total_time_per_step = total / args.steps
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total_time_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": "batch of %d synthetic saturated-tree molecules, %s heavy atoms {C,N,O,F}+H, "
                               "B3LYP/%s, grid %s per atom with Becke weights, DIIS(8), "
                               "converged at dE<1e-9 Ha & commutator<1e-7 (FP64) or dE<1e-6 Ha & "
                               "commutator<1e-5 (mixed) on that grid%s%s%s"
                               % (args.n_mol, args.heavy, "6-31G" if args.basis == "6-31g" else "STO-3G",
                                  "x".join(str(v) for v in grid_shape(args)),
                                  "" if args.coarse_grid == "0,0,0" else
                                  ", SCF started on a %s coarse grid" % args.coarse_grid.replace(",", "x"),
                                  ", integral-direct J/K" if args.direct else "",
                                  ", Schwarz screening %g" % args.schwarz_tol if args.schwarz_tol > 0 else ""),
                   "n_mol": args.n_mol, "seed": args.seed,
                   "nbf_range": [min(info["nbf"]), max(info["nbf"])],
                   "grid_points": int(sum(info["ngrid"])),
                   "coarse_grid": args.coarse_grid,
                   "precision": ("mixed: ERIs evaluated and stored in FP32 (prefactors formed in FP64); J/K "
                                 "digests FP32 integrals against the FP64 density with FP64 accumulation; XC in "
                                 "FP32 (AO values, X = Phi P on FP32 MFMAs, functional) with Phi^T W on bf16 split "
                                 "pairs (operands within 2^-17, FP32 accumulation) and E_xc summed in FP64; "
                                 "Loewdin, eigensolve, DIIS, Fock and energy in FP64")
                                if dtype == "f32" else "fp64"},
        "iterations": {"mean": float(np.mean(niter)), "max": int(max(niter)),
                       "coarse_grid_mean": float(np.mean(ncoarse))},
        "unconverged": int(sum(s != 1 for s in status)),
        "kernel_rates": rates,
        "kernel_ms_avg": {k: v[0] for k, v in kt.items()},
        "kernel_launches": {k: v[1] for k, v in kt.items()},
        "fp64": fp64,
        "accuracy": acc,
        "vs_oracle": vs_oracle,
        "configs": legs_out,
        "serving": serving,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
