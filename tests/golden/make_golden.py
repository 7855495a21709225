"""Write oracle SCF results for sampled molecules of the benchmark workloads.

Calls only the FP64 CPU oracle (oracle/) and the input generator; run from
the repository root:  python tests/golden/make_golden.py
"""
import concurrent.futures as cf
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2311_01135_amd import molgen  # noqa: E402

# (name, seed, n_heavy spec, batch size, sampled indices)
SETS = [
    ("bench_9-11_seed2", 2, (9, 11), 256, [0, 1, 2, 3, 100, 255]),
    ("c1_9_seed1", 1, 9, 256, [0, 17]),
]


def solve(args):
    name, seed, heavy, nmol, idx = args
    z, x = molgen.batch(1, seed, heavy, start=idx)[0]
    r = O.Mol(z, x).scf(xc=O.XC_B3LYP)
    return dict(set=name, index=idx, E=r["E"], homo=r["homo"], lumo=r["lumo"], gap=r["gap"],
                n_iter=r["n_iter"], status=r["status"], nbf=len(r["eps"]))


def main():
    jobs = [(n, s, h, b, i) for n, s, h, b, idx in SETS for i in idx]
    with cf.ThreadPoolExecutor(min(len(jobs), os.cpu_count() or 1)) as ex:
        out = list(ex.map(solve, jobs))
    z, x = molgen.water(0)
    w = O.Mol(z, x).scf(xc=O.XC_B3LYP)
    doc = {"source": "FP64 CPU oracle (oracle/ks_oracle.c), B3LYP (VWN RPA)/STO-3G, grid 50x12x24 with Becke "
                     "weights, atomic-occupation guess, DIIS(8), dE < 1e-9 Ha and commutator < 1e-7; written "
                     "by tests/golden/make_golden.py",
           "water_seed0": dict(E=w["E"], gap=w["gap"], n_iter=w["n_iter"]),
           "molecules": out}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_scf_samples.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
