"""Write oracle SCF results for the first 64 molecules of the 9-11-heavy-atom
benchmark batch (seed 2), the subset on which the mixed-precision results
are compared with the FP64 oracle.

Calls only the FP64 CPU oracle (oracle/) and the input generator; run from
the repository root:  python tests/golden/make_golden_subset.py [threads]
(about an hour of CPU time; one molecule per thread).
"""
import concurrent.futures as cf
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2311_01135_amd import molgen  # noqa: E402

SEED, HEAVY, N_SUBSET = 2, (9, 11), 64


def solve(idx):
    z, x = molgen.batch(1, SEED, HEAVY, start=idx)[0]
    r = O.Mol(z, x).scf(xc=O.XC_B3LYP)
    return dict(index=idx, n_atoms=int(len(z)), nbf=len(r["eps"]), E=r["E"], homo=r["homo"], lumo=r["lumo"],
                gap=r["gap"], n_iter=r["n_iter"], status=r["status"])


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(threads) as ex:
        out = list(ex.map(solve, range(N_SUBSET)))
    doc = {"source": "FP64 CPU oracle (oracle/ks_oracle.c), B3LYP (VWN RPA)/STO-3G, grid 50x12x24 with Becke "
                     "weights, atomic-occupation guess, DIIS(8), dE < 1e-9 Ha and commutator < 1e-7; molecules "
                     "0..63 of molgen.batch(seed 2, 9-11 heavy atoms); written by "
                     "tests/golden/make_golden_subset.py",
           "seed": SEED, "heavy": list(HEAVY), "molecules": out}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_scf_seed2_first64.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
