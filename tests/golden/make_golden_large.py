"""Write oracle SCF results for molecules with 20 heavy atoms (the integral
size range beyond the LDS-resident kernels: N ~ 130-142).

Calls only the FP64 CPU oracle (oracle/) and the input generator; run from
the repository root:  python tests/golden/make_golden_large.py
(several CPU-hours in total; one molecule per thread).
"""
import concurrent.futures as cf
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2311_01135_amd import molgen  # noqa: E402

SEED, N_HEAVY, INDICES = 4, 20, [0, 1]


def solve(idx):
    z, x = molgen.tree(N_HEAVY, SEED, idx)
    r = O.Mol(z, x).scf(xc=O.XC_B3LYP)
    return dict(seed=SEED, n_heavy=N_HEAVY, index=idx, E=r["E"], homo=r["homo"], lumo=r["lumo"], gap=r["gap"],
                n_iter=r["n_iter"], status=r["status"], nbf=len(r["eps"]))


def main():
    with cf.ThreadPoolExecutor(len(INDICES)) as ex:
        out = list(ex.map(solve, INDICES))
    doc = {"source": "FP64 CPU oracle (oracle/ks_oracle.c), B3LYP (VWN RPA)/STO-3G, grid 50x12x24 with Becke "
                     "weights, atomic-occupation guess, DIIS(8), dE < 1e-9 Ha and commutator < 1e-7; molecules "
                     "molgen.tree(20, 4, index); written by tests/golden/make_golden_large.py",
           "molecules": out}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_scf_large.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
