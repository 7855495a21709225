"""Write oracle SCF results with densities for the first molecules of the
9-11-heavy-atom benchmark batch (seed 2):

- molecules 0..2 at the default stopping rule (dE < 1e-9 Ha, commutator
  < 1e-7): energy, gap and the density P;
- molecules 0..7 converged tightly (dE < 1e-12 Ha, commutator < 1e-10),
  i.e. at the self-consistent fixed point to ~1e-10: energy, HOMO, LUMO,
  gap, and P for molecules 0..2.

Output: oracle_density_seed2.json (scalars) and oracle_density_seed2.npz
(densities, float64, keys P_default_<i>, P_tight_<i>).  Calls only the
FP64 CPU oracle (oracle/) and the input generator; run from the repository
root:  python tests/golden/make_golden_density.py [threads]
(a few minutes on 8 threads).
"""
import concurrent.futures as cf
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2311_01135_amd import molgen  # noqa: E402

SEED, HEAVY = 2, (9, 11)
N_P, N_TIGHT = 3, 8
TIGHT = dict(e_tol=1e-12, comm_tol=1e-10, max_iter=200)


def solve(job):
    idx, tight = job
    z, x = molgen.batch(1, SEED, HEAVY, start=idx)[0]
    r = O.Mol(z, x).scf(xc=O.XC_B3LYP, **(TIGHT if tight else {}))
    return idx, tight, r


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    jobs = [(i, True) for i in range(N_TIGHT)] + [(i, False) for i in range(N_P)]
    with cf.ThreadPoolExecutor(threads) as ex:
        out = list(ex.map(solve, jobs))
    doc = {"source": "FP64 CPU oracle (oracle/ks_oracle.c), B3LYP (VWN RPA)/STO-3G, grid 50x12x24 with Becke "
                     "weights, atomic-occupation guess, DIIS(8); molecules of molgen.batch(seed 2, 9-11 heavy "
                     "atoms); 'default': dE < 1e-9 Ha and commutator < 1e-7, 'tight': dE < 1e-12 Ha and "
                     "commutator < 1e-10; written by tests/golden/make_golden_density.py",
           "seed": SEED, "heavy": list(HEAVY), "default": [], "tight": []}
    arrays = {}
    for idx, tight, r in sorted(out, key=lambda t: (t[1], t[0])):
        key = "tight" if tight else "default"
        doc[key].append(dict(index=idx, nbf=len(r["eps"]), E=r["E"], homo=r["homo"], lumo=r["lumo"],
                             gap=r["gap"], n_iter=r["n_iter"], status=r["status"]))
        if idx < N_P:
            arrays["P_%s_%d" % (key, idx)] = r["P"]
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "oracle_density_seed2.json"), "w") as f:
        json.dump(doc, f, indent=1)
    np.savez_compressed(os.path.join(here, "oracle_density_seed2.npz"), **arrays)
    print("wrote oracle_density_seed2.json / .npz")


if __name__ == "__main__":
    main()
