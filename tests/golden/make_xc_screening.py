"""Screened XC work of the benchmark molecules: for the first molecules of
the 9-11-heavy-atom batch (seed 2), the grid in blocks of 64 consecutive
points (the XC kernel's sub-blocks), N_b = number of AOs whose value or
gradient exceeds tau = 1e-10 anywhere in block b, and the ratio
sum_b G_b N_b^2 / sum_b G_b N^2 of the screened to the dense GEMM work
(4 G N^2 per iteration), on the main 50x12x24 grid and on the 25x8x16
coarse start grid.

Calls only the FP64 CPU oracle (AO values and grid) and the input
generator; run from the repository root:
    python tests/golden/make_xc_screening.py [threads]
Writes tests/golden/xc_screening_seed2.json.
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

SEED, HEAVY, NMOL, BP, TAU = 2, (9, 11), 8, 64, 1e-10
GRIDS = {"main": (50, 12, 24), "coarse": (25, 8, 16)}


def one(idx):
    z, x = molgen.batch(1, SEED, HEAVY, start=idx)[0]
    o = O.Mol(z, x)
    N = o.nbf
    out = dict(index=idx, nbf=N)
    for name, (r, t, f) in GRIDS.items():
        g = o.grid(r, t, f)
        screened = dense = 0.0
        for c0 in range(0, len(g), BP * 256):
            ao = np.abs(o.ao(g[c0:c0 + BP * 256, :3])).max(axis=1)      # [points, N]
            for b0 in range(0, ao.shape[0], BP):
                blk = ao[b0:b0 + BP]
                nb = int((blk.max(axis=0) > TAU).sum())
                screened += blk.shape[0] * nb * nb
                dense += blk.shape[0] * N * N
        out[name] = dict(points=int(len(g)), screened=screened, dense=dense, ratio=screened / dense)
    return out


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else (os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(threads) as ex:
        mols = list(ex.map(one, range(NMOL)))
    doc = {"source": "FP64 CPU oracle AO values on its grids; molecules 0..%d of molgen.batch(seed 2, 9-11 heavy "
                     "atoms); written by tests/golden/make_xc_screening.py" % (NMOL - 1),
           "tau": TAU, "block_points": BP, "molecules": mols}
    for name in GRIDS:
        doc["ratio_" + name] = sum(m[name]["screened"] for m in mols) / sum(m[name]["dense"] for m in mols)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "xc_screening_seed2.json")
    with open(path, "w") as f:
        json.dump(doc, f, indent=1)
    print("wrote", path, doc["ratio_main"], doc["ratio_coarse"])


if __name__ == "__main__":
    main()
