"""Conformer-batched data generation: the paper's workload (section 4) is
many non-equilibrium conformers per molecule, each solved for its energy,
HOMO, LUMO and gap.  Conformers of one molecule share the atoms, the basis
size and the shell layout, so a batch of them is uniform.

generate() draws n_mol saturated-tree molecules (molgen.batch), n_conf
torsion-sampled conformers of each (molgen.conformers), solves them on the
GPU in batches of up to batch_size geometries, and returns (and optionally
writes as JSON lines) one record per conformer:
{mol, conf, n_heavy, n_atoms, nbf, Z, xyz (Angstrom), E, homo, lumo, gap,
n_iter, status}.

    python -m paper_2311_01135_amd.generate --n-mol 4 --heavy 9-11 --n-conf 64 --out records.jsonl
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def generate(n_mol, heavy, n_conf, seed=0, prec=1, batch_size=256, out=None, log=None, **options):
    from paper_2311_01135_amd import ks, molgen
    mols = molgen.batch(n_mol, seed, heavy)
    geoms, tags = [], []
    for i, (z, x) in enumerate(mols):
        for k, (zz, xx) in enumerate(molgen.conformers(z, x, n_conf, seed, i)):
            geoms.append((zz, xx))
            tags.append((i, k))
    records = []
    t0 = time.perf_counter()
    for b0 in range(0, len(geoms), batch_size):
        part = geoms[b0:b0 + batch_size]
        with ks.Batch(part, prec=prec, **options) as b:
            b.scf_solve()
            for m, (z, x) in enumerate(part):
                r = b.result(m)
                i, k = tags[b0 + m]
                records.append(dict(mol=i, conf=k, n_heavy=int((z > 1).sum()), n_atoms=len(z), nbf=b.nbf[m],
                                    Z=[int(v) for v in z], xyz=[[float(c) for c in row] for row in x],
                                    E=r["E"], homo=r["homo"], lumo=r["lumo"], gap=r["gap"], n_iter=r["n_iter"],
                                    status=r["status"]))
        if log:
            log("solved %d / %d conformers (%.1f s)" % (min(b0 + batch_size, len(geoms)), len(geoms),
                                                       time.perf_counter() - t0))
    if out:
        with open(out, "w") as f:
            for r in records:
                f.write(json.dumps(r) + "\n")
    return records


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n-mol", type=int, default=4)
    ap.add_argument("--heavy", default="9-11", help="n or lo-hi heavy atoms")
    ap.add_argument("--n-conf", type=int, default=64)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--prec", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--batch-size", type=int, default=256)
    ap.add_argument("--out", default="records.jsonl")
    a = ap.parse_args()
    sys.path.insert(0, ROOT)
    import torch
    torch.cuda.set_device(0)
    lo, hi = (int(v) for v in a.heavy.split("-")) if "-" in a.heavy else (int(a.heavy),) * 2
    t0 = time.perf_counter()
    rec = generate(a.n_mol, (lo, hi) if lo != hi else lo, a.n_conf, a.seed, 1 if a.prec == "mixed" else 0,
                   a.batch_size, a.out, log=lambda s: print(s, flush=True))
    dt = time.perf_counter() - t0
    bad = sum(r["status"] != 1 for r in rec)
    print(json.dumps(dict(records=len(rec), seconds=dt, records_per_s=len(rec) / dt, unconverged=bad, out=a.out)))


if __name__ == "__main__":
    main()
