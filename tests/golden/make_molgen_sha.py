"""Write tests/golden/molgen_sha.json: SHA-256 of the generated inputs that
the stored oracle results were computed on (the benchmark batch, the
nine-heavy-atom batch, the large-molecule batch, the serving requests and
water).  The generator holds no Kohn-Sham arithmetic; these pins only state
that the inputs behind the golden files have not moved."""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
from paper_2311_01135_amd import molgen  # noqa: E402

SETS = {
    # molecule i of a batch depends only on (seed, i), so a prefix is the
    # prefix of the full batch
    "bench_9-11_seed2_first64": lambda: molgen.batch(64, 2, (9, 11)),
    "c1_9_seed1_first32": lambda: molgen.batch(32, 1, 9),
    "direct_20-30_seed4_first4": lambda: molgen.batch(4, 4, (20, 30)),
    "serving_3-11_seed3_first64": lambda: molgen.batch(64, 3, (3, 11)),
    "water_seed0": lambda: [molgen.water(0)],
}


def digest(mols):
    h = hashlib.sha256()
    for z, x in mols:
        h.update(z.astype("<i4").tobytes())
        h.update(x.astype("<f8").tobytes())
    return h.hexdigest()


if __name__ == "__main__":
    out = {k: digest(f()) for k, f in SETS.items()}
    with open(os.path.join(HERE, "molgen_sha.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))
