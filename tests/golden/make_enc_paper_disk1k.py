"""Writes enc_paper_disk1k.json: 90 encounter steps of the paper's 1k
benchmark disk (Sec. 3: the cold planetesimal disk of 1,000 bodies, 0.5-year
steps, shells of ratio 2.08, M = 4) integrated by the encounter-step oracle
alone, with the relative energy error of the split Hamiltonian, the smallest
pair separation and the number of flagged pairs every 10 steps.

The GPU test runs the same 90 steps from the same seeded disk and compares the
three series: over this span the two trajectories stay together to rounding
(the first approach that no shell resolves comes at step 91-100, after it the
energy error jumps to about 1.6e-4 on both sides and the series are not
compared).  Takes about a minute on one core.

    python -m tests.golden.make_enc_paper_disk1k
"""
import json
import os

import numpy as np

from oracle import symba_enc as E
from paper_2304_07325_amd import diskgen as dg

STEPS = 90
EVERY = 10
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "enc_paper_disk1k.json")


def split_energy(s):
    """Energy of the split Hamiltonian (heliocentric positions, barycentric
    velocities, G = 1, unit solar mass) and the smallest pair separation."""
    x = np.stack([s["x"], s["y"], s["z"]], 1)
    v = np.stack([s["vx"], s["vy"], s["vz"]], 1)
    m = np.asarray(s["m"], dtype=np.float64)
    p = (m[:, None] * v).sum(0)
    e = float(np.sum(0.5 * m * np.sum(v * v, 1) - m / np.linalg.norm(x, axis=1)) + 0.5 * p @ p)
    d = x[:, None, :] - x[None, :, :]
    r = np.sqrt(np.sum(d * d, -1))
    iu = np.triu_indices(len(m), 1)
    return e - float(np.sum((m[:, None] * m[None, :])[iu] / r[iu])), float(r[iu].min())


def main():
    w = dg.WORKLOADS["disk1k"]
    disk = dg.make_disk(w["n"], w["n_massive"], w["kind"], w["seed"])
    s = {k: np.asarray(v, dtype=np.float64) for k, v in disk.state(0).items()}
    n_m, h, f = w["n_massive"], dg.DT_HALF_YEAR, dg.RCRIT_FACTOR
    e0, _ = split_energy(s)
    acc, pairs = E.prepare(s, n_m, h, f)
    rows = []
    for k in range(1, STEPS + 1):
        s, acc, pairs = E.step(s, n_m, h, f, acc, pairs)
        if k % EVERY == 0:
            e, rmin = split_energy(s)
            rows.append({"step": k, "energy_rel_err": abs(e - e0) / abs(e0), "min_separation": rmin,
                         "n_pairs": int(len(pairs))})
            print(rows[-1], flush=True)
    doc = {"source": "oracle/symba_enc.py step() from diskgen disk1k (seed %d), written by "
                     "tests/golden/make_enc_paper_disk1k.py" % w["seed"],
           "disk": "disk1k", "n": w["n"], "n_massive": n_m, "h": h, "rcrit_factor": f, "checkpoints": rows}
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)


if __name__ == "__main__":
    main()
