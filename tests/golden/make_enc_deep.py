"""Writes enc_deep.json: one encounter step of a tight binary and of a tight
triple (tests/test_gpu_enc.py `_binary` and `_triple`: bodies 2e-5 and
1.5e-4 AU apart, inside the deepest shell for the whole step, so the
recursion takes every substep down to level 8, 87,380 for the binary)
integrated by the encounter-step oracle alone: the state after the step, its
level-0 accelerations and pairs, and the same step from the input with one
coordinate moved by one ulp.  A binary that turns about 1,400 times in a step
carries a 1-ulp change of its input into differences of 1e-9 in position and
1e-6 in velocity, so the GPU test measures its own step against that spread.
About four minutes on one core.

    python -m tests.golden.make_enc_deep
"""
import json
import os

import numpy as np

from oracle import symba_enc as E
from paper_2304_07325_amd import diskgen as dg
from tests.test_gpu_enc import F, _binary, _triple

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "enc_deep.json")
CASES = {"binary": (_binary, 2, dg.DT_HALF_YEAR), "triple": (_triple, 3, 0.05)}


def main():
    doc = {"source": "oracle/symba_enc.py prepare() and step(), written by tests/golden/make_enc_deep.py",
           "rcrit_factor": F, "cases": {}}
    for name, (make, n_m, h) in CASES.items():
        s = make()
        acc, pairs = E.prepare(s, n_m, h, F)
        s1, acc1, pairs1 = E.step(s, n_m, h, F, acc, pairs)
        sp = dict(s)
        sp["x"] = np.array(s["x"], dtype=np.float64)
        sp["x"][0] = np.nextafter(sp["x"][0], np.inf)
        s2, acc2, _ = E.step(sp, n_m, h, F, acc, pairs)
        keys = ("x", "y", "z", "vx", "vy", "vz")
        doc["cases"][name] = {"n_m": n_m, "h": h,
                              "state": {k: [float(v) for v in np.asarray(s1[k])] for k in keys},
                              "spread": {k: float(np.abs(np.asarray(s1[k]) - np.asarray(s2[k])).max()) for k in keys},
                              "acc": np.asarray(acc1).tolist(),
                              "acc_spread": float(np.abs(np.asarray(acc1) - np.asarray(acc2)).max()),
                              "pairs": np.asarray(pairs1).tolist()}
        print(name, "done", flush=True)
    with open(OUT, "w") as fh:
        json.dump(doc, fh, indent=1)


if __name__ == "__main__":
    main()
