"""Writes tests/golden/doublet_256_oracle.json from the FP64 oracle alone.

The static doublet of the second workload (256 x 256 periodic box, no field,
a phase-2 drop of radius 40 and a phase-3 drop of radius 30 at centre
distance 55 inside phase 1, surface tensions 1e-3 / 1.2e-3 / 0.8e-3,
interface width 4, equal densities, tau 0.8) run for 20,000 steps, the
workload's full length.  Every 5000 steps: the phase masses and
max |phi_1 + phi_2 + phi_3 - 1|; at the end, per-field max and L2 norms and
the values of every field at 256 seeded nodes.

Run: python tests/golden/make_doublet_golden.py   (a few minutes on 8 host cores)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle  # noqa: E402
from paper_2608_05787_amd import inputs  # noqa: E402

FIELDS = ["phi1", "phi2", "phi3", "rho", "ux", "uy", "p", "mu1", "mu2", "mu3"]


def main(steps=20000, every=5000):
    p, init = inputs.static_doublet()
    t0 = time.time()
    o = Oracle(p, init)
    rows = []
    for t in range(every, steps + 1, every):
        o.step(every)
        ph = np.stack([o.field("phi%d" % i) for i in (1, 2, 3)])
        rows.append(dict(step=t, mass=[float(v) for v in ph.sum(axis=(1, 2))],
                         max_sum_dev=float(np.abs(ph.sum(0) - 1.0).max())))
        print("step %d max|sum-1| %.3e (%.0f s)" % (t, rows[-1]["max_sum_dev"], time.time() - t0), flush=True)
    f = {k: o.field(k) for k in FIELDS}
    rng = np.random.default_rng(20000)
    nodes = rng.choice(p["nx"] * p["ny"], size=256, replace=False)
    out = dict(case="static doublet 256x256 (inputs.static_doublet defaults)", steps=steps, every=every,
               history=rows,
               norms={k: dict(max=float(np.abs(v).max()), l2=float(np.linalg.norm(v))) for k, v in f.items()},
               nodes=[int(n) for n in nodes],
               samples={k: [float(v.reshape(-1)[n]) for n in nodes] for k, v in f.items()},
               source="FP64 oracle (oracle/lbm_ehd_oracle.c), tests/golden/make_doublet_golden.py")
    with open(os.path.join(HERE, "doublet_256_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("written (%.0f s)" % (time.time() - t0))


if __name__ == "__main__":
    main()
