"""Writes tests/golden/field_drop_512_oracle.json from the FP64 oracle alone.

The field-driven compound drop (third workload's parameters: electrodes,
Ca_e = 0.2, eps ratios 2 / 0.5, sigma ratios 3 / 0.3, tau_l = 0.6, four
potential sub-iterations per step) on a 512 x 512 box with the shell and
core radii 40 and 30 of the adjoint workload, so that it deforms within a
few thousand steps.  Cold start: 2000 fixed potential iterations.  Every
500 steps the script records the Sec. 4.4 contour deformation factors and
the second-moment forms of the outer (1 - phi1) and inner (phi3) drops; at
the end, per-field max and L2 norms and the values of every field at 256
seeded nodes.

Run: python tests/golden/make_field_drop_golden.py [steps]   (about five
minutes on 8 host cores for the default 5000 steps).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import Oracle  # noqa: E402
from oracle.deformation import contour_deformation, moment_deformation  # noqa: E402
from paper_2608_05787_amd import inputs  # noqa: E402

FIELDS = ["phi1", "phi2", "phi3", "rho", "ux", "uy", "p", "psi", "Ex", "Ey", "q", "mu1", "mu2", "mu3", "eps", "R"]
CASE = dict(n=512, r_shell=40.0, r_core=30.0, init_iters=2000, init_tol=0.0, sub=(4, 4, 0.0))


def main(steps=5000, every=500):
    p, init = inputs.field_compound_drop(**CASE)
    t0 = time.time()
    o = Oracle(p, init)
    rows = []
    for t in range(every, steps + 1, every):
        o.step(every)
        w_out, w_in = 1.0 - o.field("phi1"), o.field("phi3")
        Do, rpo, rqo = contour_deformation(w_out, walls=True)
        Di, rpi, rqi = contour_deformation(w_in, walls=True)
        rows.append(dict(step=t, D_outer=Do, D_inner=Di, r_par_outer=rpo, r_perp_outer=rqo, r_par_inner=rpi,
                         r_perp_inner=rqi, D_outer_moment=moment_deformation(np.maximum(w_out, 0.0)),
                         D_inner_moment=moment_deformation(np.maximum(w_in, 0.0))))
        print("step %d D_outer %.6e D_inner %.6e (%.0f s)" % (t, Do, Di, time.time() - t0), flush=True)
    f = {k: o.field(k) for k in FIELDS}
    rng = np.random.default_rng(5787)
    nodes = rng.choice(CASE["n"] * CASE["n"], size=256, replace=False)
    out = dict(case=dict(CASE, sub=list(CASE["sub"])), steps=steps, every=every, deformation=rows,
               norms={k: dict(max=float(np.abs(v).max()), l2=float(np.linalg.norm(v))) for k, v in f.items()},
               nodes=[int(n) for n in nodes],
               samples={k: [float(v.reshape(-1)[n]) for n in nodes] for k, v in f.items()},
               source="FP64 oracle (oracle/lbm_ehd_oracle.c), tests/golden/make_field_drop_golden.py")
    with open(os.path.join(HERE, "field_drop_512_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("written (%.0f s)" % (time.time() - t0))


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 5000)
