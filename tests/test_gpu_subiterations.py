"""Potential sub-iterations per step, measured on the field-driven compound
drop at 1024^2 (the benchmark workload, FP32), over 10,000 steps.

Runs with fixed counts K = 4, 8, 16, 32 and 64, and with the residual-
controlled loop at tolerance 1e-7 (stop once the relative L2 change of the
potential over an iteration is below it).  Reported every 2000 steps: the
Sec. 4.4 deformation of each run, its distance from the K = 64 run, the
loop's mean iteration count and the fixed counts' last-iteration change.

A small change per iteration does not mean a converged potential: the
iteration contracts slowly on the box's long modes, so the remaining error
is the change divided by one minus the contraction rate, and the potential
carried from step to step lags the charge by a fixed fraction of its
per-step change.  The checks: the deformation converges as K grows (each
doubling brings it closer to K = 64), and K = 4 stays within the bound
below of K = 64 (measured; see the printed rows)."""
import json
import os

import pytest

torch = pytest.importorskip("torch")
from paper_2608_05787_amd import binding, inputs  # noqa: E402

pytestmark = pytest.mark.gpu

STEPS, EVERY, TOL = 10000, 2000, 1e-7
KS = (4, 8, 16, 32, 64)


def _run(p, init):
    sim = binding.Sim(p, init, precision="fp32")
    rows, k_prev = [], 0
    for t in range(EVERY, STEPS + 1, EVERY):
        sim.step(EVERY)
        d = sim.diagnostics()
        assert d["status"] == 0, (t, d["status"])
        tot = sim.scalars()["k_total"]
        rows.append(dict(step=t, D_outer=d["D_outer"], D_inner=d["D_inner"], residual=d["residual"],
                         mean_k=(tot - k_prev) / EVERY))
        k_prev = tot
    del sim
    torch.cuda.empty_cache()
    return rows


def test_deformation_converges_in_subiterations():
    print("case sub-iterations K sweep", flush=True)
    p, init = inputs.field_compound_drop(1024, sub=(4, 4, 0.0), init_iters=4000, init_tol=0.0)
    runs = {}
    for K in KS:
        runs["K%d" % K] = _run(dict(p, sub_min=K, sub_max=K), init)
        print("K", K, json.dumps(runs["K%d" % K][-1]), flush=True)
    runs["tol"] = _run(dict(p, sub_min=1, sub_max=64, sub_tol=TOL), init)
    print("tol", TOL, json.dumps(runs["tol"]), flush=True)
    ref = runs["K64"]
    table = []
    for i, r in enumerate(ref):
        row = {"step": r["step"], "D_outer_K64": r["D_outer"], "D_inner_K64": r["D_inner"]}
        for name in ["K%d" % K for K in KS[:-1]] + ["tol"]:
            row["dD_outer_" + name] = abs(runs[name][i]["D_outer"] - r["D_outer"])
            row["dD_inner_" + name] = abs(runs[name][i]["D_inner"] - r["D_inner"])
        row["mean_k_tol"] = runs["tol"][i]["mean_k"]
        row["residual_K4"] = runs["K4"][i]["residual"]
        print(json.dumps(row), flush=True)
        table.append(row)
    out_dir = os.environ.get("LBM_EHD_RESULTS_DIR")
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        with open(os.path.join(out_dir, "subiterations_field_drop_1024.json"), "w") as f:
            json.dump({"runs": runs, "table": table}, f)
    last = table[-1]
    # convergence: each doubling of K brings D closer to K = 64
    for a, b in zip(KS[:-2], KS[1:-1]):
        assert last["dD_outer_K%d" % b] < last["dD_outer_K%d" % a], last
        assert last["dD_inner_K%d" % b] < last["dD_inner_K%d" % a], last
    for r in table:
        assert r["dD_outer_K4"] < 5e-4 and r["dD_inner_K4"] < 5e-4, r
