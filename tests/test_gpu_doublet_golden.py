"""The static doublet at its full length against a stored FP64 oracle run.

tests/golden/doublet_256_oracle.json was written by
tests/golden/make_doublet_golden.py, which calls only the oracle: the second
workload (256^2 periodic box, no field, phase-2 drop of radius 40 and
phase-3 drop of radius 30 at centre distance 55 in phase 1, surface
tensions 1e-3 / 1.2e-3 / 0.8e-3) for 20,000 steps.  It holds the phase
masses and max |sum phi - 1| every 5000 steps and every field's values at
256 seeded nodes at the end.

The FP64 instance must reproduce them to rounding (measured: <= 7e-13 of each
field's largest magnitude, max |sum phi - 1| to four digits at every
checkpoint).  FP32 is held to the bounds below, about three times the
measured errors (phi 2.2e-4, rho 1.7e-4, u 4.6e-3, p 1.5e-2, mu 4.9e-3,
relative to each field's largest magnitude: the equal-density doublet's
pressure and flow are ~1e-5 and its chemical potentials ~1e-4, so FP32
rounding of the populations is a visible share of them), and its phase
masses and order-parameter sum to the oracle's closely (sum: 7.752e-2
against 7.755e-2 after 20,000 steps)."""
import json
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2608_05787_amd import binding, inputs  # noqa: E402

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "doublet_256_oracle.json")
# FP32 after 20,000 steps, element-wise on the sampled nodes, relative to the
# field's max-norm
FP32_TOL = {"phi1": 6e-4, "phi2": 6e-4, "phi3": 6e-4, "rho": 5e-4, "ux": 1.5e-2, "uy": 1.5e-2, "p": 4e-2,
            "mu1": 1.5e-2, "mu2": 1.5e-2, "mu3": 1.5e-2}


def _run(prec, gold):
    p, init = inputs.static_doublet()
    sim = binding.Sim(p, init, precision=prec)
    hist = []
    for row in gold["history"]:
        sim.step(gold["every"])
        d = sim.diagnostics()
        assert d["status"] == 0, (prec, row["step"])
        hist.append((row, d))
    f = sim.fields(list(gold["samples"]))
    nodes = torch.tensor(gold["nodes"], device=f["phi1"].device)
    errs = {}
    for k, want in gold["samples"].items():
        got = f[k].reshape(-1)[nodes].cpu().numpy()
        errs[k] = float(np.abs(got - np.asarray(want)).max() / gold["norms"][k]["max"])
    return hist, errs


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_doublet_full_length_against_stored_oracle_run(prec):
    print("case doublet golden", prec, flush=True)
    gold = json.load(open(GOLD))
    hist, errs = _run(prec, gold)
    print("max-norm errors", " ".join("%s=%.1e" % kv for kv in errs.items()), flush=True)
    for row, d in hist:
        print("step %d max|sum-1| %.3e (oracle %.3e)" % (row["step"], d["max_sum_dev"], row["max_sum_dev"]),
              flush=True)
    if prec == "fp64":
        assert max(errs.values()) <= 1e-9, errs
        for row, d in hist:
            for i in range(3):
                assert abs(d["mass%d" % (i + 1)] - row["mass"][i]) <= 1e-9 * abs(row["mass"][i]), (row, d)
            assert abs(d["max_sum_dev"] - row["max_sum_dev"]) <= 1e-9
    else:
        bad = {k: v for k, v in errs.items() if not v <= FP32_TOL[k]}
        assert not bad, (bad, errs)
        for row, d in hist:
            for i in range(3):
                assert abs(d["mass%d" % (i + 1)] - row["mass"][i]) <= 1e-4 * abs(row["mass"][i]), (row, d)
            assert abs(d["max_sum_dev"] - row["max_sum_dev"]) <= 2e-4
