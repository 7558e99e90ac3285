"""Device-latched status of the C ABI (lbm_ehd_status, and the status code of
lbm_ehd_diagnostics): a residual-controlled potential loop that reaches its
cap reports LBM_EHD_ENOCONV once; a non-finite value formed while stepping
reports LBM_EHD_EDIVERGED until the handle is restored.  Both conditions are
forced from the host side (a cap of 2 with a tolerance no loop meets; a NaN
in the initial order parameters): every kernel still runs its normal,
bounded course."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_2608_05787_amd import binding, inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def test_potential_cap_latches_enoconv_once():
    print("case enoconv", flush=True)
    p, init = inputs.parity_case(40, 36, seed=3, sub=(1, 2, 1e-14))
    sim = binding.Sim(p, init, precision="fp64")
    assert sim.status() == (0, 0)  # the cold start does not latch
    sim.step(3)
    d = sim.diagnostics()
    assert d["status"] == binding.ENOCONV and d["k_sub"] == 2
    assert math.isfinite(d["mass1"]) and d["nonfinite"] == 0
    assert sim.status() == (0, 0)  # reported once, then cleared
    sim.step(1)
    assert sim.status() == (binding.ENOCONV, 2)
    # a loop that converges, and a fixed count, never latch it
    p2, init2 = inputs.parity_case(40, 36, seed=3, sub=(1, 200, 1e-3))
    ok = binding.Sim(p2, init2, precision="fp64")
    ok.step(3)
    assert ok.status() == (0, 0) and ok.diagnostics()["k_sub"] < 200
    fixed = binding.Sim(*inputs.parity_case(40, 36, seed=3, sub=(2, 2, 0.0)), precision="fp32")
    fixed.step(3)
    assert fixed.status() == (0, 0)


@pytest.mark.parametrize("prec", ["fp32", "fp16s", "fp64"])
def test_nonfinite_state_latches_ediverged(prec):
    print("case ediverged", prec, flush=True)
    p, init = inputs.parity_case(33, 17, seed=5)
    sim = binding.Sim(p, init, precision=prec)
    ck = sim.checkpoint()
    sim.step(2)
    assert sim.status() == (0, 0)
    bad = dict(init)
    phi0 = init["phi0"].copy()
    phi0[1, 8, 16] = np.nan
    bad["phi0"] = phi0
    sick = binding.Sim(p, bad, precision=prec)
    sick.step(2)
    rc, flags = sick.status()
    assert rc == binding.EDIVERGED and flags & 1
    assert sick.status()[0] == binding.EDIVERGED  # stays latched
    assert sick.diagnostics()["status"] == binding.EDIVERGED
    # a healthy handle restored from a healthy checkpoint is clean again
    sim.restore(ck)
    sim.step(1)
    assert sim.status() == (0, 0)
