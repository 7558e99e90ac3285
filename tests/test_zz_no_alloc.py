"""lbm_ehd_diagnostics_static (the diagnostics with their partial sums in the
library's static device buffer, for callers that cannot allocate) against
lbm_ehd_diagnostics, through the C ABI: bitwise the same outputs and return
codes on two calls in a row, the second on a smaller handle (the buffer
keeps the first call's partials), for a two-instance batch and a single
instance, in FP32 and FP64."""
import math

import pytest

torch = pytest.importorskip("torch")
from paper_2608_05787_amd import binding, inputs  # noqa: E402

pytestmark = pytest.mark.gpu


def _same(a, b):
    for k in binding.DIAG_KEYS + ["status"]:
        x, y = a[k], b[k]
        assert (math.isnan(x) and math.isnan(y)) or x == y, (k, x, y)


def test_static_diagnostics_equal_workspace_diagnostics():
    print("case no-alloc diagnostics", flush=True)
    big = [inputs.field_compound_drop(160, r_shell=30, r_core=20, init_iters=100, init_tol=0.0),
           inputs.parity_case(130, 70, seed=4, sub=(4, 4, 0.0))]
    big[1][0]["init_sub_max"] = 100  # a batch shares its sub-iteration settings
    a = binding.Sim([c[0] for c in big], [c[1] for c in big], precision="fp32")
    a.step(30)
    small = inputs.parity_case(40, 30, seed=6)
    b = binding.Sim(small[0], small[1], precision="fp64")
    b.step(5)
    # first call: the larger (two-instance) handle; second: the smaller one
    got_a = [a.diagnostics(i, static=True) for i in range(2)]
    got_b = b.diagnostics(0, static=True)
    for i in range(2):
        _same(got_a[i], a.diagnostics(i))
    _same(got_b, b.diagnostics(0))
    assert got_a[0]["status"] == 0 and abs(got_a[0]["D_outer"]) > 0
    # and again after more steps, the small handle first this time
    b.step(3)
    a.step(3)
    _same(b.diagnostics(0, static=True), b.diagnostics(0))
    _same(a.diagnostics(1, static=True), a.diagnostics(1))
