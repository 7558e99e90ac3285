"""The C oracle against its brute-force second transcription (oracle/brute.py)
on grids of 8 x 8 and smaller, CPU only.

The two were written separately from the paper's Sec. 3 (push against pull
streaming, vector loops against per-node Python) with the same readings; a
transcription slip in either (an index, a sign, a dropped term) shows up as
a difference far above round-off.  Every field and population family is
compared after create and after several steps, with walls, electrodes,
shear, an applied field, charge, unequal properties, a residual-controlled
potential loop, the order-parameter sum relaxation from fields whose sum is
off one, a Dirichlet charge wall and frozen phases.
"""
import numpy as np
import pytest

from oracle import Oracle
from oracle.brute import Brute
from paper_2608_05787_amd import inputs as I

FIELDS = ["phi1", "phi2", "phi3", "rho", "ux", "uy", "p", "psi", "Ex", "Ey", "q", "mu1", "mu2", "mu3", "eps", "R"]


def _cases():
    p, init = I.parity_case(8, 8, seed=11)
    yield "walls_field_shear", p, init, 4
    p, init = I.parity_case(8, 8, seed=12, walls=False)
    yield "periodic_field", p, init, 4
    p, init = I.parity_case(7, 5, seed=13, sub=(3, 3, 0.0))
    yield "ragged_7x5_K3", p, init, 3
    p, init = I.parity_case(8, 8, seed=14, sub=(1, 6, 1e-3))
    yield "adaptive_potential", p, init, 3
    p, init = I.parity_case(8, 7, seed=15)
    p["sum_relax"] = 1
    rng = np.random.default_rng(15)
    init = dict(init, phi0=init["phi0"] * (1.0 + 0.03 * rng.standard_normal(init["phi0"].shape)))
    yield "sum_relax_off_one", p, init, 4
    p, init, _ = I.eof_channel(nx=3, ny=8, debye=2.0)
    p["init_sub_max"] = 50
    yield "frozen_dirichlet_charge", p, init, 5


@pytest.mark.parametrize("case", list(_cases()), ids=lambda c: c[0])
def test_oracle_equals_brute_force(case):
    name, p, init, steps = case
    o = Oracle(p, init)
    b = Brute(p, init)
    for stage in range(2):
        if stage:
            o.step(steps)
            b.step(steps)
        bf = b.fields()
        for k in FIELDS:
            got, want = np.asarray(bf[k]), o.field(k)
            scale = max(np.abs(want).max(), 1e-300)
            assert np.abs(got - want).max() <= 1e-12 * scale + 1e-300, (name, stage, k)
        for fam in "fglh":
            got, want = np.asarray(b.pops(fam)), o.pops(fam)
            scale = max(np.abs(want).max(), 1e-300)
            assert np.abs(got - want).max() <= 1e-12 * scale, (name, stage, fam)
