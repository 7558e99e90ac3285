"""Pins of the optional restoring flux of the order-parameter sum (reading
R23), CPU.

With sum_relax on, the variable part of the diffusion flux of phase i in
Eq. (36) gains m0 (phi_i / S) grad S, S = phi_1 + phi_2 + phi_3.  What that
must do, independent of how the oracle writes it:

* Summed over the phases the weights phi_i / S add up to one, so S obeys
  the linear diffusion equation with the mobility m0: a sine mode of S
  decays at m0 k^2 (second order in k), a large one generates no second
  harmonic, and with the flux off the mode stays put.
* Each phase receives its share phi_i / S: the fractions of a mixture whose
  phases are proportional to S stay fixed, an absent phase stays exactly
  zero, and every phase's mass is conserved (the flux enters through a
  source with zero zeroth moment).
* Where S = 1 the flux vanishes: a two-phase state built as phi and 1 - phi
  takes its first step as with the flux off.

Surface tensions are 1e-7 in the mode cases so that mu, and through it the
flow, stays at the 1e-8 level.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import Oracle
from paper_2608_05787_amd import inputs

M0 = (0.8 - 0.5) / 3.0


def _mode(v, L, m):
    x = np.arange(L)
    return 2.0 * np.mean(v * np.sin(2 * np.pi * m * x / L)), 2.0 * np.mean(v * np.cos(2 * np.pi * m * x / L))


def decay(L, amp=0.01, weights=(1.0, 0.0, 0.0), relax=1, lib=None, ny=2):
    """Run half an e-folding time of a sine mode of S; return the measured
    rate over m0 k^2 and the fields before and after."""
    p = inputs.base_params(L, ny, gamma12=1e-7, gamma13=1e-7, gamma23=1e-7, sigma=(0.0, 0.0, 0.0),
                           sum_relax=relax)
    x = np.arange(L)
    e = amp * np.sin(2 * np.pi * x / L)[None, :].repeat(ny, 0)
    o = Oracle(p, {"phi0": np.stack([w * (1.0 + e) for w in weights])}, lib_path=lib)
    before = np.stack([o.field("phi%d" % i) for i in (1, 2, 3)])
    k = 2 * np.pi / L
    T = int(0.5 / (M0 * k * k))
    o.step(T)
    after = np.stack([o.field("phi%d" % i) for i in (1, 2, 3)])
    a0 = _mode(before.sum(0)[0] - 1.0, L, 1)[0]
    a1 = _mode(after.sum(0)[0] - 1.0, L, 1)[0]
    return -np.log(a1 / a0) / T / (M0 * k * k), before, after


def test_sum_mode_decays_at_mobility():
    r = {L: decay(L)[0] for L in (16, 32, 64)}
    print("rate / m0 k^2:", r)
    for L in (16, 32, 64):
        assert abs(r[L] - 1.0) < 16.0 / L ** 2, (L, r[L])
    assert 3.2 < abs(r[16] - 1) / abs(r[32] - 1) < 5.0   # second order in k
    assert 3.2 < abs(r[32] - 1) / abs(r[64] - 1) < 5.0


def test_sum_mode_stays_without_flux():
    r, _, _ = decay(32, relax=0)
    assert abs(r) < 1e-4, r


def test_large_mode_generates_no_harmonic():
    L = 32
    r, _, after = decay(L, amp=0.3)
    s = after.sum(0)[0] - 1.0
    a1, a2 = np.hypot(*_mode(s, L, 1)), np.hypot(*_mode(s, L, 2))
    print("rate ratio %.6f, harmonic 2 / fundamental %.2e" % (r, a2 / a1))
    assert abs(r - 1.0) < 16.0 / L ** 2
    assert a2 / a1 < 1e-5


def test_shares_absent_phase_and_masses():
    """Phases 1 and 2 in proportion 0.3 : 0.7 times a sine mode of S, phase
    3 absent."""
    L = 32
    r, before, after = decay(L, amp=0.05, weights=(0.3, 0.7, 0.0))
    assert abs(r - 1.0) < 16.0 / L ** 2
    assert np.abs(after[0] / after.sum(0) - 0.3).max() < 1e-6
    assert np.all(after[2] == 0.0)  # exactly
    for i in range(2):
        assert abs(after[i].sum() - before[i].sum()) <= 1e-12 * before[i].sum()


def test_printed_scheme_where_sum_is_one():
    """A drop of phase 2 in phase 1 (phase 3 absent), built as phi and
    1 - phi: the first step, whose collision sees S = 1 to rounding, gives
    the same populations with and without the flux."""
    n = 24
    phi2 = inputs.tanh_drop(n, n, 11.3, 12.1, 6.0, 4.0)
    phi0 = np.stack([1.0 - phi2, phi2, np.zeros_like(phi2)])
    outs = []
    for relax in (0, 1):
        p = inputs.base_params(n, n, gamma12=2e-3, gamma13=2e-3, gamma23=2e-3, sigma=(0.0, 0.0, 0.0),
                               sum_relax=relax)
        o = Oracle(p, {"phi0": phi0})
        o.step(1)
        outs.append(o.pops("f"))
    assert np.abs(outs[0] - outs[1]).max() < 1e-15


# planted mistakes in the oracle's restoring flux, each failing a pin above
_OLD = "  return s->m0 * ph[i] / (ph[0] + ph[1] + ph[2]) * gS;"
MUTANTS = {
    "sign": (_OLD, "  return -s->m0 * ph[i] / (ph[0] + ph[1] + ph[2]) * gS;"),
    "no_division": (_OLD, "  return s->m0 * ph[i] * gS;"),
    "equal_shares": (_OLD, "  return s->m0 / 3.0 * gS;"),
    "double": (_OLD, "  return 2.0 * s->m0 * ph[i] / (ph[0] + ph[1] + ph[2]) * gS;"),
}


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("sum_mutants"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_planted_mistake(name, mutant_dir):
    old, new = MUTANTS[name]
    src = oracle.source_text()
    assert src.count(old) == 1
    lib = oracle.compile_variant(src.replace(old, new), os.path.join(mutant_dir, name + ".so"))
    if name in ("sign", "double"):
        r, _, _ = decay(16, lib=lib)
        assert not abs(r - 1.0) < 16.0 / 16 ** 2, r
    elif name == "no_division":
        L = 32
        _, _, after = decay(L, amp=0.3, lib=lib)
        s = after.sum(0)[0] - 1.0
        assert np.hypot(*_mode(s, L, 2)) / np.hypot(*_mode(s, L, 1)) > 1e-3
    else:
        _, _, after = decay(32, amp=0.05, weights=(0.3, 0.7, 0.0), lib=lib)
        assert np.abs(after[2]).max() > 1e-6
