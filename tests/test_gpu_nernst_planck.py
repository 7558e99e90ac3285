"""The two-ion Nernst-Planck charge model (Eq. 52) on the GPU, through the
C ABI: parity with the FP64 oracle on D2Q9 and D3Q15 (FP64 to rounding, FP32
within the per-field bounds of the leaky-dielectric tests), the
electro-osmotic channel against the Debye-Hueckel profiles of Eq. (53),
forward-mode gradients against finite differences, and the refused
combinations."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from oracle import Oracle  # noqa: E402
from paper_2608_05787_amd import binding, inputs  # noqa: E402

from test_gpu_parity import FP32_TOL, FP64_TOL, rel_err  # noqa: E402

# the ion charge e (n_+ - n_-) is a difference of two O(1) concentrations:
# measured 5.3e-6 element-wise after 12 FP32 steps
FP32_TOL = dict(FP32_TOL, q=1.5e-5)

pytestmark = pytest.mark.gpu

FIELDS_NP = ["phi1", "phi2", "phi3", "rho", "ux", "uy", "p", "psi", "Ex", "Ey", "q",
             "mu1", "mu2", "mu3", "eps", "R", "n_plus", "n_minus"]


def compare_np(sim, ref, tol, names):
    metric = rel_err  # element-wise, relative to the largest magnitude
    if isinstance(tol, dict):
        tol = dict(tol, n_plus=tol["phi1"], n_minus=tol["phi1"], uz=tol["ux"], Ez=tol["Ex"])
    got = {k: v.cpu().numpy() for k, v in sim.fields(names).items()}
    errs = {k: metric(got[k], ref.field(k)) for k in names}
    for fam in "fglh":
        errs["pop_" + fam] = metric(sim.populations(fam).cpu().numpy(), ref.pops(fam))
    lim = (lambda k: tol[k]) if isinstance(tol, dict) else (lambda k: tol)
    print("max-norm errors", " ".join("%s=%.1e" % kv for kv in errs.items()), flush=True)
    bad = {k: v for k, v in errs.items() if not v <= lim(k)}
    assert not bad, (bad, errs)


@pytest.mark.parametrize("nx,ny,walls", [(11, 9, True), (37, 29, False), (130, 70, True)])
def test_np_fp64_matches_oracle(nx, ny, walls):
    print("case np fp64", nx, ny, walls, flush=True)
    p, init = inputs.np_parity_case(nx, ny, seed=nx, walls=walls)
    ref = Oracle(p, init)
    sim = binding.Sim(p, init, precision="fp64")
    compare_np(sim, ref, FP64_TOL, FIELDS_NP)
    ref.step(8)
    sim.step(8)
    compare_np(sim, ref, FP64_TOL, FIELDS_NP)


def test_np_fp32_matches_oracle():
    print("case np fp32", flush=True)
    p, init = inputs.np_parity_case(64, 48, seed=3)
    ref = Oracle(p, init)
    sim = binding.Sim(p, init, precision="fp32")
    ref.step(10)
    sim.step(10)
    compare_np(sim, ref, FP32_TOL, FIELDS_NP)


def test_np_d3q15_fp64_matches_oracle():
    print("case np d3q15", flush=True)
    p, init = inputs.np_parity_case(11, 10, 7, seed=5)
    ref = Oracle(p, init)
    sim = binding.Sim(p, init, precision="fp64")
    names = FIELDS_NP + ["uz", "Ez"]
    ref.step(6)
    sim.step(6)
    compare_np(sim, ref, FP64_TOL, names)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_np_eof_channel_debye_hueckel(prec):
    """Steady electro-osmotic flow of the two-ion electrolyte: u, psi and q
    against Eq. (53); ion numbers conserved."""
    print("case np eof", prec, flush=True)
    p, init, m = inputs.np_eof_channel(nx=4, ny=32)
    sim = binding.Sim(p, init, precision=prec)
    n0 = {k: float(v.sum()) for k, v in sim.fields(["n_plus", "n_minus"]).items()}
    sim.step(12000)
    f = {k: v.cpu().numpy()[:, 0] for k, v in sim.fields(["ux", "psi", "q", "n_plus", "n_minus"]).items()}
    yc = np.arange(32) - 15.5
    c = np.cosh(m["kappa"] * yc) / math.cosh(m["kappa"] * m["h"])
    u_ex = -(m["eps"] * m["zeta"] * m["E"] / m["mu"]) * (1 - c)
    q_ex = -m["eps"] * m["kappa"] ** 2 * m["zeta"] * c
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)  # noqa: E731
    e = (rel(f["ux"], u_ex), rel(f["psi"], m["zeta"] * c), rel(f["q"], q_ex))
    assert e[0] < 4e-3 and e[1] < 2e-2 and e[2] < 6e-3, e
    tol = 1e-11 if prec == "fp64" else 1e-4
    for k, v in sim.fields(["n_plus", "n_minus"]).items():
        assert abs(float(v.sum()) / n0[k] - 1) < tol, k


def test_np_tangent_gradient_matches_fd():
    """Forward mode runs the Nernst-Planck kernels in tangent arithmetic:
    dJ/d(eps ratios, E0) against central differences of FP64 runs (the
    conductivity directions vanish: sigma = 0 scales to 0)."""
    print("case np tangent", flush=True)
    p, init = inputs.np_parity_case(24, 20, seed=7, sub=(2, 2, 0.0))
    steps = 10
    rng = np.random.default_rng(2)
    seed = {k: rng.standard_normal((20, 24)) for k in ("q", "n_plus", "ux")}
    g = np.array(binding.Sim(p, init, precision="fp64").tangent_gradient(
        steps, {k: torch.from_numpy(v) for k, v in seed.items()}))

    def J(cfg, ini):
        s = binding.Sim(cfg, ini, precision="fp64")
        s.step(steps)
        f = s.fields(list(seed))
        return sum(float((f[k].cpu().numpy() * v).sum()) for k, v in seed.items())

    th = inputs.theta_of(dict(p, sigma=(1.0, 1.0, 1.0)))  # sigma ratios unused here
    for k in (0, 1, 4):
        h = 1e-3 * th[k]
        tp, tm = list(th), list(th)
        tp[k] += h
        tm[k] -= h
        cp, ip = inputs.with_theta(p, init, tp)
        cm, im = inputs.with_theta(p, init, tm)
        for c in (cp, cm):
            c["sigma"] = (0.0, 0.0, 0.0)
        fd = (J(cp, ip) - J(cm, im)) / (2 * h)
        assert abs(g[k] - fd) <= 1e-4 * abs(fd) + 1e-9, (k, g[k], fd)
    assert g[2] == 0.0 and g[3] == 0.0


def test_np_refusals():
    p, init = inputs.np_parity_case(12, 10, seed=1)
    with pytest.raises(binding.LbmEhdError):
        binding.Sim(p, init, precision="fp16s")
    with pytest.raises(binding.LbmEhdError):
        binding.Sim(dict(p, sigma=(1e-3, 1e-3, 1e-3)), init, precision="fp32")
    no_ions = dict(init)
    no_ions.pop("ions0")
    with pytest.raises(binding.LbmEhdError):
        binding.Sim(p, no_ions, precision="fp32")
    sim = binding.Sim(p, init, precision="fp64")
    with pytest.raises(binding.LbmEhdError):
        sim.record(4, 2)
    leaky, linit = inputs.parity_case(12, 10, seed=1)
    with pytest.raises(binding.LbmEhdError):
        binding.Sim(leaky, linit, precision="fp32").fields(["n_plus"])
