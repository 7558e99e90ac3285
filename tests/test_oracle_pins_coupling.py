"""Pins of the oracle's electric, advective and viscous couplings.

CPU only.  Each pin measures the FP64 oracle against a closed form or an
exact property of the governing equations (27a)-(27e), at two resolutions
where the scheme's error should fall.  Each pin is also run on a copy of the
oracle source with one planted mistake (a dropped term, a flipped sign, a
wrong factor) and must reject it: `test_pin_rejects_planted_mistake` compiles
those copies into a temporary directory.

Pins:
  maxwell_jump        Eq. 20's electric term -eps'(phi_i)|E|^2/2 against the
                      Maxwell-stress jump of P = p + sum phi_i mu_i across a
                      flat dielectric layer in a normal field.
  leaky_layer         Eq. 47's gradient terms against current continuity
                      (sigma E equal in both bulk layers) and Gauss's law for
                      the interface charge, in a layered leaky dielectric.
  dielectric_layer    the applied-field reading R15 (Eq. 42 for the full
                      potential) against a continuous displacement D = eps E
                      in a periodic layered dielectric.
  translation         Eqs. 35-36 (advection c_j.(phi_i u) and the source
                      d_t(phi_i u)) against Galilean invariance: a compound
                      drop in uniform flow equals the resting drop shifted by
                      U t.
  two_layer_couette   Eq. 29 and the local tau_g (R6) against the bulk shear
                      rates of a two-layer Couette flow: mu_1 du_1 = mu_2 du_2.
  plug_fixed_point    the moving-wall bounce-back of f and l (R10): a uniform
                      state moving with the walls is a fixed point.
  charge_conservation Eq. 17 (sum q conserved): exactly with sigma = 0, to
                      truncation error (falling under refinement) otherwise.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import Oracle
from oracle.deformation import contour_deformation, moment_deformation
from paper_2608_05787_amd import inputs as I


# ------------------------------------------------------------ measurements

def _layer_masks(ny, lo, hi, W):
    y = np.arange(ny)
    inside = (y > lo + 3 * W) & (y < hi - 3 * W)
    outside = (y < lo - 3 * W) | (y > hi + 3 * W)
    return inside, outside


def maxwell_jump(scale=1, eps_in=0.4, lib=None):
    """Jump of P = p + sum phi_i mu_i from the host into a flat layer of
    phase 2 between electrodes, divided by the Maxwell-stress jump
    D^2/2 (1/eps_in - 1/eps_out) (D = eps E, uniform without charge).  The
    identity follows from the force -sum phi_i grad mu_i at rest:
    dP/dy = sum_i mu_i dphi_i/dy, whose electric part integrates to
    -1/2 int E^2 d eps."""
    ny, W = 96 * scale, 4.0 * scale
    lo, hi = 32.5 * scale, 63.5 * scale
    dV = 0.96 * scale
    phi0 = I.flat_layers(1, ny, lo, hi, W, phase=1)
    # initial potential guess: the quadrature of 1/eps over the layer (a
    # guess only; it speeds the cold start)
    band = phi0[1][:, 0]
    inv = 1.0 / (0.1 + (eps_in - 0.1) * band)
    cum = np.cumsum(inv) - 0.5 * inv
    psi0 = (dV * cum / inv.sum())[:, None]
    p = I.base_params(1, ny, bc_y=1, wall_phi=(0.0, dV), sigma=(0, 0, 0), eps=(0.1, eps_in, 0.1),
                      width=W, visc=(0.3, 0.3, 0.3), init_sub_max=4000 * scale * scale)
    o = Oracle(p, {"phi0": phi0, "psi0": psi0}, lib_path=lib)
    o.step(8000 * scale * scale)
    f = o.fields()
    P = (f["p"] + f["phi1"] * f["mu1"] + f["phi2"] * f["mu2"] + f["phi3"] * f["mu3"])[:, 0]
    inside, outside = _layer_masks(ny, lo, hi, W)
    D = (f["eps"] * f["Ey"])[:, 0]
    Dm = D[inside].mean()
    pred = 0.5 * Dm ** 2 * (1.0 / eps_in - 1.0 / 0.1)
    return (P[inside].mean() - P[outside].mean()) / pred


def layered_field(scale=1, eps_in=0.4, sig_in=4e-3, sig_out=1e-3, lib=None):
    """A layer of phase 2 in a box periodic in y under the applied field
    E_ext = (0, E0), order parameters frozen.  Returns the bulk fields, the
    charge around the lower interface and the steady-state residuals."""
    ny, W = 96 * scale, 4.0 * scale
    lo, hi = 24.5 * scale, 72.5 * scale
    s2 = scale * scale
    phi0 = I.flat_layers(1, ny, lo, hi, W, phase=1)
    p = I.base_params(1, ny, bc_y=0, E_ext=(0.0, 1e-3 / scale), eps=(0.1, eps_in, 0.1),
                      sigma=(sig_out / s2, sig_in / s2, sig_out / s2), width=W, phase_mode=1,
                      sub_min=2, sub_max=2, init_sub_max=4000 * s2)
    o = Oracle(p, {"phi0": phi0}, lib_path=lib)
    o.step(8000 * s2)
    f = o.fields()
    Ey, q = f["Ey"][:, 0], f["q"][:, 0]
    inside, outside = _layer_masks(ny, lo, hi, W)
    y = np.arange(ny)
    lower = (y >= 0.5 * (lo - (ny - hi))) & (y < 0.5 * (lo + hi))
    Ein, Eout = Ey[inside].mean(), Ey[outside].mean()
    return dict(Ein=Ein, Eout=Eout, Q=q[lower].sum(), eps_in=eps_in, sig_in=sig_in / s2, sig_out=sig_out / s2,
                Dspread=np.ptp((f["eps"] * f["Ey"])[:, 0]) / abs(0.1 * Eout), qsum=q.sum(), qabs=np.abs(q).sum())


def translation_error(scale=1, lib=None):
    """Max |phi_i(moving run) - phi_i(resting run shifted by U t)| for a
    compound drop (diffusive scaling: U ~ 1/scale, t ~ scale^2)."""
    n, R, W = 32 * scale, 8.0 * scale, 2.0 * scale
    U = (0.04 / scale, 0.02 / scale)
    t = 200 * scale * scale
    p = I.base_params(n, n, width=W, sigma=(0, 0, 0))
    phi0 = I.compound_drop(n, n, n / 2 - 0.5, n / 2 - 0.5, R, 0.6 * R, W)
    u0 = np.zeros((2, n, n))
    u0[0], u0[1] = U
    rest = Oracle(p, {"phi0": phi0}, lib_path=lib)
    move = Oracle(p, {"phi0": phi0, "u0": u0}, lib_path=lib)
    rest.step(t + 1)
    move.step(t + 1)
    kx = np.fft.fftfreq(n) * 2 * np.pi
    shift = np.exp(-1j * (kx[None, :] * U[0] * t + kx[:, None] * U[1] * t))
    err = 0.0
    for k in ("phi2", "phi3"):
        shifted = np.real(np.fft.ifft2(np.fft.fft2(rest.field(k)) * shift))
        err = max(err, np.abs(move.field(k) - shifted).max())
    return err


def band_period_error(n=64, U=0.05, lib=None):
    """A band of phase 2 (flat tanh interfaces, width n/16) carried once
    around a periodic box by a uniform flow U (n/U steps) against the same
    band at rest after as many steps: max |difference|.  Convective scaling:
    U fixed while the box and the width grow."""
    W = n / 16.0
    t = int(round(n / U))
    x = np.arange(n, dtype=float)
    s = (0.5 + 0.5 * np.tanh(2 * (x - n / 4 + 0.5) / W)) * (0.5 + 0.5 * np.tanh(2 * (3 * n / 4 - 0.5 - x) / W))
    phi0 = np.zeros((3, 1, n))
    phi0[1, 0], phi0[0, 0] = s, 1 - s
    p = I.base_params(n, 1, width=W, sigma=(0, 0, 0))
    u0 = np.zeros((2, 1, n))
    u0[0] = U
    rest = Oracle(p, {"phi0": phi0}, lib_path=lib)
    move = Oracle(p, {"phi0": phi0, "u0": u0}, lib_path=lib)
    rest.step(t + 1)
    move.step(t + 1)
    return np.abs(rest.field("phi2") - move.field("phi2")).max()


def two_layer_couette(ny=32, lib=None, mu=(0.1, 0.4), rho=(1.0, 2.5), U=1e-3):
    """Bulk shear-rate ratio (lower/upper) divided by mu_2/mu_1, and the
    shear stress mu du/dy of the lower bulk against 2U / int dy/mu(y)."""
    W = 4.0
    y = np.arange(ny, dtype=float)
    s = 0.5 + 0.5 * np.tanh(2 * (y - ny / 2 + 0.5) / W)
    phi0 = np.zeros((3, ny, 1))
    phi0[1, :, 0], phi0[0, :, 0] = s, 1 - s
    p = I.base_params(1, ny, bc_y=1, width=W, sigma=(0, 0, 0), wall_u=(-U, U),
                      visc=(mu[0], mu[1], 0.1), rho=(rho[0], rho[1], 1.0))
    o = Oracle(p, {"phi0": phi0}, lib_path=lib)
    o.step(12000)
    du = np.diff(o.field("ux")[:, 0])
    lo = du[1: ny // 2 - 3 * int(W)].mean()
    hi = du[ny // 2 + 3 * int(W): -1].mean()
    # the stress balance across the layers with the linear rule of Eq. (29)
    # and the half-way walls (distance H = ny)
    phi2 = o.field("phi2")[:, 0]
    muy = mu[0] * (1 - phi2) + mu[1] * phi2
    tau = 2 * U / np.sum(1.0 / muy)
    return (lo / hi) / (mu[1] / mu[0]), mu[0] * lo / tau


def plug_drift(lib=None, steps=100):
    """Largest change of the f, g, l populations over `steps` steps, relative
    to the population scale, for a uniform mixture with a uniform charge
    moving at U with both walls (moving-wall bounce-back keeps the
    equilibrium a fixed point)."""
    nx, ny, U = 8, 6, 0.05
    phi0 = np.empty((3, ny, nx))
    phi0[0], phi0[1], phi0[2] = 0.85, 0.08, 0.07
    u0 = np.zeros((2, ny, nx))
    u0[0] = U
    # a large permittivity keeps the field of the uniform charge (electrodes
    # at zero potential) and its force q E below round-off
    p = I.base_params(nx, ny, bc_y=1, wall_u=(U, U), sigma=(0, 0, 0), eps=(1e4, 1e4, 1e4))
    o = Oracle(p, {"phi0": phi0, "u0": u0, "q0": np.full((ny, nx), 1e-6)}, lib_path=lib)
    before = {k: o.pops(k) for k in "fgl"}
    o.step(steps)
    out = {}
    for k in "fgl":
        scale = max(np.abs(before[k]).max(), 1e-300)
        out[k] = np.abs(o.pops(k) - before[k]).max() / scale
    return out


def charge_drift(scale=1, lib=None, sigma_scale=1.0, q0=None, steps=None):
    """|sum q| / sum |q| after 400 scale^2 steps for an asymmetric compound
    drop (core off-centre) in a periodic box under an oblique applied field,
    starting without charge (Eq. 17 in a periodic domain: sum q stays 0)."""
    n, W, R = 32 * scale, 4.0 * scale, 9.6 * scale
    s2 = scale * scale
    p = I.base_params(n, n, E_ext=(0.7e-3 / scale, 2e-3 / scale), eps=(0.1, 0.25, 0.05),
                      sigma=tuple(v * sigma_scale / s2 for v in (2e-3, 6e-3, 4e-4)), width=W,
                      sub_min=2, sub_max=2, init_sub_max=200 * scale)
    c = n / 2 - 0.5
    core = I.tanh_drop(n, n, c + 0.12 * R, c + 0.25 * R, 0.45 * R, W)
    shell = (1 - core) * I.tanh_drop(n, n, c, c, R, W)
    init = {"phi0": np.stack([1 - core - shell, shell, core])}
    if q0 is not None:
        init["q0"] = q0
    o = Oracle(p, init, lib_path=lib)
    q_start = o.field("q").sum()
    o.step(steps if steps is not None else 400 * s2)
    q = o.field("q")
    return (q.sum() - q_start) / np.abs(q).sum()


# -------------------------------------------------------------- the pins

def test_maxwell_stress_jump_second_order():
    """Eq. 20's electric term: the jump of P across a flat layer equals the
    Maxwell-stress jump D^2/2 (1/eps_in - 1/eps_out), for a 4:1 and a 1:4
    permittivity contrast, converging at second order (layer and interface
    width refined together).  Without the term the jump would be zero."""
    r1 = maxwell_jump(1, 0.4)
    r2 = maxwell_jump(2, 0.4)
    r3 = maxwell_jump(1, 0.025)
    assert abs(r1 - 1) < 0.02 and abs(r3 - 1) < 0.02, (r1, r3)
    assert abs(r2 - 1) < 0.006 and abs(r1 - 1) / abs(r2 - 1) > 3.0, (r1, r2)


def test_leaky_dielectric_layer_current_and_charge():
    """Eq. 47 (with R7): at steady state the conduction current sigma E is the
    same in both bulk layers, and the interface charge is the jump of eps E
    (Gauss).  A layer with sigma/eps equal to the host's carries no free
    charge (Taylor's charge-free case); one with the host's permittivity and
    4x its conductivity carries charge.  The current error falls under 2x
    refinement."""
    a1 = layered_field(1, 0.4, 4e-3)   # sigma/eps matched: no free charge
    a2 = layered_field(2, 0.4, 4e-3)
    b1 = layered_field(1, 0.1, 4e-3)   # equal eps: charged interfaces
    ja1 = a1["sig_in"] * a1["Ein"] / (a1["sig_out"] * a1["Eout"])
    ja2 = a2["sig_in"] * a2["Ein"] / (a2["sig_out"] * a2["Eout"])
    jb1 = b1["sig_in"] * b1["Ein"] / (b1["sig_out"] * b1["Eout"])
    assert abs(ja1 - 1) < 0.03 and abs(jb1 - 1) < 0.01, (ja1, jb1)
    assert abs(ja2 - 1) < 0.01 and abs(ja1 - 1) / abs(ja2 - 1) > 2.5, (ja1, ja2)
    dD = b1["eps_in"] * b1["Ein"] - 0.1 * b1["Eout"]
    assert abs(b1["Q"] / dD - 1) < 0.01, b1["Q"] / dD
    # matched case: the interface charge (against the host's eps E) and the
    # departure of the layer's field from 1/4 of the host's are truncation
    # errors that fall at second order
    qa1, qa2 = (abs(a["Q"] / (0.1 * a["Eout"])) for a in (a1, a2))
    assert qa1 < 0.03 and qa2 < 0.008 and qa1 / qa2 > 3.0, (qa1, qa2)
    assert abs(a1["Ein"] / a1["Eout"] - 0.25) < 0.01 and abs(a2["Ein"] / a2["Eout"] - 0.25) < 0.003


def test_periodic_dielectric_layer_applied_field():
    """Reading R15: an applied field in a periodic box with a permittivity
    contrast polarises the interfaces so that D = eps E is uniform (Eq. 42
    for the full potential); no conductivity, no free charge."""
    r = layered_field(1, 0.4, 0.0, 0.0)
    assert r["Dspread"] < 1e-3, r
    assert abs(r["Ein"] / r["Eout"] - 0.25) < 1e-3, r
    assert abs(r["qsum"]) < 1e-15 and r["qabs"] < 1e-15


def test_drop_translation_galilean_second_order():
    """Eqs. 35-36: a compound drop carried by a uniform flow equals the
    resting drop shifted by U t; the difference falls ~4x under 2x
    refinement (diffusive scaling).  At a fixed flow speed (convective
    scaling) a band carried once around the box returns to the resting
    band with an error that falls more than 4x under 2x refinement; the
    d_t(phi_i u) source of Eq. 36 removes the O(U^2) numerical diffusion
    that would otherwise make it first order."""
    e1 = translation_error(1)
    e2 = translation_error(2)
    assert e2 < 0.06 and e1 / e2 > 3.0, (e1, e2)
    b1 = band_period_error(64)
    b2 = band_period_error(128)
    assert b2 < 0.03 and b1 / b2 > 4.0, (b1, b2)


def test_two_layer_couette_variable_viscosity():
    """Eq. 29 with the local relaxation time tau_g = 1/2 + mu(phi)/(rho cs2)
    (R6): in plane Couette flow through two layers the bulk shear rates are
    inversely proportional to the dynamic viscosities (4:1 contrast, 2.5:1
    density contrast, so a kinematic mapping would be off by 2.5x), and the
    stress equals 2U / int dy/mu(y)."""
    ratio, stress = two_layer_couette()
    assert abs(ratio - 1) < 1e-4, ratio
    assert abs(stress - 1) < 5e-3, stress


def test_moving_walls_keep_plug_flow_equilibrium():
    """R10: with both walls moving with a uniform flow, the uniform
    equilibria of the order-parameter, flow and charge families are a fixed
    point of the scheme, wall rows included (the moving-wall term restores
    exactly the odd part a plain reflection would flip)."""
    d = plug_drift()
    assert d["f"] < 1e-13 and d["g"] < 1e-12 and d["l"] < 1e-13, d


def test_charge_conservation():
    """Eq. 17 in a periodic box: sum q is conserved.  With sigma = 0 the
    charge family conserves it to round-off from a random start; with
    conductivity contrasts the Ohmic source of Eq. 47 (not in flux form)
    conserves it to truncation error, which falls under refinement."""
    rng = np.random.default_rng(17)
    q0 = 1e-4 * rng.standard_normal((32, 32))
    d0 = charge_drift(1, sigma_scale=0.0, q0=q0, steps=300)
    assert abs(d0) < 1e-13, d0
    d1 = charge_drift(1)
    d2 = charge_drift(2)
    assert abs(d1) < 4e-3 and abs(d2) < 2e-3 and abs(d1) / abs(d2) > 1.6, (d1, d2)


def test_permittivity_interpolation_properties():
    """Eq. 30 (Hermite interpolation), checked through the oracle's eps field
    on properties rather than the formula: pure phases give eps_i exactly; on
    a two-phase interface eps is symmetric about phi = 1/2 (the mean there)
    and flat at the pure ends (d eps / d phi -> 0: quadratic approach)."""
    ny = 64
    phi0 = np.zeros((3, ny, 1))
    s = np.concatenate([np.linspace(0, 1, ny // 2), [0.0] * (ny // 2)])
    phi0[1, :, 0] = s
    phi0[0, :, 0] = 1 - s
    p = I.base_params(1, ny, eps=(0.1, 0.7, 0.05), sigma=(0, 0, 0), phase_mode=1)
    e = Oracle(p, {"phi0": phi0}).field("eps")[:, 0]
    h = s[: ny // 2]
    ee = e[: ny // 2]
    assert ee[0] == 0.1 and ee[-1] == 0.7 and np.all(e[ny // 2:] == 0.1)
    # symmetry: eps(s) + eps(1 - s) = eps_1 + eps_2
    np.testing.assert_allclose(ee + ee[::-1], 0.8, atol=1e-15)
    # flat ends: the first increments scale like s^2
    d1, d2 = ee[1] - ee[0], ee[2] - ee[0]
    assert abs(d2 / d1 - 4.0) < 0.2, (d1, d2)
    assert np.all(np.diff(ee) > 0)
    assert h[1] > 0


# --------------------------------------------- contour deformation (Sec. 4.4)

def _ellipse(nx, ny, xc, yc, a, b, W):
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    rr = np.sqrt(((x - xc) / a) ** 2 + ((y - yc) / b) ** 2)
    return 0.5 + 0.5 * np.tanh(2 * (1 - rr) * math.sqrt(a * b) / W)


def test_contour_deformation_on_ellipses():
    """The Sec. 4.4 contour deformation of a diffuse ellipse whose w = 1/2
    level set is x^2/a^2 + y^2/b^2 = 1 is (b - a)/(b + a) (field along y),
    for off-grid centres, both orientations and a circle; the radii are the
    semi-axes.  The sharp-ellipse moment form agrees."""
    for (a, b, xc, yc) in ((30.0, 36.0, 60.3, 57.7), (36.0, 30.0, 59.5, 61.25), (25.0, 25.0, 64.0, 64.0)):
        w = _ellipse(128, 128, xc, yc, a, b, 4.0)
        D, rpar, rperp = contour_deformation(w)
        assert abs(rpar - b) < 0.02 and abs(rperp - a) < 0.02, (rpar, rperp)
        assert abs(D - (b - a) / (b + a)) < 3e-4, D
        sharp = _ellipse(256, 256, 2 * xc, 2 * yc, 2 * a, 2 * b, 0.05)
        assert abs(moment_deformation(sharp) - (b - a) / (b + a)) < 2e-3
    # walls: a drop reaching a wall has no crossing there
    w = _ellipse(64, 40, 32.0, 20.0, 10.0, 30.0, 4.0)
    assert math.isnan(contour_deformation(w, walls=True)[0])
    # 3-D: a spheroid elongated along y
    z, y, x = np.mgrid[0:48, 0:48, 0:48].astype(float)
    rr = np.sqrt(((x - 23.5) / 12) ** 2 + ((y - 24.2) / 15) ** 2 + ((z - 23.0) / 12) ** 2)
    w3 = 0.5 + 0.5 * np.tanh(2 * (1 - rr) * 13 / 4.0)
    D3, rp, rq = contour_deformation(w3)
    assert abs(rp - 15) < 0.05 and abs(rq - 12) < 0.05 and abs(D3 - 3 / 27) < 1e-3


# ------------------------------------------------------- planted mistakes

MUTANTS = {
    # Eq. 20 electric term dropped / sign flipped / factor 1/2 lost
    "mu_no_electric": ([("const double elec = 0.5 * (6.0 * s->p.eps[i] * ph * (1.0 - ph)) * e2;",
                         "const double elec = 0.0 * e2;")], "maxwell"),
    "mu_electric_sign": ([("s->mu[i * N + n] = bulk - grad - elec;", "s->mu[i * N + n] = bulk - grad + elec;")],
                         "maxwell"),
    "mu_electric_factor": ([("const double elec = 0.5 * (6.0", "const double elec = 1.0 * (6.0")], "maxwell"),
    # Eq. 47: the (sigma/eps) grad(eps).E term dropped; grad(sigma).E sign flipped
    "R_no_grad_eps": ([("const double Rp = se * ge - gs;", "const double Rp = 0.0 * ge - gs;")], "leaky"),
    "R_grad_sigma_sign": ([("const double Rp = se * ge - gs;", "const double Rp = se * ge + gs;")], "leaky"),
    "R_grad_sigma_sign_q": ([("const double Rp = se * ge - gs;", "const double Rp = se * ge + gs;")], "charge"),
    # applied field added after the solve (the reading R15 replaces)
    "Eext_after_solve": ([("g[d] = -(m[d] + CS2 * s->tau_h * s->Eext[d]) / den;", "g[d] = -m[d] / den;"),
                          ("s->E[d * N + n] = -g[d];", "s->E[d * N + n] = -g[d] + s->Eext[d];")], "dielectric"),
    # Eqs. 35-36: advection in the equilibrium, d_t(phi u) in the source
    "feq_no_advection": ([("L->w[j] * mu + L->w[j] * cu / CS2;\n          /* source",
                           "L->w[j] * mu + 0.0 * cu / CS2;\n          /* source")], "translation"),
    "F_no_dt_phiu": ([("(dotc(L, j, dpu[i]) / CS2 - dotc(L, j, X) / m0)", "(0.0 * dpu[i][0] - dotc(L, j, X) / m0)")],
                     "band"),
    # R6: kinematic instead of dynamic viscosity in tau_g
    "tau_g_kinematic": ([("const double tg = 0.5 + s->visc[n] / (rho * CS2);",
                          "const double tg = 0.5 + s->visc[n] / CS2;")], "couette"),
    # R10: plain reflection of f / l at moving walls
    "f_no_wall_term": ([("0, s->phi + i * N, 0, 0);", "0, NULL, 0, 0);")], "plug_f"),
    "l_no_wall_term": ([("stream_family(s, s->ln, s->l, 0, s->q, 0, 0);",
                         "stream_family(s, s->ln, s->l, 0, NULL, 0, 0);")], "plug_l"),
}


@pytest.fixture(scope="module")
def mutant_dir(tmp_path_factory):
    return str(tmp_path_factory.mktemp("oracle_mutants"))


def _mutant_lib(name, mutant_dir):
    src = oracle.source_text()
    for old, new in MUTANTS[name][0]:
        assert src.count(old) == 1, (name, old)
        src = src.replace(old, new)
    return oracle.compile_variant(src, os.path.join(mutant_dir, name + ".so"))


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pin_rejects_planted_mistake(name, mutant_dir):
    """Every pin above fails on an oracle with the mistake it guards
    against, at the coarse resolution of its own check."""
    lib = _mutant_lib(name, mutant_dir)
    kind = MUTANTS[name][1]
    if kind == "maxwell":
        r = maxwell_jump(1, 0.4, lib=lib)
        assert abs(r - 1) > 0.2, r
    elif kind == "leaky":
        a = layered_field(1, 0.4, 4e-3, lib=lib)
        b = layered_field(1, 0.1, 4e-3, lib=lib)
        ja = a["sig_in"] * a["Ein"] / (a["sig_out"] * a["Eout"])
        dD = b["eps_in"] * b["Ein"] - 0.1 * b["Eout"]
        assert abs(ja - 1) > 0.1 or abs(b["Q"] / dD - 1) > 0.1, (ja, b["Q"] / dD)
    elif kind == "dielectric":
        r = layered_field(1, 0.4, 0.0, 0.0, lib=lib)
        assert abs(r["Ein"] / r["Eout"] - 0.25) > 0.1, r
    elif kind == "charge":
        d = charge_drift(1, lib=lib)
        assert abs(d) > 2e-2, d
    elif kind == "translation":
        e = translation_error(1, lib=lib)
        assert e > 0.3, e
    elif kind == "band":
        e = band_period_error(128, lib=lib)
        assert e > 0.05, e
    elif kind == "couette":
        ratio, stress = two_layer_couette(lib=lib)
        assert abs(ratio - 1) > 0.1 or abs(stress - 1) > 0.1, (ratio, stress)
    elif kind == "plug_f":
        assert plug_drift(lib=lib)["f"] > 1e-6
    elif kind == "plug_l":
        assert plug_drift(lib=lib)["l"] > 1e-6
