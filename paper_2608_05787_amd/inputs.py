"""Seeded synthetic workloads: parameter sets and initial fields.

This module is shared by the GPU path's callers and by the oracle's tests, so
it holds none of the lattice-Boltzmann arithmetic: it only builds parameter
dictionaries and initial order-parameter / velocity / charge / potential
fields from closed-form shapes (tanh interface profiles of Eqs. (54) and (56),
linear electrode profiles, the Debye-Hueckel profile of Eq. (53)).

Phase numbering follows the workloads: phase 1 (index 0) is the host/bulk
fluid, phase 2 (index 1) the shell or first drop, phase 3 (index 2) the core
or second drop.

A parameter dict carries:
  nx, ny, bc_y (0 periodic, 1 walls), wall_u, wall_phi, wall_q_mode, wall_q,
  E_ext, gamma12, gamma13, gamma23, width, rho[3], visc[3], eps[3], sigma[3],
  tau_f, tau_l, eps_ref_phase, phase_mode, sub_min, sub_max, sub_tol,
  init_sub_max, init_tol, nz, lattice (0 D2Q9, 1 D3Q15), E_ext_z,
  charge_model (0 leaky dielectric, 1 two-ion Nernst-Planck), ion_tau,
  ion_beta, ion_charge.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "base_params", "tanh_drop", "compound_drop", "doublet", "flat_layers",
    "eof_channel", "static_doublet", "field_compound_drop", "batch_sweep",
    "adjoint_case", "parity_case", "applied_field", "theta_of", "with_theta", "liquid_lens",
    "base_params3d", "sphere_drop", "compound_drop3d", "parity_case3d", "field_compound_drop3d",
    "two_compound_drops", "np_eof_channel", "np_parity_case",
]


def base_params(nx: int, ny: int, **kw) -> dict:
    """Equal-property defaults used by the compound-drop workloads: gamma_ij =
    1e-3, interface width 4, rho = 1, dynamic viscosity 0.1 (tau = 0.8),
    tau_f = 0.8, eps = 0.1, sigma = 1e-3, tau_l = 0.8."""
    p = dict(nx=int(nx), ny=int(ny), bc_y=0, wall_u=(0.0, 0.0), wall_phi=(0.0, 0.0),
             wall_q_mode=0, wall_q=(0.0, 0.0), E_ext=(0.0, 0.0),
             gamma12=1e-3, gamma13=1e-3, gamma23=1e-3, width=4.0,
             rho=(1.0, 1.0, 1.0), visc=(0.1, 0.1, 0.1), eps=(0.1, 0.1, 0.1),
             sigma=(1e-3, 1e-3, 1e-3), tau_f=0.8, tau_l=0.8, eps_ref_phase=0,
             phase_mode=0, sub_min=1, sub_max=1, sub_tol=0.0,
             init_sub_max=0, init_tol=0.0, nz=1, lattice=0, E_ext_z=0.0,
             charge_model=0, ion_tau=0.8, ion_beta=0.0, ion_charge=0.0, sum_relax=0)
    p.update(kw)
    return p


def base_params3d(nx: int, ny: int, nz: int, **kw) -> dict:
    """base_params on the D3Q15 lattice (Eq. 32): an nx x ny x nz box,
    periodic in x and z, y periodic or walled."""
    return base_params(nx, ny, nz=int(nz), lattice=1, **kw)


def _grid(nx, ny):
    y, x = np.mgrid[0:ny, 0:nx].astype(np.float64)
    return x, y


def _grid3(nx, ny, nz):
    z, y, x = np.mgrid[0:nz, 0:ny, 0:nx].astype(np.float64)
    return x, y, z


def sphere_drop(nx, ny, nz, c, r, width):
    """The profile of Eq. (54) around a sphere: [nz, ny, nx]."""
    x, y, z = _grid3(nx, ny, nz)
    d = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    return 0.5 + 0.5 * np.tanh(2.0 * (r - d) / width)


def compound_drop3d(nx, ny, nz, c, r_shell, r_core, width):
    """Concentric spherical compound drop: phi0 [3, nz, ny, nx]."""
    core = sphere_drop(nx, ny, nz, c, r_core, width)
    shell = (1.0 - core) * sphere_drop(nx, ny, nz, c, r_shell, width)
    return np.stack([1.0 - core - shell, shell, core])


def tanh_drop(nx, ny, cx, cy, r, width):
    """1/2 + 1/2 tanh(2 (r - |x - c|) / W): the drop profile of Eq. (54)."""
    x, y = _grid(nx, ny)
    d = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return 0.5 + 0.5 * np.tanh(2.0 * (r - d) / width)


def compound_drop(nx, ny, cx, cy, r_shell, r_core, width):
    """Concentric compound drop built as in Eq. (54): core (phase 3) inside
    shell (phase 2) inside host (phase 1).  Returns phi0 [3, ny, nx]."""
    core = tanh_drop(nx, ny, cx, cy, r_core, width)
    shell = (1.0 - core) * tanh_drop(nx, ny, cx, cy, r_shell, width)
    return np.stack([1.0 - core - shell, shell, core])


def doublet(nx, ny, c2, r2, c3, r3, width):
    """Two overlapping drops: phase 2 first, then phase 3 carved from what is
    left, host = remainder.  Returns phi0 [3, ny, nx]."""
    p2 = tanh_drop(nx, ny, c2[0], c2[1], r2, width)
    p3 = (1.0 - p2) * tanh_drop(nx, ny, c3[0], c3[1], r3, width)
    return np.stack([1.0 - p2 - p3, p2, p3])


def flat_layers(nx, ny, y_lo, y_hi, width, phase=1):
    """A band of `phase` between y_lo and y_hi (tanh edges), host elsewhere."""
    _, y = _grid(nx, ny)
    band = (0.5 + 0.5 * np.tanh(2.0 * (y - y_lo) / width)) * \
           (0.5 + 0.5 * np.tanh(2.0 * (y_hi - y) / width))
    phi = np.zeros((3, ny, nx))
    phi[phase] = band
    phi[0] = 1.0 - band
    return phi


# --------------------------------------------------------------- workloads

def eof_channel(nx=64, ny=32, zeta=1.0, debye=4.0, E=1e-4, tau=0.8, closed_form_start=True):
    """Electro-osmotic channel (single phase, frozen order parameters).

    Walls at y = -1/2 and ny - 1/2 hold potential zeta and the Dirichlet charge
    of the Debye-Hueckel profile; tau = 0.8 for flow, charge and potential gives
    mu = eps = alpha = 0.1, and sigma = eps * alpha / debye^2 fixes the Debye
    length.  Returns (params, init)."""
    cs2 = 1.0 / 3.0
    nu = cs2 * (tau - 0.5)
    eps = nu
    alpha = nu
    kappa = 1.0 / debye
    sigma = eps * alpha * kappa * kappa
    qw = -eps * kappa * kappa * zeta
    p = base_params(nx, ny, bc_y=1, wall_phi=(zeta, zeta), wall_q_mode=1, wall_q=(qw, qw),
                    E_ext=(E, 0.0), visc=(nu, nu, nu), eps=(eps, eps, eps),
                    sigma=(sigma, sigma, sigma), tau_f=tau, tau_l=tau, phase_mode=1,
                    sub_min=1, sub_max=1, init_sub_max=4000, init_tol=1e-13)
    phi0 = np.zeros((3, ny, nx))
    phi0[0] = 1.0
    init = {"phi0": phi0}
    if closed_form_start:
        _, y = _grid(nx, ny)
        yc = y - 0.5 * (ny - 1)
        h = 0.5 * ny
        psi = zeta * np.cosh(kappa * yc) / math.cosh(kappa * h)
        init["psi0"] = psi
        init["q0"] = -eps * kappa * kappa * psi
    meta = dict(kappa=kappa, h=0.5 * ny, zeta=zeta, E=E, eps=eps, mu=nu, alpha=alpha, sigma=sigma)
    return p, init, meta


def np_eof_channel(nx=4, ny=32, zeta=0.05, debye=4.0, E=1e-4, beta=1.0, n0=1.0, tau=0.8,
                   ion_tau=0.8, closed_form_start=True):
    """Electro-osmotic channel with a two-ion Nernst-Planck electrolyte
    (Eq. 52, valences +1/-1; single phase, frozen order parameters).

    Walls at y = -1/2 and ny - 1/2 hold potential zeta and no ion flux; the
    Debye length follows kappa^2 = 2 e n0 beta / eps (Eq. 53) with the
    elementary charge e chosen for it; beta = e/(k_B T); beta zeta << 1 is the
    Debye-Hueckel regime.  The start is the closed-form potential with
    Boltzmann ion profiles n_+- = n0 exp(-+ beta psi), fluid at rest.
    Returns (params, init, meta)."""
    cs2 = 1.0 / 3.0
    nu = cs2 * (tau - 0.5)
    eps = nu
    kappa = 1.0 / debye
    e = kappa * kappa * eps / (2.0 * n0 * beta)
    p = base_params(nx, ny, bc_y=1, wall_phi=(zeta, zeta), E_ext=(E, 0.0), visc=(nu, nu, nu),
                    eps=(eps, eps, eps), sigma=(0.0, 0.0, 0.0), tau_f=tau, tau_l=tau, phase_mode=1,
                    sub_min=1, sub_max=1, init_sub_max=4000, init_tol=1e-13,
                    charge_model=1, ion_tau=ion_tau, ion_beta=beta, ion_charge=e)
    phi0 = np.zeros((3, ny, nx))
    phi0[0] = 1.0
    _, y = _grid(nx, ny)
    yc = y - 0.5 * (ny - 1)
    h = 0.5 * ny
    psi = zeta * np.cosh(kappa * yc) / math.cosh(kappa * h) if closed_form_start else np.zeros((ny, nx))
    init = {"phi0": phi0, "psi0": psi, "ions0": np.stack([n0 * np.exp(-beta * psi), n0 * np.exp(beta * psi)])}
    meta = dict(kappa=kappa, h=h, zeta=zeta, E=E, eps=eps, mu=nu, e=e, beta=beta, n0=n0,
                D=cs2 * (ion_tau - 0.5))
    return p, init, meta


def static_doublet(n=256, r2=40.0, r3=30.0, dist=55.0, gammas=(1.0e-3, 1.2e-3, 0.8e-3)):
    """Static overlapping doublet in a periodic box, no field (workload 2)."""
    g12, g13, g23 = gammas
    p = base_params(n, n, gamma12=g12, gamma13=g13, gamma23=g23,
                    sigma=(0.0, 0.0, 0.0))
    c2 = (0.5 * n - 27.5 * dist / 55.0, 0.5 * n)
    c3 = (c2[0] + dist, 0.5 * n)
    init = {"phi0": doublet(n, n, c2, r2, c3, r3, 4.0)}
    return p, init


def field_compound_drop(n=1024, r_shell=80.0, r_core=60.0, ca_e=0.2,
                        eps_ratio=(2.0, 0.5), sigma_ratio=(3.0, 0.3), tau_l=0.6,
                        sub=(4, 4, 0.0), init_iters=20000, init_tol=1e-7, wall_u=0.0):
    """Concentric compound drop between electrodes (workload 3 and the
    adjoint / batch variants).  The electrode potential difference gives the
    electric capillary number ca_e = eps1 E0^2 R_shell / gamma (Eq. 51)."""
    eps1, sig1, gamma = 0.1, 1e-3, 1e-3
    E0 = math.sqrt(ca_e * gamma / (eps1 * r_shell))
    dV = E0 * n
    eps = (eps1, eps1 * eps_ratio[0], eps1 * eps_ratio[1])
    sig = (sig1, sig1 * sigma_ratio[0], sig1 * sigma_ratio[1])
    p = base_params(n, n, bc_y=1, wall_phi=(0.0, dV), eps=eps, sigma=sig, tau_l=tau_l,
                    wall_u=(-wall_u, wall_u), sub_min=int(sub[0]), sub_max=int(sub[1]),
                    sub_tol=float(sub[2]), init_sub_max=int(init_iters), init_tol=float(init_tol))
    c = 0.5 * (n - 1)
    phi0 = compound_drop(n, n, c, c, r_shell, r_core, 4.0)
    _, y = _grid(n, n)
    init = {"phi0": phi0, "psi0": dV * (y + 0.5) / n}
    if wall_u != 0.0:
        u0 = np.zeros((2, n, n))
        u0[0] = wall_u * (2.0 * (y + 0.5) / n - 1.0)
        init["u0"] = u0
    return p, init


# Phase ratios of the two-drop interaction runs (Sec. 4.5), in this code's
# numbering (phase 1 host, 2 shell, 3 core; the paper numbers the bulk 3 and
# the core 1): (eps2/eps1, eps3/eps1), (sigma2/sigma1, sigma3/sigma1).
TWO_DROP_REGIMES = {
    # S_shell/bulk = 8, R_shell/bulk = 6, S_core/shell = 1/8, R_core/shell = 1/6
    "coalescence": ((8.0, 1.0), (6.0, 1.0)),
    # S_shell/bulk = 0.2, R_shell/bulk = 1.04, S_core/shell = 5, R_core/shell = 1/1.04
    "separation": ((0.2, 1.0), (1.04, 1.0)),
}


def two_compound_drops(nx=256, ny=384, r_shell=30.0, r_core=18.0, gap=8.0, regime="coalescence",
                       ca_e=0.2, tau_l=0.8, sub=(4, 4, 0.0), init_iters=4000, init_tol=0.0):
    """Two equal concentric compound drops on the vertical centre line,
    aligned with the field between electrodes (walls in y), shells `gap`
    nodes apart (Sec. 4.5); equal densities and viscosities; ca_e =
    eps1 E0^2 R_shell / gamma."""
    eps_ratio, sigma_ratio = TWO_DROP_REGIMES[regime]
    eps1, sig1, gamma = 0.1, 1e-3, 1e-3
    E0 = math.sqrt(ca_e * gamma / (eps1 * r_shell))
    dV = E0 * ny
    eps = (eps1, eps1 * eps_ratio[0], eps1 * eps_ratio[1])
    sig = (sig1, sig1 * sigma_ratio[0], sig1 * sigma_ratio[1])
    p = base_params(nx, ny, bc_y=1, wall_phi=(0.0, dV), eps=eps, sigma=sig, tau_l=tau_l,
                    sub_min=int(sub[0]), sub_max=int(sub[1]), sub_tol=float(sub[2]),
                    init_sub_max=int(init_iters), init_tol=float(init_tol))
    cx, cy = 0.5 * (nx - 1), 0.5 * (ny - 1)
    off = r_shell + 0.5 * gap
    core = sum(tanh_drop(nx, ny, cx, cy + s * off, r_core, 4.0) for s in (-1, 1))
    shell = (1.0 - core) * sum(tanh_drop(nx, ny, cx, cy + s * off, r_shell, 4.0) for s in (-1, 1))
    _, y = _grid(nx, ny)
    return p, {"phi0": np.stack([1.0 - core - shell, shell, core]), "psi0": dV * (y + 0.5) / ny}


def batch_sweep(n_inst=64, seed=5787, lo=128, hi=512, sub=(4, 4, 0.0), init_iters=2000):
    """Parameter sweep of compound drops (workload 4): grid sizes uniform over
    multiples of 32 in [lo, hi], Ca_e ~ U[0.05, 0.4], eps and sigma ratios
    log-uniform in [1/4, 4], half the instances sheared at wall speed 0.01."""
    rng = np.random.default_rng(seed)
    draws = []
    for _ in range(n_inst):
        n = lo + 32 * int(rng.integers(0, (hi - lo) // 32 + 1))
        ca = float(rng.uniform(0.05, 0.4))
        ln = rng.uniform(math.log(0.25), math.log(4.0), size=4)
        draws.append((n, ca, tuple(float(v) for v in np.exp(ln))))
    sheared = set(int(i) for i in rng.permutation(n_inst)[: n_inst // 2])
    out = []
    for i, (n, ca, r) in enumerate(draws):
        p, init = field_compound_drop(n, r_shell=5.0 * n / 32.0, r_core=15.0 * n / 128.0,
                                      ca_e=ca, eps_ratio=(r[0], r[1]), sigma_ratio=(r[2], r[3]),
                                      sub=sub, init_iters=init_iters,
                                      wall_u=0.01 if i in sheared else 0.0)
        out.append((p, init))
    return out


def liquid_lens(n=200, radius=30.0, ratio=(1.0, 1.0, 1.0), gamma=2e-3, rho=(10.0, 1.0, 5.0), width=4.0,
                tau=0.8, sum_relax=1):
    """Liquid lens (Eq. 56): a drop of phase 1 centred on the flat interface
    between phase 2 (above) and phase 3 (below); walls at top and bottom,
    periodic in x.  Surface tensions gamma * ratio (gamma12 : gamma13 :
    gamma23); densities rho; dynamic viscosities 0.1 rho_i so that the flow
    relaxation time is tau = 0.8 in every phase.  No field.  The restoring
    flux of the order-parameter sum is on unless sum_relax=0 (the triple
    junctions at the density jumps would otherwise carry the sum off one)."""
    xc = yc = 0.5 * (n - 1)
    phi1 = tanh_drop(n, n, xc, yc, radius, width)
    _, y = _grid(n, n)
    phi2 = np.maximum(0.5 + 0.5 * np.tanh(2.0 * (y - yc) / width) - phi1, 0.0)
    phi0 = np.stack([phi1, phi2, 1.0 - phi1 - phi2])
    g12, g13, g23 = (gamma * r for r in ratio)
    cs2 = 1.0 / 3.0
    visc = tuple(cs2 * (tau - 0.5) * r for r in rho)
    p = base_params(n, n, bc_y=1, gamma12=g12, gamma13=g13, gamma23=g23, width=width,
                    rho=tuple(rho), visc=visc, sigma=(0.0, 0.0, 0.0), tau_f=tau, sum_relax=sum_relax)
    return p, {"phi0": phi0}


def adjoint_case(n=512):
    """Workload 5: workload 3 scaled to a 512^2 box with radii 40/30."""
    return field_compound_drop(n, r_shell=40.0, r_core=30.0)


def parity_case(nx, ny, seed=0, walls=True, field=True, shear=True, sub=(2, 2, 0.0)):
    """Small seeded case that switches on every term of the step: three
    phases with unequal densities/viscosities, electrodes, applied field,
    conductivity and permittivity contrast, moving walls and a non-zero
    initial velocity and charge."""
    rng = np.random.default_rng(seed)
    r2 = 0.30 * min(nx, ny) + rng.uniform(-0.5, 0.5)
    r3 = 0.18 * min(nx, ny) + rng.uniform(-0.5, 0.5)
    cx = 0.5 * (nx - 1) + rng.uniform(-1, 1)
    cy = 0.5 * (ny - 1) + rng.uniform(-1, 1)
    width = 2.5
    phi0 = compound_drop(nx, ny, cx, cy, r2, r3, width)
    x, y = _grid(nx, ny)
    u0 = np.stack([1e-3 * np.sin(2 * np.pi * (y + 0.5) / ny) + 2e-4 * rng.standard_normal((ny, nx)),
                   1e-3 * np.cos(2 * np.pi * x / nx) + 2e-4 * rng.standard_normal((ny, nx))])
    q0 = 1e-3 * rng.standard_normal((ny, nx))
    q0 -= q0.mean()
    p = base_params(nx, ny, bc_y=1 if walls else 0,
                    gamma12=1.0e-2, gamma13=1.3e-2, gamma23=0.8e-2, width=width,
                    rho=(1.0, 1.3, 0.8), visc=(0.1, 0.15, 0.07),
                    eps=(0.1, 0.25, 0.05), sigma=(2e-3, 5e-3, 4e-4), tau_f=0.9, tau_l=0.7,
                    sub_min=int(sub[0]), sub_max=int(sub[1]), sub_tol=float(sub[2]),
                    init_sub_max=6, init_tol=0.0)
    if walls:
        p.update(wall_u=(-3e-3, 5e-3) if shear else (0.0, 0.0),
                 wall_phi=(0.0, 0.4) if field else (0.0, 0.0))
    if field:
        p.update(E_ext=(2e-3, -1e-3))
    psi0 = 0.4 * (y + 0.5) / ny if (walls and field) else np.zeros((ny, nx))
    return p, {"phi0": phi0, "u0": u0, "q0": q0, "psi0": psi0}


def np_parity_case(nx, ny, nz=0, seed=0, walls=True, sub=(2, 2, 0.0)):
    """parity_case (D2Q9, nz = 0) or parity_case3d (D3Q15, nz > 0) under
    the two-ion Nernst-Planck charge model: conductivities zero, seeded ion
    concentrations around 1 (so a non-zero initial charge), drift strong
    enough to move them within a few steps."""
    if nz > 0:
        p, init = parity_case3d(nx, ny, nz, seed=seed, walls=walls, sub=sub)
    else:
        p, init = parity_case(nx, ny, seed=seed, walls=walls, sub=sub)
    rng = np.random.default_rng(1000 + seed)
    shape = init["phi0"].shape[1:]
    ions = np.stack([1.0 + 0.05 * rng.standard_normal(shape), 1.0 + 0.05 * rng.standard_normal(shape)])
    p.update(sigma=(0.0, 0.0, 0.0), charge_model=1, ion_tau=0.75, ion_beta=5.0, ion_charge=2e-3)
    init = dict(init, ions0=ions)
    init.pop("q0", None)
    return p, init


def parity_case3d(nx, ny, nz, seed=0, walls=True, field=True, shear=True, sub=(2, 2, 0.0)):
    """parity_case on the D3Q15 lattice: a spherical compound drop with every
    term of the step on (three phases with unequal properties, electrodes,
    an applied field with a z component, moving walls, a non-zero initial
    3-D velocity and charge)."""
    rng = np.random.default_rng(seed)
    m = min(nx, ny, nz)
    r2 = 0.30 * m + rng.uniform(-0.3, 0.3)
    r3 = 0.18 * m + rng.uniform(-0.3, 0.3)
    c = tuple(0.5 * (k - 1) + rng.uniform(-0.7, 0.7) for k in (nx, ny, nz))
    width = 2.5
    phi0 = compound_drop3d(nx, ny, nz, c, r2, r3, width)
    x, y, z = _grid3(nx, ny, nz)
    noise = lambda: 2e-4 * rng.standard_normal((nz, ny, nx))  # noqa: E731
    u0 = np.stack([1e-3 * np.sin(2 * np.pi * (y + 0.5) / ny) + noise(),
                   1e-3 * np.cos(2 * np.pi * x / nx) + noise(),
                   8e-4 * np.sin(2 * np.pi * (x + z) / max(nx, nz)) + noise()])
    q0 = 1e-3 * rng.standard_normal((nz, ny, nx))
    q0 -= q0.mean()
    p = base_params3d(nx, ny, nz, bc_y=1 if walls else 0,
                      gamma12=1.0e-2, gamma13=1.3e-2, gamma23=0.8e-2, width=width,
                      rho=(1.0, 1.3, 0.8), visc=(0.1, 0.15, 0.07),
                      eps=(0.1, 0.25, 0.05), sigma=(2e-3, 5e-3, 4e-4), tau_f=0.9, tau_l=0.7,
                      sub_min=int(sub[0]), sub_max=int(sub[1]), sub_tol=float(sub[2]),
                      init_sub_max=6, init_tol=0.0)
    if walls:
        p.update(wall_u=(-3e-3, 5e-3) if shear else (0.0, 0.0),
                 wall_phi=(0.0, 0.4) if field else (0.0, 0.0))
    if field:
        p.update(E_ext=(2e-3, -1e-3), E_ext_z=1.5e-3)
    psi0 = 0.4 * (y + 0.5) / ny if (walls and field) else np.zeros((nz, ny, nx))
    return p, {"phi0": phi0, "u0": u0, "q0": q0, "psi0": psi0}


def field_compound_drop3d(n=128, r_shell=40.0, r_core=30.0, ca_e=0.2,
                          eps_ratio=(2.0, 0.5), sigma_ratio=(3.0, 0.3), tau_l=0.6,
                          sub=(4, 4, 0.0), init_iters=2000, init_tol=0.0):
    """The field-driven compound drop in 3-D (Sec. 4.4): a spherical core
    inside a spherical shell centred in an n^3 box between electrodes (walls
    at y = -1/2, n - 1/2), periodic in x and z; parameters of workload 3."""
    eps1, sig1, gamma = 0.1, 1e-3, 1e-3
    E0 = math.sqrt(ca_e * gamma / (eps1 * r_shell))
    dV = E0 * n
    eps = (eps1, eps1 * eps_ratio[0], eps1 * eps_ratio[1])
    sig = (sig1, sig1 * sigma_ratio[0], sig1 * sigma_ratio[1])
    p = base_params3d(n, n, n, bc_y=1, wall_phi=(0.0, dV), eps=eps, sigma=sig, tau_l=tau_l,
                      sub_min=int(sub[0]), sub_max=int(sub[1]), sub_tol=float(sub[2]),
                      init_sub_max=int(init_iters), init_tol=float(init_tol))
    c = (0.5 * (n - 1),) * 3
    phi0 = compound_drop3d(n, n, n, c, r_shell, r_core, 4.0)
    _, y, _ = _grid3(n, n, n)
    return p, {"phi0": phi0, "psi0": dV * (y + 0.5) / n}


# ---------------------------------------------- gradient parameterisation
# theta = (eps2/eps1, eps3/eps1, sigma2/sigma1, sigma3/sigma1, E0).  Phases
# 2 and 3 scale against phase 1; E0 is the applied field magnitude, and
# changing it scales E_ext, the electrode potentials and the initial
# potential guess about the electrodes' mean potential.

def applied_field(cfg: dict):
    """(E0, mean electrode potential) with the conventions of dtheta."""
    walls = int(cfg.get("bc_y", 0)) == 1
    wp = cfg.get("wall_phi", (0.0, 0.0))
    ex, ey = cfg.get("E_ext", (0.0, 0.0))
    ez = float(cfg.get("E_ext_z", 0.0)) if int(cfg.get("lattice", 0)) == 1 else 0.0
    ey = ey + ((wp[0] - wp[1]) / cfg["ny"] if walls else 0.0)
    mean = 0.5 * (wp[0] + wp[1]) if walls else 0.0
    return math.sqrt(ex * ex + ey * ey + ez * ez), mean


def theta_of(cfg: dict):
    e, s = cfg["eps"], cfg["sigma"]
    return [e[1] / e[0], e[2] / e[0], s[1] / s[0], s[2] / s[0], applied_field(cfg)[0]]


def with_theta(cfg: dict, init: dict, theta):
    """Copy of (cfg, init) with the five parameters set to theta."""
    t = [float(v) for v in theta]
    c = dict(cfg)
    e, s = list(cfg["eps"]), list(cfg["sigma"])
    c["eps"] = (e[0], e[0] * t[0], e[0] * t[1])
    c["sigma"] = (s[0], s[0] * t[2], s[0] * t[3])
    E0, mean = applied_field(cfg)
    new = dict(init)
    if E0 > 0:
        r = t[4] / E0
        c["E_ext"] = tuple(v * r for v in cfg.get("E_ext", (0.0, 0.0)))
        c["E_ext_z"] = float(cfg.get("E_ext_z", 0.0)) * r
        if int(cfg.get("bc_y", 0)) == 1:
            c["wall_phi"] = tuple(mean + (v - mean) * r for v in cfg["wall_phi"])
        if init.get("psi0") is not None:
            new["psi0"] = mean + (np.asarray(init["psi0"]) - mean) * r
    return c, new


