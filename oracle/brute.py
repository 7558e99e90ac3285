"""Brute-force second transcription of the D2Q9 leaky-dielectric step.

TEST INFRASTRUCTURE ONLY (part of the oracle).  A pure-Python, node-by-node
restatement of the coupled step of Sec. 3 (Eqs. 20, 28-50) with the same
readings as the C oracle (R1-R16), written independently of it: plain
Python floats in nested lists, pull streaming instead of push, the lattice
tables built from the velocity set rather than typed in, and no vector
arithmetic.  It exists to catch transcription slips in the C oracle: on
grids of a few nodes (8 x 8) the two must agree to round-off.  It is far
too slow for anything larger.

Indices: field[y][x]; populations pop[j][y][x]; phases i = 0, 1, 2.
"""
from __future__ import annotations

import math

CS2 = 1.0 / 3.0

# D2Q9 velocity set (Eq. 31) and its weights; the opposite directions and
# the potential-source weights (Eq. 43: none at rest, equal elsewhere) are
# derived from it.
C = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
W = [4.0 / 9.0] + [1.0 / 9.0] * 4 + [1.0 / 36.0] * 4
OPP = [C.index((-a, -b)) for (a, b) in C]
VARPI = [0.0] + [1.0 / 8.0] * 8
Q = 9


def _zeros(ny, nx):
    return [[0.0] * nx for _ in range(ny)]


class Brute:
    """cfg: the parameter dict of the workloads (D2Q9, leaky dielectric);
    init: phi0 [3][ny][nx], optional u0 [2][ny][nx], q0, psi0 [ny][nx] as
    nested sequences or arrays."""

    def __init__(self, cfg, init):
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        self.walls = int(cfg.get("bc_y", 0)) == 1
        self.cfg = cfg
        g12, g13, g23 = cfg["gamma12"], cfg["gamma13"], cfg["gamma23"]
        self.lam = [g12 + g13 - g23, g12 + g23 - g13, g13 + g23 - g12]  # Eq. (9)
        self.Dw = float(cfg["width"])
        self.tau_f, self.tau_l = float(cfg["tau_f"]), float(cfg["tau_l"])
        self.m0 = CS2 * (self.tau_f - 0.5)
        self.eps_i = [float(v) for v in cfg["eps"]]
        self.sig_i = [float(v) for v in cfg["sigma"]]
        self.rho_i = [float(v) for v in cfg["rho"]]
        self.visc_i = [float(v) for v in cfg["visc"]]
        self.eps_ref = self.eps_i[int(cfg.get("eps_ref_phase", 0))]
        self.tau_h = 0.5 + self.eps_ref / CS2
        self.Eext = [float(v) for v in cfg.get("E_ext", (0.0, 0.0))]
        self.wall_u = [float(v) for v in cfg.get("wall_u", (0.0, 0.0))]
        self.wall_phi = [float(v) for v in cfg.get("wall_phi", (0.0, 0.0))]
        self.wall_q = [float(v) for v in cfg.get("wall_q", (0.0, 0.0))]
        self.q_dirichlet = int(cfg.get("wall_q_mode", 0)) == 1
        self.frozen = int(cfg.get("phase_mode", 0)) == 1
        self.sum_relax = int(cfg.get("sum_relax", 0)) == 1
        nx, ny = self.nx, self.ny

        def grab(a):
            return [[float(a[y][x]) for x in range(nx)] for y in range(ny)]

        self.phi = [grab(init["phi0"][i]) for i in range(3)]
        u0 = init.get("u0")
        self.u = [grab(u0[d]) if u0 is not None else _zeros(ny, nx) for d in range(2)]
        self.q = grab(init["q0"]) if init.get("q0") is not None else _zeros(ny, nx)
        psi0 = grab(init["psi0"]) if init.get("psi0") is not None else _zeros(ny, nx)
        self.R = _zeros(ny, nx)
        self.p = _zeros(ny, nx)
        self.E = [_zeros(ny, nx), _zeros(ny, nx)]
        self._properties()
        # potential populations at the equilibrium (Eq. 44) of the initial guess
        self.h = [[[(W[j] - 1.0 if j == 0 else W[j]) * psi0[y][x] for x in range(nx)] for y in range(ny)]
                  for j in range(Q)]
        self._solve_potential(1, int(cfg.get("init_sub_max", 0)), float(cfg.get("init_tol", 0.0)))
        self._chemical_potential()
        # every family at the equilibrium of the initial fields, p = 0
        self.f = [[[[0.0] * nx for _ in range(ny)] for _ in range(Q)] for _ in range(3)]
        self.g = [_zeros(ny, nx) for _ in range(Q)]
        self.l = [_zeros(ny, nx) for _ in range(Q)]
        self.hpu = [[_zeros(ny, nx) for _ in range(2)] for _ in range(3)]
        self.hqu = [_zeros(ny, nx) for _ in range(2)]
        for y in range(ny):
            for x in range(nx):
                u = (self.u[0][y][x], self.u[1][y][x])
                for i in range(3):
                    ph, mu = self.phi[i][y][x], self.mu[i][y][x]
                    for j in range(Q):
                        self.f[i][j][y][x] = self._feq(j, ph, mu, u)
                    for d in range(2):
                        self.hpu[i][d][y][x] = ph * u[d]
                for j in range(Q):
                    self.g[j][y][x] = self._geq(j, 0.0, self.rho[y][x], u)
                    self.l[j][y][x] = W[j] * self.q[y][x] * (1.0 + self._cdot(j, u) / CS2)
                for d in range(2):
                    self.hqu[d][y][x] = self.q[y][x] * u[d]

    # ------------------------------------------------------------ helpers

    @staticmethod
    def _cdot(j, v):
        return C[j][0] * v[0] + C[j][1] * v[1]

    def _fd_node(self, x, y, j):
        """Stencil point x + c_j of Eq. (33): periodic in x; in y periodic or
        the mirror of the first/last row beyond a wall (R11)."""
        xx = (x + C[j][0]) % self.nx
        yy = y + C[j][1]
        if self.walls:
            yy = min(max(yy, 0), self.ny - 1)
        else:
            yy %= self.ny
        return xx, yy

    def _grad(self, fld, x, y):
        gx = gy = 0.0
        for j in range(Q):
            xx, yy = self._fd_node(x, y, j)
            gx += W[j] * C[j][0] * fld[yy][xx]
            gy += W[j] * C[j][1] * fld[yy][xx]
        return gx / CS2, gy / CS2

    def _lap(self, fld, x, y):
        s = 0.0
        for j in range(Q):
            xx, yy = self._fd_node(x, y, j)
            s += 2.0 * W[j] * (fld[yy][xx] - fld[y][x])
        return s / CS2

    def _feq(self, j, ph, mu, u):  # Eq. (35)
        if j == 0:
            return ph - (1.0 - W[0]) * mu
        return W[j] * mu + W[j] * ph * self._cdot(j, u) / CS2

    @staticmethod
    def _s(j, u):  # Eq. (40)
        cu = C[j][0] * u[0] + C[j][1] * u[1]
        return W[j] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - (u[0] * u[0] + u[1] * u[1]) / (2.0 * CS2))

    def _geq(self, j, p, rho, u):  # Eq. (39)
        return (W[j] - 1.0 if j == 0 else W[j]) * p / CS2 + rho * self._s(j, u)

    def _properties(self):
        """Eqs. (29)-(30) at every node."""
        nx, ny = self.nx, self.ny
        self.rho, self.visc, self.sig, self.eps = (_zeros(ny, nx) for _ in range(4))
        for y in range(ny):
            for x in range(nx):
                ph = [self.phi[i][y][x] for i in range(3)]
                self.rho[y][x] = sum(self.rho_i[i] * ph[i] for i in range(3))
                self.visc[y][x] = sum(self.visc_i[i] * ph[i] for i in range(3))
                self.sig[y][x] = sum(self.sig_i[i] * ph[i] for i in range(3))
                self.eps[y][x] = sum(self.eps_i[i] * ph[i] * ph[i] * (3.0 - 2.0 * ph[i]) for i in range(3))

    # ------------------------------------------------------------ potential
    def _pot_and_grad(self, x, y):
        """Eq. (45) with the applied field as an imposed mean gradient (R15):
        potential of the populations and the full gradient."""
        hs = [self.h[j][y][x] for j in range(Q)]
        pot = sum(hs[1:]) / (1.0 - W[0])
        den = (self.eps[y][x] - self.eps_ref) + CS2 * self.tau_h
        g = []
        for d in range(2):
            m = sum(C[j][d] * hs[j] for j in range(Q))
            g.append(-(m + CS2 * self.tau_h * self.Eext[d]) / den)
        return pot, g

    def _potential_field(self):
        return [[self._pot_and_grad(x, y)[0] for x in range(self.nx)] for y in range(self.ny)]

    def _poisson_iteration(self):
        nx, ny = self.nx, self.ny
        post = [_zeros(ny, nx) for _ in range(Q)]
        for y in range(ny):
            for x in range(nx):
                pot, g = self._pot_and_grad(x, y)
                eh = self.eps[y][x] - self.eps_ref
                for j in range(Q):
                    hj = self.h[j][y][x]
                    heq = (W[j] - 1.0 if j == 0 else W[j]) * pot  # Eq. (44)
                    post[j][y][x] = (hj - (hj - heq) / self.tau_h
                                     - (eh / CS2) * W[j] * self._cdot(j, g) / self.tau_h
                                     + VARPI[j] * self.q[y][x])  # Eq. (43)
        self.h = self._pull(post, lambda k, x, y, side: -post[OPP[k]][y][x] + 2.0 * W[k] * self.wall_phi[side])

    def _pull(self, post, beyond):
        """Pull streaming: level(k, x) = post(k, x - c_k), or beyond(k, x, side)
        when x - c_k lies beyond a wall (side 0 bottom, 1 top)."""
        nx, ny = self.nx, self.ny
        out = [_zeros(ny, nx) for _ in range(Q)]
        for k in range(Q):
            for y in range(ny):
                for x in range(nx):
                    sx, sy = (x - C[k][0]) % nx, y - C[k][1]
                    if self.walls and (sy < 0 or sy >= ny):
                        out[k][y][x] = beyond(k, x, y, 0 if sy < 0 else 1)
                    else:
                        out[k][y][x] = post[k][sy % ny][sx]
        return out

    def _solve_potential(self, kmin, kmax, tol):
        adaptive = tol > 0.0 and kmax > kmin
        prev = None
        for k in range(1, kmax + 1):
            cur = self._potential_field()
            r_prev = None
            if k >= 2:
                d2 = sum((cur[y][x] - prev[y][x]) ** 2 for y in range(self.ny) for x in range(self.nx))
                a2 = sum(cur[y][x] ** 2 for y in range(self.ny) for x in range(self.nx))
                r_prev = math.sqrt(d2) / max(math.sqrt(a2), 1e-30)
            prev = cur
            self._poisson_iteration()
            if adaptive and k >= 2 and k >= kmin and r_prev < tol:
                break
        self.psi = self._potential_field()
        for y in range(self.ny):
            for x in range(self.nx):
                _, g = self._pot_and_grad(x, y)
                self.E[0][y][x], self.E[1][y][x] = -g[0], -g[1]

    def _chemical_potential(self):
        """Eq. (20) (R1)."""
        nx, ny = self.nx, self.ny
        self.mu = [_zeros(ny, nx) for _ in range(3)]
        for i in range(3):
            for y in range(ny):
                for x in range(nx):
                    ph = self.phi[i][y][x]
                    e2 = self.E[0][y][x] ** 2 + self.E[1][y][x] ** 2
                    self.mu[i][y][x] = (24.0 / self.Dw * self.lam[i] * ph * (ph - 0.5) * (ph - 1.0)
                                        - 0.75 * self.Dw * self.lam[i] * self._lap(self.phi[i], x, y)
                                        - 0.5 * 6.0 * self.eps_i[i] * ph * (1.0 - ph) * e2)

    # ------------------------------------------------------------ one step
    def step(self, n=1):
        for _ in range(n):
            self._one_step()

    def _one_step(self):
        nx, ny = self.nx, self.ny
        # order parameters and the charge population sum
        for i in range(3):
            for y in range(ny):
                for x in range(nx):
                    self.phi[i][y][x] = sum(self.f[i][j][y][x] for j in range(Q))
        lsum = [[sum(self.l[j][y][x] for j in range(Q)) for x in range(nx)] for y in range(ny)]
        self._properties()
        # charge and Ohmic source with the previous field (Eq. 47, R7)
        for y in range(ny):
            for x in range(nx):
                ge = self._grad(self.eps, x, y)
                gs = self._grad(self.sig, x, y)
                E = (self.E[0][y][x], self.E[1][y][x])
                se = self.sig[y][x] / self.eps[y][x]
                rp = se * (ge[0] * E[0] + ge[1] * E[1]) - (gs[0] * E[0] + gs[1] * E[1])
                qq = (lsum[y][x] + 0.5 * rp) / (1.0 + 0.5 * se)
                self.q[y][x] = qq
                self.R[y][x] = -se * qq + rp
        c = self.cfg
        self._solve_potential(int(c.get("sub_min", 1)), int(c.get("sub_max", 1)), float(c.get("sub_tol", 0.0)))
        self._chemical_potential()
        # collisions
        fpost = [[_zeros(ny, nx) for _ in range(Q)] for _ in range(3)]
        gpost = [_zeros(ny, nx) for _ in range(Q)]
        lpost = [_zeros(ny, nx) for _ in range(Q)]
        for y in range(ny):
            for x in range(nx):
                self._collide_node(x, y, fpost, gpost, lpost)
        # streaming with the wall rules (R10)
        if not self.frozen:
            for i in range(3):
                ph = [row[:] for row in self.phi[i]]
                self.f[i] = self._pull(fpost[i], self._moving_wall(fpost[i], ph))
        self.g = self._pull(gpost, self._moving_wall(gpost, self.rho))
        if self.q_dirichlet:
            self.l = self._pull(lpost, lambda k, x, y, side: -lpost[OPP[k]][y][x] + 2.0 * W[k] * self.wall_q[side])
        else:
            qc = [row[:] for row in self.q]
            self.l = self._pull(lpost, self._moving_wall(lpost, qc))

    def _moving_wall(self, post, carrier):
        def beyond(k, x, y, side):
            j = OPP[k]  # the direction that left the node toward the wall
            return post[j][y][x] - 2.0 * W[j] * carrier[y][x] * C[j][0] * self.wall_u[side] / CS2
        return beyond

    def _collide_node(self, x, y, fpost, gpost, lpost):
        ph = [self.phi[i][y][x] for i in range(3)]
        gmu = [self._grad(self.mu[i], x, y) for i in range(3)]
        grho = self._grad(self.rho, x, y)
        q = self.q[y][x]
        E = (self.E[0][y][x], self.E[1][y][x])
        rho = self.rho[y][x]
        # force of Eq. (27b) (R5) and the moments of Eq. (41)
        F = [q * E[d] - sum(ph[i] * gmu[i][d] for i in range(3)) for d in range(2)]
        gs = [self.g[j][y][x] for j in range(Q)]
        u = [(sum(C[j][d] * gs[j] for j in range(Q)) + 0.5 * F[d]) / rho for d in range(2)]
        udr = u[0] * grho[0] + u[1] * grho[1]
        p = CS2 / (1.0 - W[0]) * (sum(gs[1:]) + 0.5 * udr + rho * self._s(0, u))
        self.u[0][y][x], self.u[1][y][x] = u
        self.p[y][x] = p
        # first-order time derivatives (R8)
        dpu = []
        for i in range(3):
            now = (ph[i] * u[0], ph[i] * u[1])
            dpu.append((now[0] - self.hpu[i][0][y][x], now[1] - self.hpu[i][1][y][x]))
            self.hpu[i][0][y][x], self.hpu[i][1][y][x] = now
        qu = (q * u[0], q * u[1])
        dqu = (qu[0] - self.hqu[0][y][x], qu[1] - self.hqu[1][y][x])
        self.hqu[0][y][x], self.hqu[1][y][x] = qu
        # order-parameter families, Eqs. (34)-(36) with the mobility of Eq. (28)
        if not self.frozen:
            for i in range(3):
                off = [-self.m0 * ph[i] * ph[k] if k != i else 0.0 for k in range(3)]
                mii = -sum(off)
                X = [(mii - self.m0) * gmu[i][d] + sum(off[k] * gmu[k][d] for k in range(3) if k != i)
                     for d in range(2)]
                if self.sum_relax:
                    # restoring flux m0 (phi_i / S) grad S of the order-parameter sum (R23)
                    S = ph[0] + ph[1] + ph[2]
                    gS = [sum(self._grad(self.phi[k], x, y)[d] for k in range(3)) for d in range(2)]
                    X = [X[d] + self.m0 * ph[i] / S * gS[d] for d in range(2)]
                for j in range(Q):
                    fj = self.f[i][j][y][x]
                    Fj = W[j] * (self._cdot(j, dpu[i]) / CS2 - self._cdot(j, X) / self.m0)
                    fpost[i][j][y][x] = (fj - (fj - self._feq(j, ph[i], self.mu[i][y][x], u)) / self.tau_f
                                         + (1.0 - 0.5 / self.tau_f) * Fj)
        # flow family, Eqs. (37)-(40), local tau_g (R6)
        tg = 0.5 + self.visc[y][x] / (rho * CS2)
        for j in range(Q):
            cu = self._cdot(j, u)
            Gb = W[j] * (udr + self._cdot(j, F) / CS2 + (cu * self._cdot(j, grho) - CS2 * udr) / CS2)
            gpost[j][y][x] = gs[j] - (gs[j] - self._geq(j, p, rho, u)) / tg + (1.0 - 0.5 / tg) * Gb
        # charge family, Eqs. (48)-(50)
        cl = 1.0 - 0.5 / self.tau_l
        for j in range(Q):
            lj = self.l[j][y][x]
            leq = W[j] * q * (1.0 + self._cdot(j, u) / CS2)
            lpost[j][y][x] = (lj - (lj - leq) / self.tau_l + cl * W[j] * self.R[y][x]
                              + cl * W[j] * self._cdot(j, dqu) / CS2)

    # ------------------------------------------------------------ outputs
    def fields(self):
        """The fields of the last step (after create: the initial fields),
        named as the C oracle names them."""
        out = {"phi%d" % (i + 1): self.phi[i] for i in range(3)}
        out.update(rho=self.rho, ux=self.u[0], uy=self.u[1], p=self.p, psi=self.psi, Ex=self.E[0],
                   Ey=self.E[1], q=self.q, eps=self.eps, R=self.R)
        out.update({"mu%d" % (i + 1): self.mu[i] for i in range(3)})
        return out

    def pops(self, fam):
        if fam == "f":
            return [self.f[i][j] for i in range(3) for j in range(Q)]
        return {"g": self.g, "l": self.l, "h": self.h}[fam]
