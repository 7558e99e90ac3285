/*
 * FP64 CPU oracle for the three-phase leaky-dielectric EHD lattice Boltzmann
 * step (Liu, Qian, Xiong, Wang: "Onsager-variational-principle-based lattice
 * Boltzmann model for three-phase dielectric fluid flows", arXiv 2608.05787).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it.  It shares no code, header, table
 * or helper with the HIP library, and it never reads anything the HIP path
 * produced.
 *
 * Everything is double precision, one lattice node at a time, one stage at a
 * time, in the order the paper's Sec. 3 describes the scheme.  OpenMP only
 * splits node loops over rows; per-node arithmetic and every reduction order
 * are fixed, so results are bitwise reproducible for any thread count.
 *
 * Two lattices (Sec. 3.1): D2Q9 (Eq. 31) on an nx x ny plane, and D3Q15
 * (Eq. 32) on an nx x ny x nz box.  x (and z) are periodic; y is periodic or
 * bounded by half-way walls.  Node n = (z ny + y) nx + x; vector fields are
 * stored as D planes (x, y[, z]).
 *
 * Where the paper is silent or garbled, the reading taken is stated at the
 * point of use (and listed, numbered R1..R21, in the design notes):
 *   R1  mu_i follows Eq. (20) (derivative form); Eq. (27c) is a misprint.
 *   R2  the CH source Eq. (36) is w_j c_j . [d_t(phi_i u)/cs2 - X_i/m0].
 *   R3  phi_i is the zeroth moment of f^i (sum of f, not of f^eq).
 *   R4  M_ii = -sum_{k!=i} M_ik literally (zero row sums hold exactly).
 *   R5  the -1/2 grad(alpha q^2/sigma) force of Eq. (26) is dropped (Eq. 27b).
 *   R6  tau_g is local: tau_g = 1/2 + mu_v(phi)/(rho cs2), mu_v from Eq. (29).
 *   R7  q = sum l + R/2 is solved for q because R depends on q.
 *   R8  d_t(phi_i u), d_t(q u): first-order backward differences in time.
 *   R9  step order: moments, stencils, charge (with E of the previous step),
 *       potential sub-iterations, mu, grad mu, force/u/p, collisions, streaming.
 *   R10 walls are half-way: bounce-back with the moving-wall term for every
 *       family whose equilibrium carries c_j.(psi u), anti-bounce-back for a
 *       Dirichlet potential (and a Dirichlet charge when asked for).
 *   R11 finite-difference ghosts at walls mirror the first fluid row.
 *   R12 grad(eps), grad(sigma), grad(rho) apply Eq. (33) to the eps, sigma
 *       and rho fields built from phi (Eqs. 29-30) at each stencil node.
 *   R13 potential sub-iterations stop after iteration k once k >= sub_min,
 *       k >= 2 and the potential change of the previous iteration is below
 *       tol; sub_min == sub_max or tol <= 0 runs a fixed count.
 *   R14 the reference permittivity of the h equation is that of one chosen
 *       (bulk) phase: eps_ref = eps[eps_ref_phase], tau_h = 1/2 + eps_ref/cs2.
 *   R15 a uniform applied field E_ext is an imposed mean gradient: the
 *       potential is psi = psi' - E_ext . x with psi' periodic (the h
 *       populations carry psi'); Eq. (42) holds for the full psi, so the
 *       eps_hat source of Eq. (43) and the gradient of Eq. (45) are those of
 *       psi, and E = -grad(psi).  With uniform eps this is the plain sum
 *       E = -grad(psi') + E_ext.
 *   R16 initial populations are the equilibria of the initial fields; the
 *       potential is first iterated with q0 (cold start).
 *   R20 D3Q15: the potential source weights are varpi_0 = 0 and 1/14 for
 *       the 14 moving directions (Eq. 43 gives 1/8 for D2Q9: the same rule,
 *       weights summing to one with zero first moment); every other formula
 *       is written for a general lattice and dimension.
 *   R21 two-ion Nernst-Planck charge model (Eq. 52, symmetric binary
 *       electrolyte, valences +1 and -1): each ion concentration n_s is the
 *       zeroth moment of a BGK advection-diffusion family with equilibrium
 *       w_j n_s (1 + c_j . (u + v_s)/cs2), drift v_s = z_s beta D E (beta =
 *       e/(k_B T), E of the current step), D = cs2 (tau_n - 1/2); the charge
 *       is q = e (n_+ - n_-) with no Ohmic source (conductivities zero);
 *       walls are no-flux bounce-back.  The paper gives no LB for Eq. (52).
 *   R23 (optional, sum_relax) the variable part of the diffusion flux of
 *       phase i in Eq. (36) gains m0 (phi_i / S) grad S, S = phi_1 + phi_2 +
 *       phi_3: the sum diffuses back to the constraint S = 1 and each phase
 *       keeps its mass.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define QMAX 15
static const double CS2 = 1.0 / 3.0;

/* Lattices of Eqs. (31)-(32), c = dx/dt = 1, cs^2 = 1/3. */
typedef struct {
  int Q, D;
  int c[QMAX][3];
  double w[QMAX];
  int opp[QMAX];
  double varpi[QMAX]; /* potential source weights, Eq. (43) (R20) */
} lattice;

static const lattice D2Q9 = {
    9, 2,
    {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0}, {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}},
    {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36},
    {0, 3, 4, 1, 2, 7, 8, 5, 6},
    {0.0, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125}};

static const lattice D3Q15 = {
    15, 3,
    {{0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}, {1, 1, 1},
     {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}},
    {2.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72,
     1.0 / 72, 1.0 / 72, 1.0 / 72, 1.0 / 72},
    {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13},
    {0.0, 1.0 / 14, 1.0 / 14, 1.0 / 14, 1.0 / 14, 1.0 / 14, 1.0 / 14, 1.0 / 14, 1.0 / 14, 1.0 / 14, 1.0 / 14,
     1.0 / 14, 1.0 / 14, 1.0 / 14, 1.0 / 14}};

typedef struct {
  int32_t nx, ny;
  int32_t bc_y;          /* 0 periodic, 1 half-way walls at y=-1/2, ny-1/2 */
  int32_t wall_q_mode;   /* 0 charge bounce-back (no flux), 1 Dirichlet q */
  int32_t eps_ref_phase; /* index of the phase whose eps is eps_ref (R14) */
  int32_t phase_mode;    /* 0 evolve f^1..3, 1 order parameters frozen */
  int32_t sub_min, sub_max;
  int32_t init_sub_max, pad0;
  double sub_tol, init_tol;
  double wall_u[2];   /* tangential (x) wall speed, [0] bottom, [1] top */
  double wall_phi[2]; /* Dirichlet potential at the walls */
  double wall_q[2];   /* Dirichlet charge at the walls (wall_q_mode 1) */
  double E_ext[2];
  double gamma12, gamma13, gamma23, width;
  double rho[3], visc[3], eps[3], sigma[3];
  double tau_f, tau_l;
  int32_t nz;         /* layers in z (1 for D2Q9) */
  int32_t lattice;    /* 0 D2Q9, 1 D3Q15 */
  double E_ext_z;     /* z component of the applied field (D3Q15) */
  int32_t charge_model; /* 0 leaky dielectric (Eqs. 46-50), 1 two-ion Nernst-Planck (R21) */
  int32_t sum_relax;    /* 1: restoring flux of the order-parameter sum (R23) */
  double ion_tau;     /* relaxation time of the ion families: D = cs2 (ion_tau - 1/2) */
  double ion_beta;    /* e / (k_B T) in potential units */
  double ion_charge;  /* e: q = e (n_+ - n_-) */
} or_params;

typedef struct {
  or_params p;
  const lattice *L;
  int nx, ny, nz, N, Q, D;
  double lam[3], m0, alpha, eps_ref, tau_h, Eext[3];
  double *f, *g, *l, *h;       /* populations, [family][q][N]; l holds the two ion
                                  families [2][Q][N] under the Nernst-Planck model */
  double *fn, *gn, *ln, *hn;   /* streaming targets */
  double *phi, *lsum;          /* [3][N], [N] */
  double *rho, *sig, *eps, *visc;
  double *gphi, *lphi;         /* [3][D][N], [3][N] */
  double *grho, *gsig, *geps;  /* [D][N] */
  double *q, *R, *psi, *psi_prev, *E; /* E is [D][N]: E of the last solve */
  double *mu, *gmu;            /* [3][N], [3][D][N] */
  double *u, *pr;              /* [D][N], [N] */
  double *hpu, *hqu;           /* history (phi_i u)^{n-1} [3][D][N], (q u)^{n-1} [D][N] */
  double *ion;                 /* Nernst-Planck: ion concentrations n_+, n_- [2][N] */
  int nl;                      /* families in l: 1, or 2 under the Nernst-Planck model */
  double *rowbuf;              /* per-row partial sums (deterministic reductions) */
  int64_t nstep;
  int k_used;
  double res_last;
} or_state;

/* ---------------------------------------------------------------- helpers */

static double *zalloc(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

static inline int wrap(int v, int n) { return (v % n + n) % n; }

/* Row index of a finite-difference neighbour (R11: mirror ghosts at walls). */
static inline int fd_row(const or_state *s, int y) {
  if (s->p.bc_y == 0) return wrap(y, s->ny);
  if (y < 0) return 0;
  if (y >= s->ny) return s->ny - 1;
  return y;
}

static inline int node(const or_state *s, int x, int y, int z) { return (z * s->ny + y) * s->nx + x; }

/* Isotropic second-order gradient and Laplacian of Eq. (33) at node
 * (x, y, z); g receives D components (may be NULL). */
static void stencil(const or_state *s, const double *chi, int x, int y, int z, double *g, double *lap) {
  const lattice *L = s->L;
  const double c0 = chi[node(s, x, y, z)];
  double sg[3] = {0, 0, 0}, sl = 0;
  for (int j = 0; j < L->Q; ++j) {
    const int xx = wrap(x + L->c[j][0], s->nx), yy = fd_row(s, y + L->c[j][1]);
    const int zz = wrap(z + L->c[j][2], s->nz);
    const double v = chi[node(s, xx, yy, zz)];
    for (int d = 0; d < L->D; ++d) sg[d] += L->w[j] * L->c[j][d] * v;
    sl += 2.0 * L->w[j] * (v - c0);
  }
  if (g)
    for (int d = 0; d < L->D; ++d) g[d] = sg[d] / CS2;
  if (lap) *lap = sl / CS2;
}

/* Eq. (33) on a plane field, writing gradient planes [D][N] and the Laplacian. */
static void stencil_field(or_state *s, const double *chi, double *g, double *lap) {
  const int N = s->N, D = s->D;
#pragma omp parallel for schedule(static)
  for (int r = 0; r < s->ny * s->nz; ++r) {
    const int y = r % s->ny, z = r / s->ny;
    for (int x = 0; x < s->nx; ++x) {
      const int n = node(s, x, y, z);
      double gg[3];
      stencil(s, chi, x, y, z, g ? gg : NULL, lap ? lap + n : NULL);
      if (g)
        for (int d = 0; d < D; ++d) g[d * N + n] = gg[d];
    }
  }
}

static double dotc(const lattice *L, int j, const double *v) {
  double a = 0;
  for (int d = 0; d < L->D; ++d) a += L->c[j][d] * v[d];
  return a;
}

/* Properties of Eqs. (29)-(30). */
static double prop_lin(const double *c, double p1, double p2, double p3) {
  return c[0] * p1 + c[1] * p2 + c[2] * p3;
}
static double herm(double ph) { return ph * ph * (3.0 - 2.0 * ph); }
static double prop_eps(const double *e, double p1, double p2, double p3) {
  return e[0] * herm(p1) + e[1] * herm(p2) + e[2] * herm(p3);
}

/*
 * Streaming of one family with half-way walls (R10).
 * post: post-collision values; dst: pre-collision values of the next level.
 * mode 0: bounce-back with moving-wall term -2 w_j psi (c_j . u_w)/cs2,
 *         psi per node given by `carrier` (NULL means psi = 0).
 * mode 1: anti-bounce-back for a Dirichlet value (bot, top): -post + 2 w_j v.
 */
static void stream_family(const or_state *s, const double *post, double *dst,
                          int mode, const double *carrier, double bot, double top) {
  const lattice *L = s->L;
  const int nx = s->nx, ny = s->ny, N = s->N;
#pragma omp parallel for schedule(static)
  for (int r = 0; r < ny * s->nz; ++r) {
    const int y = r % ny, z = r / ny;
    for (int x = 0; x < nx; ++x) {
      const int n = node(s, x, y, z);
      for (int j = 0; j < L->Q; ++j) {
        const double v = post[j * N + n];
        const int xd = wrap(x + L->c[j][0], nx), zd = wrap(z + L->c[j][2], s->nz);
        int yd = y + L->c[j][1];
        if (s->p.bc_y == 0) {
          dst[j * N + node(s, xd, wrap(yd, ny), zd)] = v;
        } else if (yd >= 0 && yd < ny) {
          dst[j * N + node(s, xd, yd, zd)] = v;
        } else {
          const int side = (yd < 0) ? 0 : 1;
          double out;
          if (mode == 0) {
            const double psi = carrier ? carrier[n] : 0.0;
            out = v - 2.0 * L->w[j] * psi * (L->c[j][0] * s->p.wall_u[side]) / CS2;
          } else {
            out = -v + 2.0 * L->w[j] * (side ? top : bot);
          }
          dst[L->opp[j] * N + n] = out;
        }
      }
    }
  }
}

static void swap_ptr(double **a, double **b) {
  double *t = *a;
  *a = *b;
  *b = t;
}

/* ------------------------------------------------------ potential (h) LB */

/* Potential and the gradient of the full potential from the local h
 * moments, Eq. (45).  The populations carry the periodic part psi' of the
 * potential psi = psi' - E_ext . x (R15); the eps_hat source of Eq. (43)
 * carries eps_hat grad(psi), so the first moment is
 * -(cs2 tau_h) grad(psi') - eps_hat grad(psi), which gives
 * grad(psi) = -(m + cs2 tau_h E_ext) / (eps_hat + cs2 tau_h). */
static void h_moments(const or_state *s, int n, double epshat, double *pot, double *g) {
  const lattice *L = s->L;
  const int N = s->N;
  double s0 = 0, m[3] = {0, 0, 0};
  for (int j = 1; j < L->Q; ++j) s0 += s->h[j * N + n];
  for (int j = 0; j < L->Q; ++j)
    for (int d = 0; d < L->D; ++d) m[d] += L->c[j][d] * s->h[j * N + n];
  *pot = s0 / (1.0 - L->w[0]);
  const double den = epshat + CS2 * s->tau_h;
  for (int d = 0; d < L->D; ++d) g[d] = -(m[d] + CS2 * s->tau_h * s->Eext[d]) / den;
}

static void eval_potential(or_state *s, double *dst) {
#pragma omp parallel for schedule(static)
  for (int n = 0; n < s->N; ++n) {
    double g[3];
    h_moments(s, n, s->eps[n] - s->eps_ref, &dst[n], g);
  }
}

/* One potential sub-iteration: collision of Eq. (43) with the equilibrium of
 * Eq. (44), then streaming with anti-bounce-back electrodes. */
static void poisson_iteration(or_state *s) {
  const lattice *L = s->L;
  const int N = s->N;
  const double th = s->tau_h;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    const double epshat = s->eps[n] - s->eps_ref;
    double pot, g[3];
    h_moments(s, n, epshat, &pot, g);
    for (int j = 0; j < L->Q; ++j) {
      const double hj = s->h[j * N + n];
      const double heq = (j == 0) ? (L->w[0] - 1.0) * pot : L->w[j] * pot;
      const double cg = dotc(L, j, g);
      s->hn[j * N + n] = hj - (hj - heq) / th - (epshat / CS2) * L->w[j] * cg / th + L->varpi[j] * s->q[n];
    }
  }
  /* collided values are in hn; stream them back into h */
  stream_family(s, s->hn, s->h, 1, NULL, s->p.wall_phi[0], s->p.wall_phi[1]);
}

static double rel_change(or_state *s, const double *a, const double *b) {
  const int nx = s->nx, R = s->ny * s->nz;
#pragma omp parallel for schedule(static)
  for (int r = 0; r < R; ++r) {
    double d2 = 0, a2 = 0;
    for (int x = 0; x < nx; ++x) {
      const double d = a[r * nx + x] - b[r * nx + x];
      d2 += d * d;
      a2 += a[r * nx + x] * a[r * nx + x];
    }
    s->rowbuf[2 * r] = d2;
    s->rowbuf[2 * r + 1] = a2;
  }
  double d2 = 0, a2 = 0;
  for (int r = 0; r < R; ++r) {
    d2 += s->rowbuf[2 * r];
    a2 += s->rowbuf[2 * r + 1];
  }
  const double na = sqrt(a2);
  return sqrt(d2) / (na > 1e-30 ? na : 1e-30);
}

/* Sub-iteration loop with the stopping rule R13.  On return psi holds the
 * potential of the final h, res_last the relative change of the potential over
 * the last iteration, and E = -grad(psi) of the full potential (Eq. 45, R15). */
static void solve_potential(or_state *s, int kmin, int kmax, double tol) {
  const int adaptive = (tol > 0.0) && (kmax > kmin);
  int kdone = kmax > 0 ? kmax : 0;
  double r_prev = 0.0;
  for (int k = 1; k <= kmax; ++k) {
    eval_potential(s, s->psi); /* phi_{k-1}: potential of this iteration's input */
    if (k >= 2) r_prev = rel_change(s, s->psi, s->psi_prev); /* phi_{k-2} -> phi_{k-1} */
    swap_ptr(&s->psi, &s->psi_prev);                         /* psi_prev := phi_{k-1} */
    poisson_iteration(s);
    if (adaptive && k >= 2 && k >= kmin && r_prev < tol) {
      kdone = k;
      break;
    }
  }
  s->k_used = kdone;
  eval_potential(s, s->psi); /* phi_K */
  s->res_last = (kdone > 0) ? rel_change(s, s->psi, s->psi_prev) : 0.0;
  const int N = s->N, D = s->D;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    double pot, g[3];
    h_moments(s, n, s->eps[n] - s->eps_ref, &pot, g);
    for (int d = 0; d < D; ++d) s->E[d * N + n] = -g[d];
  }
}

/* ------------------------------------------------------------ other steps */

/* Order-parameter and charge moments (R3): phi_i = sum_j f^i_j. */
static void moments(or_state *s) {
  const int N = s->N, Q = s->Q;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    for (int i = 0; i < 3; ++i) {
      double a = 0;
      for (int j = 0; j < Q; ++j) a += s->f[(i * Q + j) * N + n];
      s->phi[i * N + n] = a;
    }
    if (s->p.charge_model == 1) {
      /* ion concentrations and the charge they carry (R21) */
      for (int k = 0; k < 2; ++k) {
        double a = 0;
        for (int j = 0; j < Q; ++j) a += s->l[(k * Q + j) * N + n];
        s->ion[k * N + n] = a;
      }
      s->lsum[n] = s->p.ion_charge * (s->ion[n] - s->ion[N + n]);
    } else {
      double b = 0;
      for (int j = 0; j < Q; ++j) b += s->l[j * N + n];
      s->lsum[n] = b;
    }
  }
}

/* Properties (Eqs. 29-30) and the Eq. (33) stencils of phi_i, rho, sigma, eps. */
static void properties_and_stencils(or_state *s) {
  const int N = s->N, D = s->D;
  const or_params *P = &s->p;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    const double p1 = s->phi[n], p2 = s->phi[N + n], p3 = s->phi[2 * N + n];
    s->rho[n] = prop_lin(P->rho, p1, p2, p3);
    s->visc[n] = prop_lin(P->visc, p1, p2, p3);
    s->sig[n] = prop_lin(P->sigma, p1, p2, p3);
    s->eps[n] = prop_eps(P->eps, p1, p2, p3);
  }
  for (int i = 0; i < 3; ++i) stencil_field(s, s->phi + i * N, s->gphi + i * D * N, s->lphi + i * N);
  stencil_field(s, s->rho, s->grho, NULL);
  stencil_field(s, s->sig, s->gsig, NULL);
  stencil_field(s, s->eps, s->geps, NULL);
}

/* Charge density and the Ohmic source, Eq. (47) with R7; E of the previous
 * step (R9). */
static void charge(or_state *s) {
  const int N = s->N, D = s->D;
  if (s->p.charge_model == 1) {
    /* Nernst-Planck: the ions carry the charge, no Ohmic source (R21) */
    for (int n = 0; n < N; ++n) {
      s->q[n] = s->lsum[n];
      s->R[n] = 0.0;
    }
    return;
  }
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    const double se = s->sig[n] / s->eps[n];
    double ge = 0, gs = 0;
    for (int d = 0; d < D; ++d) {
      ge += s->geps[d * N + n] * s->E[d * N + n];
      gs += s->gsig[d * N + n] * s->E[d * N + n];
    }
    const double Rp = se * ge - gs;
    const double qq = (s->lsum[n] + 0.5 * Rp) / (1.0 + 0.5 * se);
    s->q[n] = qq;
    s->R[n] = -se * qq + Rp;
  }
}

/* Chemical potentials, Eq. (20) with eps'(phi_i) = 6 eps_i phi_i (1-phi_i) (R1). */
static void chem_potential(or_state *s) {
  const int N = s->N, D = s->D;
  const double Dw = s->p.width;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    double e2 = 0;
    for (int d = 0; d < D; ++d) e2 += s->E[d * N + n] * s->E[d * N + n];
    for (int i = 0; i < 3; ++i) {
      const double ph = s->phi[i * N + n];
      const double bulk = 24.0 / Dw * s->lam[i] * ph * (ph - 0.5) * (ph - 1.0);
      const double grad = 0.75 * Dw * s->lam[i] * s->lphi[i * N + n];
      const double elec = 0.5 * (6.0 * s->p.eps[i] * ph * (1.0 - ph)) * e2;
      s->mu[i * N + n] = bulk - grad - elec;
    }
  }
  for (int i = 0; i < 3; ++i) stencil_field(s, s->mu + i * N, s->gmu + i * D * N, NULL);
}

/* Body force of Eq. (27b) (R5) and the flow moments of Eq. (41). */
static void force_and_flow(or_state *s, int n, double *F, double *u, double *pp) {
  const lattice *L = s->L;
  const int N = s->N, D = s->D;
  double m[3] = {0, 0, 0}, s1 = 0;
  for (int d = 0; d < D; ++d) {
    F[d] = s->q[n] * s->E[d * N + n];
    for (int i = 0; i < 3; ++i) F[d] -= s->phi[i * N + n] * s->gmu[(i * D + d) * N + n];
  }
  for (int j = 0; j < L->Q; ++j) {
    for (int d = 0; d < D; ++d) m[d] += L->c[j][d] * s->g[j * N + n];
    if (j) s1 += s->g[j * N + n];
  }
  const double rho = s->rho[n];
  double udr = 0, usq = 0;
  for (int d = 0; d < D; ++d) {
    u[d] = (m[d] + 0.5 * F[d]) / rho;
    udr += u[d] * s->grho[d * N + n];
    usq += u[d] * u[d];
  }
  const double s0 = L->w[0] * (-usq / (2.0 * CS2));
  *pp = CS2 / (1.0 - L->w[0]) * (s1 + 0.5 * udr + rho * s0);
}

/* R23 (sum_relax on): component d of the flux m0 (phi_i / S) grad S added to
 * the variable part of the diffusion flux of phase i, S = phi_1 + phi_2 +
 * phi_3; grad S is the sum of the Eq. (33) gradients of the three.  Summed
 * over i it is m0 grad S: the sum diffuses back to one while every phase's
 * mass stays conserved. */
static double restoring_flux(const or_state *s, const double *ph, int i, int d, int n) {
  const int N = s->N, D = s->D;
  double gS = 0;
  for (int k = 0; k < 3; ++k) gS += s->gphi[(k * D + d) * N + n];
  return s->m0 * ph[i] / (ph[0] + ph[1] + ph[2]) * gS;
}

/* Collisions of Eqs. (34)-(36), (37)-(40) and (48)-(50). */
static void collide(or_state *s) {
  const lattice *L = s->L;
  const int N = s->N, D = s->D, Q = s->Q;
  const or_params *P = &s->p;
  const double tf = P->tau_f, tl = P->tau_l, m0 = s->m0;
#pragma omp parallel for schedule(static)
  for (int n = 0; n < N; ++n) {
    double F[3], u[3], pp;
    force_and_flow(s, n, F, u, &pp);
    for (int d = 0; d < D; ++d) s->u[d * N + n] = u[d];
    s->pr[n] = pp;
    const double rho = s->rho[n];
    double usq = 0;
    for (int d = 0; d < D; ++d) usq += u[d] * u[d];

    /* time derivatives of phi_i u and q u (R8), history update */
    double dpu[3][3], dq[3];
    for (int i = 0; i < 3; ++i) {
      const double ph = s->phi[i * N + n];
      for (int d = 0; d < D; ++d) {
        dpu[i][d] = ph * u[d] - s->hpu[(i * D + d) * N + n];
        s->hpu[(i * D + d) * N + n] = ph * u[d];
      }
    }
    const double qq = s->q[n];
    for (int d = 0; d < D; ++d) {
      dq[d] = qq * u[d] - s->hqu[d * N + n];
      s->hqu[d * N + n] = qq * u[d];
    }

    /* three order-parameter families */
    if (P->phase_mode == 0) {
      double ph[3], Mm[3][3];
      for (int i = 0; i < 3; ++i) ph[i] = s->phi[i * N + n];
      /* degenerate mobility, Eq. (28), with R4 */
      for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) Mm[i][k] = (i == k) ? 0.0 : -m0 * ph[i] * ph[k];
      for (int i = 0; i < 3; ++i) {
        double d = 0;
        for (int k = 0; k < 3; ++k)
          if (k != i) d -= Mm[i][k];
        Mm[i][i] = d;
      }
      for (int i = 0; i < 3; ++i) {
        /* variable part of the diffusion flux (split mobility) */
        double X[3];
        for (int d = 0; d < D; ++d) {
          X[d] = (Mm[i][i] - m0) * s->gmu[(i * D + d) * N + n];
          for (int k = 0; k < 3; ++k)
            if (k != i) X[d] += Mm[i][k] * s->gmu[(k * D + d) * N + n];
          if (P->sum_relax) X[d] += restoring_flux(s, ph, i, d, n);
        }
        const double mu = s->mu[i * N + n];
        for (int j = 0; j < Q; ++j) {
          const double fj = s->f[(i * Q + j) * N + n];
          const double cu = ph[i] * dotc(L, j, u);
          const double feq = (j == 0) ? ph[i] - (1.0 - L->w[0]) * mu : L->w[j] * mu + L->w[j] * cu / CS2;
          /* source of Eq. (36), reading R2 */
          const double Fj = L->w[j] * (dotc(L, j, dpu[i]) / CS2 - dotc(L, j, X) / m0);
          s->fn[(i * Q + j) * N + n] = fj - (fj - feq) / tf + (1.0 - 0.5 / tf) * Fj;
        }
      }
    }

    /* flow family: local tau_g (R6), forcing of Eq. (38), equilibrium (39)-(40) */
    const double tg = 0.5 + s->visc[n] / (rho * CS2);
    double gr[3], udr = 0;
    for (int d = 0; d < D; ++d) {
      gr[d] = s->grho[d * N + n];
      udr += u[d] * gr[d];
    }
    for (int j = 0; j < Q; ++j) {
      const double gj = s->g[j * N + n];
      const double cu = dotc(L, j, u);
      const double sj = L->w[j] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - usq / (2.0 * CS2));
      const double geq = ((j == 0) ? (L->w[0] - 1.0) * pp / CS2 : L->w[j] * pp / CS2) + rho * sj;
      const double cF = dotc(L, j, F);
      const double cgr = dotc(L, j, gr);
      const double Gb = L->w[j] * (udr + cF / CS2 + (cu * cgr - CS2 * udr) / CS2);
      s->gn[j * N + n] = gj - (gj - geq) / tg + (1.0 - 0.5 / tg) * Gb;
    }

    if (P->charge_model == 1) {
      /* two ion families (R21): BGK advection-diffusion with the drift
         velocity z_s beta D E of the current field */
      const double tn = P->ion_tau, Dn = CS2 * (tn - 0.5);
      for (int k = 0; k < 2; ++k) {
        const double z = k == 0 ? 1.0 : -1.0, ns = s->ion[k * N + n];
        double v[3];
        for (int d = 0; d < D; ++d) v[d] = u[d] + z * P->ion_beta * Dn * s->E[d * N + n];
        for (int j = 0; j < Q; ++j) {
          const double mj = s->l[(k * Q + j) * N + n];
          const double meq = L->w[j] * ns * (1.0 + dotc(L, j, v) / CS2);
          s->ln[(k * Q + j) * N + n] = mj - (mj - meq) / tn;
        }
      }
      continue;
    }

    /* charge family, Eqs. (48)-(50) */
    const double Rn = s->R[n];
    for (int j = 0; j < Q; ++j) {
      const double lj = s->l[j * N + n];
      const double cu = dotc(L, j, u);
      const double leq = L->w[j] * qq * (1.0 + cu / CS2);
      const double Sj = (1.0 - 0.5 / tl) * L->w[j] * Rn;
      const double Tj = (1.0 - 0.5 / tl) * L->w[j] * dotc(L, j, dq) / CS2;
      s->ln[j * N + n] = lj - (lj - leq) / tl + Sj + Tj;
    }
  }
}

static void stream_all(or_state *s) {
  const int N = s->N, Q = s->Q;
  if (s->p.phase_mode == 0) {
    for (int i = 0; i < 3; ++i)
      stream_family(s, s->fn + i * Q * N, s->f + i * Q * N, 0, s->phi + i * N, 0, 0);
  }
  stream_family(s, s->gn, s->g, 0, s->rho, 0, 0);
  if (s->p.charge_model == 1) {
    for (int k = 0; k < 2; ++k) stream_family(s, s->ln + k * Q * N, s->l + k * Q * N, 0, s->ion + k * N, 0, 0);
    return;
  }
  if (s->p.wall_q_mode == 1)
    stream_family(s, s->ln, s->l, 1, NULL, s->p.wall_q[0], s->p.wall_q[1]);
  else
    stream_family(s, s->ln, s->l, 0, s->q, 0, 0);
}

/* ---------------------------------------------------------------- public */

void or_free(or_state *s) {
  if (!s) return;
  double **all[] = {&s->f, &s->g, &s->l, &s->h, &s->fn, &s->gn, &s->ln, &s->hn,
                    &s->phi, &s->lsum, &s->rho, &s->sig, &s->eps, &s->visc,
                    &s->gphi, &s->lphi, &s->grho, &s->gsig, &s->geps, &s->q,
                    &s->R, &s->psi, &s->psi_prev, &s->E, &s->mu, &s->gmu,
                    &s->u, &s->pr, &s->hpu, &s->hqu, &s->ion, &s->rowbuf};
  for (size_t i = 0; i < sizeof(all) / sizeof(all[0]); ++i) free(*all[i]);
  free(s);
}

/* Create: parameter mapping, initial fields, cold-start potential, equilibria.
 * phi0 [3][N] (required); u0 [D][N], q0 [N], psi0 [N] may be NULL (zero);
 * ions0 [2][N] (n_+, n_-; Nernst-Planck model only, then required; q0 is
 * ignored and q = e (n_+ - n_-)).  Returns NULL on invalid parameters. */
or_state *or_create(const or_params *P, const double *phi0, const double *u0,
                    const double *q0, const double *psi0, const double *ions0) {
  if (!P || !phi0 || P->nx < 1 || P->ny < 1) return NULL;
  if (P->tau_f <= 0.5 || P->tau_l <= 0.5) return NULL;
  if (P->eps_ref_phase < 0 || P->eps_ref_phase > 2) return NULL;
  if (P->lattice != 0 && P->lattice != 1) return NULL;
  if (P->lattice == 0 && P->nz != 1) return NULL;
  if (P->nz < 1) return NULL;
  if (P->charge_model != 0 && P->charge_model != 1) return NULL;
  if (P->charge_model == 1 && (!ions0 || P->ion_tau <= 0.5)) return NULL;
  or_state *s = (or_state *)calloc(1, sizeof(or_state));
  s->p = *P;
  s->L = P->lattice == 1 ? &D3Q15 : &D2Q9;
  s->Q = s->L->Q;
  s->D = s->L->D;
  s->nx = P->nx;
  s->ny = P->ny;
  s->nz = P->nz;
  const int N = s->N = P->nx * P->ny * P->nz;
  const int Q = s->Q, D = s->D;
  /* spreading coefficients, Eq. (9) */
  s->lam[0] = P->gamma12 + P->gamma13 - P->gamma23;
  s->lam[1] = P->gamma12 + P->gamma23 - P->gamma13;
  s->lam[2] = P->gamma13 + P->gamma23 - P->gamma12;
  /* relaxation-time couplings: m0 (Eq. 34 text), alpha (Eq. 49 text), tau_h */
  s->m0 = CS2 * (P->tau_f - 0.5);
  s->alpha = CS2 * (P->tau_l - 0.5);
  s->eps_ref = P->eps[P->eps_ref_phase];
  s->tau_h = 0.5 + s->eps_ref / CS2;
  s->Eext[0] = P->E_ext[0];
  s->Eext[1] = P->E_ext[1];
  s->Eext[2] = P->E_ext_z;

  s->f = zalloc(3 * Q * (size_t)N); s->fn = zalloc(3 * Q * (size_t)N);
  s->g = zalloc(Q * (size_t)N);  s->gn = zalloc(Q * (size_t)N);
  s->nl = P->charge_model == 1 ? 2 : 1;
  s->l = zalloc(s->nl * Q * (size_t)N);  s->ln = zalloc(s->nl * Q * (size_t)N);
  s->ion = zalloc(2 * (size_t)N);
  s->h = zalloc(Q * (size_t)N);  s->hn = zalloc(Q * (size_t)N);
  s->phi = zalloc(3 * (size_t)N); s->lsum = zalloc(N);
  s->rho = zalloc(N); s->sig = zalloc(N); s->eps = zalloc(N); s->visc = zalloc(N);
  s->gphi = zalloc(3 * D * (size_t)N); s->lphi = zalloc(3 * (size_t)N);
  s->grho = zalloc(D * (size_t)N); s->gsig = zalloc(D * (size_t)N);
  s->geps = zalloc(D * (size_t)N);
  s->q = zalloc(N); s->R = zalloc(N); s->psi = zalloc(N); s->psi_prev = zalloc(N);
  s->E = zalloc(D * (size_t)N);
  s->mu = zalloc(3 * (size_t)N); s->gmu = zalloc(3 * D * (size_t)N);
  s->u = zalloc(D * (size_t)N); s->pr = zalloc(N);
  s->hpu = zalloc(3 * D * (size_t)N); s->hqu = zalloc(D * (size_t)N);
  s->rowbuf = zalloc(2 * (size_t)s->ny * s->nz);

  memcpy(s->phi, phi0, 3 * (size_t)N * sizeof(double));
  if (u0) memcpy(s->u, u0, D * (size_t)N * sizeof(double));
  if (P->charge_model == 1) {
    memcpy(s->ion, ions0, 2 * (size_t)N * sizeof(double));
    for (int n = 0; n < N; ++n) s->q[n] = P->ion_charge * (s->ion[n] - s->ion[N + n]);
  } else if (q0) {
    memcpy(s->q, q0, (size_t)N * sizeof(double));
  }
  properties_and_stencils(s);

  /* potential: equilibrium of the initial guess, then cold-start iterations
     with the initial charge (R16) */
  for (int n = 0; n < N; ++n) {
    const double v = psi0 ? psi0[n] : 0.0;
    for (int j = 0; j < Q; ++j) s->h[j * N + n] = (j == 0) ? (s->L->w[0] - 1.0) * v : s->L->w[j] * v;
  }
  solve_potential(s, 1, P->init_sub_max, P->init_tol);
  chem_potential(s);

  /* equilibria of the initial fields; p = 0 */
  const lattice *L = s->L;
  for (int n = 0; n < N; ++n) {
    double u[3] = {0, 0, 0}, usq = 0;
    for (int d = 0; d < D; ++d) {
      u[d] = s->u[d * N + n];
      usq += u[d] * u[d];
    }
    const double rho = s->rho[n];
    for (int i = 0; i < 3; ++i) {
      const double ph = s->phi[i * N + n], mu = s->mu[i * N + n];
      for (int j = 0; j < Q; ++j) {
        const double cu = ph * dotc(L, j, u);
        s->f[(i * Q + j) * N + n] = (j == 0) ? ph - (1.0 - L->w[0]) * mu : L->w[j] * mu + L->w[j] * cu / CS2;
      }
      for (int d = 0; d < D; ++d) s->hpu[(i * D + d) * N + n] = ph * u[d];
    }
    for (int j = 0; j < Q; ++j) {
      const double cu = dotc(L, j, u);
      s->g[j * N + n] = rho * L->w[j] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - usq / (2.0 * CS2));
      if (P->charge_model == 0) s->l[j * N + n] = L->w[j] * s->q[n] * (1.0 + cu / CS2);
    }
    if (P->charge_model == 1) {
      /* ion equilibria with the drift of the cold-start field */
      const double Dn = CS2 * (P->ion_tau - 0.5);
      for (int k = 0; k < 2; ++k) {
        const double z = k == 0 ? 1.0 : -1.0, ns = s->ion[k * N + n];
        double v[3];
        for (int d = 0; d < D; ++d) v[d] = u[d] + z * P->ion_beta * Dn * s->E[d * N + n];
        for (int j = 0; j < Q; ++j) s->l[(k * Q + j) * N + n] = L->w[j] * ns * (1.0 + dotc(L, j, v) / CS2);
      }
    }
    for (int d = 0; d < D; ++d) s->hqu[d * N + n] = s->q[n] * u[d];
    s->pr[n] = 0.0;
  }
  s->nstep = 0;
  return s;
}

/* n time steps, each in the order R9. */
void or_step(or_state *s, int64_t nsteps) {
  for (int64_t t = 0; t < nsteps; ++t) {
    moments(s);
    properties_and_stencils(s);
    charge(s);
    solve_potential(s, s->p.sub_min, s->p.sub_max, s->p.sub_tol);
    chem_potential(s);
    collide(s);
    stream_all(s);
    s->nstep++;
  }
}

/* Field ids for or_field; fields are those computed during the last step
 * (after create: the initial fields).  UZ and EZ are zero on D2Q9. */
enum {
  OR_PHI1 = 0, OR_PHI2, OR_PHI3, OR_RHO, OR_UX, OR_UY, OR_P, OR_PSI, OR_EX, OR_EY,
  OR_Q, OR_MU1, OR_MU2, OR_MU3, OR_EPS, OR_R, OR_UZ, OR_EZ, OR_NPLUS, OR_NMINUS, OR_NFIELDS
};

int or_field(const or_state *s, int id, double *out) {
  const int N = s->N;
  const double *src = NULL;
  switch (id) {
    case OR_PHI1: case OR_PHI2: case OR_PHI3: src = s->phi + (id - OR_PHI1) * N; break;
    case OR_RHO: src = s->rho; break;
    case OR_UX: src = s->u; break;
    case OR_UY: src = s->u + N; break;
    case OR_UZ: src = s->D == 3 ? s->u + 2 * N : NULL; break;
    case OR_P: src = s->pr; break;
    case OR_PSI: src = s->psi; break;
    case OR_EX: src = s->E; break;
    case OR_EY: src = s->E + N; break;
    case OR_EZ: src = s->D == 3 ? s->E + 2 * N : NULL; break;
    case OR_Q: src = s->q; break;
    case OR_MU1: case OR_MU2: case OR_MU3: src = s->mu + (id - OR_MU1) * N; break;
    case OR_EPS: src = s->eps; break;
    case OR_R: src = s->R; break;
    case OR_NPLUS: case OR_NMINUS: src = s->p.charge_model == 1 ? s->ion + (id - OR_NPLUS) * N : NULL; break;
    default: return -1;
  }
  if (src)
    memcpy(out, src, (size_t)N * sizeof(double));
  else
    memset(out, 0, (size_t)N * sizeof(double));
  return 0;
}

/* Raw pre-collision populations of the current level.
 * fam 0: f [3][Q][N], 1: g [Q][N], 2: l [Q][N] (ions: [2][Q][N]), 3: h [Q][N]. */
int or_pops(const or_state *s, int fam, double *out) {
  const size_t N = (size_t)s->N, Q = (size_t)s->Q;
  switch (fam) {
    case 0: memcpy(out, s->f, 3 * Q * N * sizeof(double)); return 0;
    case 1: memcpy(out, s->g, Q * N * sizeof(double)); return 0;
    case 2: memcpy(out, s->l, s->nl * Q * N * sizeof(double)); return 0;
    case 3: memcpy(out, s->h, Q * N * sizeof(double)); return 0;
    default: return -1;
  }
}

/* Scalars: [0] steps, [1] sub-iterations of the last solve, [2] residual of
 * the last solve, [3..5] lambda_i, [6] m0, [7] alpha, [8] tau_h. */
void or_scalars(const or_state *s, double *out) {
  out[0] = (double)s->nstep;
  out[1] = s->k_used;
  out[2] = s->res_last;
  out[3] = s->lam[0];
  out[4] = s->lam[1];
  out[5] = s->lam[2];
  out[6] = s->m0;
  out[7] = s->alpha;
  out[8] = s->tau_h;
}

/* Eq. (33) on a plain field (unit checks of the stencil): g [D][N], lap [N]. */
void or_stencil(const or_params *P, const double *chi, double *g, double *lap) {
  or_state tmp;
  memset(&tmp, 0, sizeof(tmp));
  tmp.p = *P;
  tmp.L = P->lattice == 1 ? &D3Q15 : &D2Q9;
  tmp.Q = tmp.L->Q;
  tmp.D = tmp.L->D;
  tmp.nx = P->nx;
  tmp.ny = P->ny;
  tmp.nz = P->nz > 0 ? P->nz : 1;
  tmp.N = P->nx * P->ny * tmp.nz;
  for (int z = 0; z < tmp.nz; ++z)
    for (int y = 0; y < tmp.ny; ++y)
      for (int x = 0; x < tmp.nx; ++x) {
        const int n = node(&tmp, x, y, z);
        double gg[3];
        stencil(&tmp, chi, x, y, z, gg, lap + n);
        for (int d = 0; d < tmp.D; ++d) g[d * tmp.N + n] = gg[d];
      }
}

int or_sizeof_params(void) { return (int)sizeof(or_params); }
