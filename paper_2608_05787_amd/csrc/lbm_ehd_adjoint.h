// Reverse-mode (discrete adjoint) kernels of the three-phase EHD LB step for
// gfx950, on the D2Q9 lattice.  Included once, by lbm_ehd.hip, after
// lbm_ehd_kernels.h.
//
// The adjoint of one time step runs the step's kernels backwards: the
// collide-and-push kernel (flow, charge and order-parameter families), the
// chemical-potential kernel, the potential sub-iterations (last first), the
// charge-recovery kernel and the order-parameter moments.  Each adjoint
// kernel is a gather: the transpose of a push is a pull from the slots the
// node pushed to, and the transpose of an Eq. (33) stencil is a sum over the
// nodes whose stencil reaches this node (mirror ghosts included).  So every
// thread writes only its own node and no atomics are needed.  Forward values
// come from the step's record (Rec, written by the forward kernels during a
// recording run) and are recomputed locally where cheaper.
//
// Adjoint state between steps (planes of N values, type T):
//   a[2]   f 27, g 9, l 9 (adjoint of the populations a step reads, without
//          the moment part), hpu 6, hqu 2, E 2 (previous-step field)
//   hb[2]  potential populations 9 (ping-pong over the sub-iterations)
//   pb[2]  phi 3 and sum-of-l 1: the adjoint of the step's moments, which
//          the next (earlier) step's pull adds to every f^i_j and l_j.
// Parameter adjoints (d/d eps_i, d/d sigma_i, d/d E0) accumulate in per-block
// FP64 slots, block b owning slot b: the sweep's kernels run in stream order,
// so += needs no atomics, and the final sum has a fixed order.
#pragma once

namespace lbm {

constexpr int ADJ_PLANES = 55;  // f 27, g 9, l 9, hpu 6, hqu 2, E 2
constexpr int AO_G = 27, AO_L = 36, AO_HPU = 45, AO_HQU = 51, AO_E = 53;
constexpr int TB_SLOTS = 8;     // eps 3, sigma 3, E0 1, spare

template <typename T> struct AdjBufs {
  T *a[2], *hb[2], *pb[2];
  // per-step intermediates: mu-bar (local part) 3, grad(mu)-bar 6,
  // grad(rho)-bar 2, q-bar, R-bar, E-bar of the step's field 2, eps-bar,
  // Laplacian-bar 3, and with the restoring flux of the order-parameter
  // sum S, grad(S)-bar 2
  T *muL, *gm, *gr, *qb, *rb, *en, *eb, *lb, *gS;
  double *tb;      // nblk x TB_SLOTS
  double dEext[2]; // d E_ext / d E0
  double dwall[2]; // d wall_phi / d E0
};

// v c_x(j) and v c_y(j) for the D2Q9 components -1, 0, 1: exact; a zero
// component gives -0, which an addition drops at compile time, so the
// unrolled loops carry no multiplications by zero.
template <typename T> __device__ __forceinline__ T mcx(int j, T v) { return cx(j) > 0 ? v : (cx(j) < 0 ? -v : T(-0.0)); }
template <typename T> __device__ __forceinline__ T mcy(int j, T v) { return cy(j) > 0 ? v : (cy(j) < 0 ? -v : T(-0.0)); }

// Destination slot of the population (x, y, j) pushed by the forward step:
// returns false at a wall, where the slot is (opp(j), this node).
__device__ __forceinline__ bool push_slot(const Inst &I, int x, int y, int n, int j, size_t &slot, int &dn,
                                          bool &top) {
  const int nx = I.nx, ny = I.ny, N = I.N;
  const int xd = wrapx(x + cx(j), nx);
  int yd = y + cy(j);
  top = yd >= ny;
  if (!I.bc_y) {
    yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
  } else if (yd < 0 || yd >= ny) {
    dn = n;
    slot = (size_t)opp(j) * N + n;
    return false;
  }
  dn = yd * nx + xd;
  slot = (size_t)j * N + dn;
  return true;
}

// Transpose of an Eq. (33) stencil: calls f(j, m) for every node m and
// direction j whose stencil point m + c_j is the node (x, y), through the
// periodic wrap or the mirror ghost rows at walls.
template <typename F>
__device__ __forceinline__ void for_sources(const Inst &I, int x, int y, F &&f) {
  const int nx = I.nx, ny = I.ny;
  if (!I.bc_y || (y > 0 && y < ny - 1)) {
    // away from walls every source is a plain (wrapped) neighbour: calls
    // without conditions, whose gathers the compiler can issue together
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      int sy = y - cy(j);
      sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
      f(j, sy * nx + wrapx(x - cx(j), nx));
    }
    return;
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int sx = wrapx(x - cx(j), nx);
    int sy = y - cy(j);
    if (!I.bc_y) {
      sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
      f(j, sy * nx + sx);
    } else {
      if (sy >= 0 && sy < ny) f(j, sy * nx + sx);
      // a stencil point beyond a wall reads the first fluid row
      if ((y == 0 && cy(j) == -1) || (y == ny - 1 && cy(j) == 1)) f(j, y * nx + sx);
    }
  }
}

// Adds the block's parameter adjoints to its slot.
__device__ __forceinline__ void add_theta(const Inst &I, double *tb, int lblk, double (&v)[TB_SLOTS]) {
  block_sum<TB_SLOTS>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < TB_SLOTS; ++k) tb[(size_t)lblk * TB_SLOTS + k] += v[k];
}

// Adjoint of the collide-and-push kernel of one step.  Reads the adjoint of
// the next level (a[cur], pb[cur]); writes the adjoint of this level's
// populations and history (a[cur ^ 1]), the local phi-bar (pb[cur ^ 1]) and
// the intermediates consumed by the following adjoint kernels.
template <typename T>
__global__ __launch_bounds__(NT) void k_adj_collide(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                    Rec<T> rc, AdjBufs<T> ab, int cur) {
  const Inst *Ip;
  int lblk;
  const Node nd = locate(insts, b2i, Ip, lblk);
  if (!nd.valid) return;
  const Inst &I = *Ip;
  const Phys<T> &P = phys<T>(I);
  const int N = I.N, nx = I.nx, n = nd.n, x = nd.x, y = nd.y;
  const T *A = ab.a[cur];
  T *An = ab.a[cur ^ 1];
  const T *PBc = ab.pb[cur];
  T *PBn = ab.pb[cur ^ 1];

  // ---- forward values
  int m[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) m[j] = fdrow(y + cy(j), I.ny, I.bc_y) * nx + wrapx(x + cx(j), nx);
  T ph[3], rv[Q], sv[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const T p1 = rc.phi[m[j]], p2 = rc.phi[(size_t)N + m[j]], p3 = rc.phi[(size_t)2 * N + m[j]];
    rv[j] = P.rho[0] * p1 + P.rho[1] * p2 + P.rho[2] * p3;
    sv[j] = p1 + p2 + p3;
    if (j == 0) {
      ph[0] = p1;
      ph[1] = p2;
      ph[2] = p3;
    }
  }
  T grx, gry, dummy;
  fd9(rv, grx, gry, dummy);
  // restoring flux of the sum S = phi_1 + phi_2 + phi_3 (off: gS = 0, and
  // none of its adjoint terms below is formed)
  const bool relax = I.sum_relax != 0 && I.phase_mode == 0;
  T gSx = 0, gSy = 0;
  if (relax) fd9(sv, gSx, gSy, dummy);
  T gmx[3], gmy[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T v[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) v[j] = rc.mu[(size_t)i * N + m[j]];
    fd9(v, gmx[i], gmy[i], dummy);
  }
  const T rho = rv[0];
  const T q = rc.q[n];
  const T ex = rc.En[n], ey = rc.En[(size_t)N + n];
  T Fx = q * ex, Fy = q * ey;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Fx -= ph[i] * gmx[i];
    Fy -= ph[i] * gmy[i];
  }
  T g[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) g[j] = rc.g[(size_t)j * N + n];
  T mxg = 0, myg = 0, s1 = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    mxg += mcx(j, g[j]);
    myg += mcy(j, g[j]);
    if (j) s1 += g[j];
  }
  // the sweep multiplies by reciprocals (its values need not match the
  // forward's rounding, only its arithmetic)
  const T irho = T(1) / rho;
  const T ux = (mxg + T(0.5) * Fx) * irho, uy = (myg + T(0.5) * Fy) * irho;
  const T udr = ux * grx + uy * gry;
  const T usq = ux * ux + uy * uy;
  const T s0 = wgt<T>(0) * (-usq * T(1.5));
  const T pp = (s1 + T(0.5) * udr + rho * s0) / (T(3) * (T(1) - wgt<T>(0)));
  const T mv = P.visc[0] * ph[0] + P.visc[1] * ph[1] + P.visc[2] * ph[2];
  const T tg = T(0.5) + mv * T(3) * irho;
  const T itg = T(1) / tg, cg = T(1) - T(0.5) * itg;

  // ---- where each population was pushed: neighbour rows and columns once;
  // at a wall the slot is plane opp(j) of this node and the moving-wall
  // term -6 w_j c_jx u_wall multiplies the carrier
  const int xm = wrapx(x - 1, nx), xp = wrapx(x + 1, nx);
  int ym = y - 1, yp = y + 1;
  bool wb = false, wt = false;
  if (I.bc_y) {
    wb = ym < 0;
    wt = yp >= I.ny;
  } else {
    ym = ym < 0 ? ym + I.ny : ym;
    yp = yp >= I.ny ? yp - I.ny : yp;
  }
  auto wall = [&](int j) { return (cy(j) < 0 && wb) || (cy(j) > 0 && wt); };
  auto at = [&](const T *plane0, int j) {
    const int xx = cx(j) < 0 ? xm : (cx(j) > 0 ? xp : x);
    const int yy = cy(j) < 0 ? ym : (cy(j) > 0 ? yp : y);
    const bool w = wall(j);
    return plane0[(size_t)(w ? opp(j) : j) * N + (w ? n : yy * nx + xx)];
  };
  auto dnode = [&](int j) {
    const int xx = cx(j) < 0 ? xm : (cx(j) > 0 ? xp : x);
    const int yy = cy(j) < 0 ? ym : (cy(j) > 0 ? yp : y);
    return wall(j) ? n : yy * nx + xx;
  };
  auto wu = [&](int j) {
    return wall(j) ? -T(6) * wgt<T>(j) * T(cx(j)) * (cy(j) > 0 ? P.wall_u[1] : P.wall_u[0]) : T(0);
  };

  // ---- the pulled adjoints (and the moment adjoint they carry), loaded
  // before the first store: stores to planes the compiler cannot tell apart
  // from A would otherwise hold back every later load
  T la[Q], ga[Q], fa[3][Q], hp[3][2];
#pragma unroll
  for (int j = 0; j < Q; ++j) la[j] = at(A + (size_t)AO_L * N, j) + PBc[(size_t)3 * N + dnode(j)];
#pragma unroll
  for (int j = 0; j < Q; ++j) ga[j] = at(A + (size_t)AO_G * N, j);
  if (I.phase_mode == 0)
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < Q; ++j) fa[i][j] = at(A + (size_t)(i * Q) * N, j) + PBc[(size_t)i * N + dnode(j)];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    hp[i][0] = A[(size_t)(AO_HPU + 2 * i) * N + n];
    hp[i][1] = A[(size_t)(AO_HPU + 2 * i + 1) * N + n];
  }
  const T hqx = A[(size_t)AO_HQU * N + n], hqy = A[(size_t)(AO_HQU + 1) * N + n];

  // ---- adjoint accumulators
  T ph_b[3] = {T(0), T(0), T(0)}, mu_b[3] = {T(0), T(0), T(0)};
  T gmx_b[3] = {T(0), T(0), T(0)}, gmy_b[3] = {T(0), T(0), T(0)};
  T ux_b = 0, uy_b = 0, rho_b = 0, pp_b = 0, Fx_b = 0, Fy_b = 0, grx_b = 0, gry_b = 0;
  T q_b = 0, R_b = 0, itg_b = 0;
  // restoring flux: grad(S)-bar, and sum_i phi_i (X_i-bar . grad S)
  T gSx_b = 0, gSy_b = 0, relax_t = 0;

  // ---- charge family (Eqs. 48-50)
  {
    const T itl = T(1) / P.tau_l, cl = T(1) - T(0.5) * itl;
    const bool dir = I.wall_q_mode == 1;
    T dqx_b = 0, dqy_b = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const T a = la[j];
      const T vb = (dir && wall(j)) ? -a : a;
      if (!dir) q_b += a * wu(j);
      An[(size_t)AO_L * N + (size_t)j * N + n] = vb * (T(1) - itl);
      const T cu = mcx(j, ux) + mcy(j, uy);
      const T wv = vb * itl * wgt<T>(j);
      q_b += wv * (T(1) + T(3) * cu);
      ux_b += mcx(j, wv * q * T(3));
      uy_b += mcy(j, wv * q * T(3));
      R_b += vb * cl * wgt<T>(j);
      dqx_b += mcx(j, vb * cl * wgt<T>(j) * T(3));
      dqy_b += mcy(j, vb * cl * wgt<T>(j) * T(3));
    }
    // dq = q u - (q u)_prev; (q u) is also this step's history output
    const T hx = hqx, hy = hqy;
    q_b += (dqx_b + hx) * ux + (dqy_b + hy) * uy;
    ux_b += q * (dqx_b + hx);
    uy_b += q * (dqy_b + hy);
    An[(size_t)AO_HQU * N + n] = -dqx_b;
    An[(size_t)(AO_HQU + 1) * N + n] = -dqy_b;
  }

  // ---- flow family (Eqs. 37-40), local tau_g
  T g_b[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const T vb = ga[j];
    rho_b += vb * wu(j);
    const T cu = mcx(j, ux) + mcy(j, uy);
    const T sj = wgt<T>(j) * (cu * T(3) + cu * cu * T(4.5) - usq * T(1.5));
    const T geq = (j == 0 ? (wgt<T>(0) - T(1)) * pp * T(3) : wgt<T>(j) * pp * T(3)) + rho * sj;
    const T cF = mcx(j, Fx) + mcy(j, Fy);
    const T cgr = mcx(j, grx) + mcy(j, gry);
    const T Gb = wgt<T>(j) * (udr + cF * T(3) + (cu * cgr - udr / T(3)) * T(3));
    g_b[j] = vb * (T(1) - itg);
    itg_b += vb * (-(g[j] - geq) - T(0.5) * Gb);
    pp_b += vb * itg * (j == 0 ? T(3) * (wgt<T>(0) - T(1)) : T(3) * wgt<T>(j));
    rho_b += vb * itg * sj;
    const T ws = vb * itg * rho * wgt<T>(j);
    ux_b += ws * (mcx(j, T(3) + T(9) * cu) - T(3) * ux);
    uy_b += ws * (mcy(j, T(3) + T(9) * cu) - T(3) * uy);
    const T Gb_b = vb * cg * T(3) * wgt<T>(j);
    Fx_b += mcx(j, Gb_b);
    Fy_b += mcy(j, Gb_b);
    ux_b += mcx(j, Gb_b * cgr);
    uy_b += mcy(j, Gb_b * cgr);
    grx_b += mcx(j, Gb_b * cu);
    gry_b += mcy(j, Gb_b * cu);
  }
  {
    const T tg_b = -itg_b * itg * itg;
    const T mv_b = tg_b * T(3) * irho;
    rho_b -= tg_b * T(3) * mv * irho * irho;
#pragma unroll
    for (int i = 0; i < 3; ++i) ph_b[i] += P.visc[i] * mv_b;
  }

  // ---- order-parameter families (Eqs. 34-36) and their history
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T hx = hp[i][0], hy = hp[i][1];
    T dpx_b = 0, dpy_b = 0;
    if (I.phase_mode == 0) {
      const T m0 = P.m0, itf = T(1) / P.tau_f, cf = T(1) - T(0.5) * itf, im0 = T(1) / P.m0;
      T dtx_b = 0, dty_b = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const T vb = fa[i][j];
        ph_b[i] += vb * wu(j);
        An[(size_t)(i * Q + j) * N + n] = vb * (T(1) - itf);
        if (j == 0) {
          ph_b[i] += vb * itf;
          mu_b[i] -= vb * itf * (T(1) - wgt<T>(0));
        } else {
          const T wv = vb * itf * wgt<T>(j);
          ph_b[i] += wv * T(3) * (mcx(j, ux) + mcy(j, uy));
          ux_b += mcx(j, wv * T(3) * ph[i]);
          uy_b += mcy(j, wv * T(3) * ph[i]);
          mu_b[i] += wv;
        }
        dtx_b += mcx(j, cf * vb * wgt<T>(j));
        dty_b += mcy(j, cf * vb * wgt<T>(j));
      }
      dpx_b = T(3) * dtx_b;
      dpy_b = T(3) * dty_b;
      // X_i = sum_{k != i} M_ik grad mu_k + (M_ii - m0) grad mu_i (Eq. 28)
      const T Xx_b = -dtx_b * im0, Xy_b = -dty_b * im0;
      T mii = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k != i) mii += m0 * ph[i] * ph[k];
      const T si = Xx_b * gmx[i] + Xy_b * gmy[i];
      gmx_b[i] += (mii - m0) * Xx_b;
      gmy_b[i] += (mii - m0) * Xy_b;
#pragma unroll
      for (int k = 0; k < 3; ++k)
        if (k != i) {
          const T sk = Xx_b * gmx[k] + Xy_b * gmy[k];
          gmx_b[k] -= m0 * ph[i] * ph[k] * Xx_b;
          gmy_b[k] -= m0 * ph[i] * ph[k] * Xy_b;
          ph_b[i] += m0 * ph[k] * (si - sk);
          ph_b[k] += m0 * ph[i] * (si - sk);
        }
      if (relax) {
        // + (m0 / S) phi_i grad S: phi_i directly, S through m0 / S, and
        // grad S, whose stencil the chemical-potential adjoint transposes
        const T wsum = m0 / sv[0];
        const T ti = Xx_b * gSx + Xy_b * gSy;
        ph_b[i] += wsum * ti;
        relax_t += ph[i] * ti;
        gSx_b += wsum * ph[i] * Xx_b;
        gSy_b += wsum * ph[i] * Xy_b;
      }
    } else {
#pragma unroll
      for (int j = 0; j < Q; ++j) An[(size_t)(i * Q + j) * N + n] = T(0);
    }
    // dp = phi_i u - (phi_i u)_prev; (phi_i u) is also the history output
    ph_b[i] += (dpx_b + hx) * ux + (dpy_b + hy) * uy;
    ux_b += ph[i] * (dpx_b + hx);
    uy_b += ph[i] * (dpy_b + hy);
    An[(size_t)(AO_HPU + 2 * i) * N + n] = -dpx_b;
    An[(size_t)(AO_HPU + 2 * i + 1) * N + n] = -dpy_b;
  }

  // ---- flow moments (Eq. 41)
  {
    const T c3 = T(1) / (T(3) * (T(1) - wgt<T>(0)));
    const T s1_b = pp_b * c3, udr_b = T(0.5) * pp_b * c3;
    rho_b += s0 * pp_b * c3;
    const T usq_b = rho * pp_b * c3 * wgt<T>(0) * T(-1.5);
    ux_b += T(2) * ux * usq_b + udr_b * grx;
    uy_b += T(2) * uy * usq_b + udr_b * gry;
    grx_b += udr_b * ux;
    gry_b += udr_b * uy;
    const T mx_b = ux_b * irho, my_b = uy_b * irho;
    Fx_b += T(0.5) * mx_b;
    Fy_b += T(0.5) * my_b;
    rho_b -= (ux_b * ux + uy_b * uy) * irho;
#pragma unroll
    for (int j = 0; j < Q; ++j)
      An[(size_t)(AO_G + j) * N + n] = g_b[j] + mcx(j, mx_b) + mcy(j, my_b) + (j ? s1_b : T(-0.0));
  }

  // ---- force -sum phi_i grad mu_i + q E (Eq. 27b) and rho of Eq. (29)
  q_b += Fx_b * ex + Fy_b * ey;
  // d(m0 / S) / dS = -(m0 / S) / S reaches every phase alike
  const T S_b = relax ? -(P.m0 / sv[0]) / sv[0] * relax_t : T(0);
  if (relax) {
    ab.gS[n] = gSx_b;
    ab.gS[(size_t)N + n] = gSy_b;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    ph_b[i] += S_b;
    ph_b[i] -= Fx_b * gmx[i] + Fy_b * gmy[i] - P.rho[i] * rho_b;
    gmx_b[i] -= ph[i] * Fx_b;
    gmy_b[i] -= ph[i] * Fy_b;
    PBn[(size_t)i * N + n] = ph_b[i];
    ab.muL[(size_t)i * N + n] = mu_b[i];
    ab.gm[(size_t)(2 * i) * N + n] = gmx_b[i];
    ab.gm[(size_t)(2 * i + 1) * N + n] = gmy_b[i];
  }
  ab.gr[n] = grx_b;
  ab.gr[(size_t)N + n] = gry_b;
  ab.qb[n] = q_b;
  ab.rb[n] = R_b;
  ab.en[n] = q * Fx_b;
  ab.en[(size_t)N + n] = q * Fy_b;
}

// Adjoint of the chemical-potential kernel (Eq. 20 and the field of
// Eq. 45).  with_step: the collide adjoint ran (its grad-mu-bar,
// grad-rho-bar and field-bar are added); at create only the local mu-bar
// and the state's field-bar are there.  Adds grad(h)-terms to hb[hsel] in
// place and starts eps-bar.
template <typename T>
__global__ __launch_bounds__(NT) void k_adj_mu(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                               Rec<T> rc, AdjBufs<T> ab, int cur, int hsel, int with_step) {
  const Inst *Ip;
  int lblk;
  const Node nd = locate(insts, b2i, Ip, lblk);
  const Inst &I = *Ip;
  double th[TB_SLOTS] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (nd.valid) {
    const Phys<T> &P = phys<T>(I);
    const int N = I.N, n = nd.n;
    T mu_b[3], ph_b[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int i = 0; i < 3; ++i) mu_b[i] = ab.muL[(size_t)i * N + n];
    T ex_b = ab.a[cur][(size_t)AO_E * N + n], ey_b = ab.a[cur][(size_t)(AO_E + 1) * N + n];
    // the accumulators this node adds to, read now (distinct buffers from
    // every plane the kernel writes first; a read after a store would wait
    // for it)
    T *hb = ab.hb[hsel];
    T *PBn = ab.pb[cur ^ 1];
    T hb0[Q], pb0[3];
#pragma unroll
    for (int j = 1; j < Q; ++j) hb0[j] = hb[(size_t)j * N + n];
#pragma unroll
    for (int i = 0; i < 3; ++i) pb0[i] = PBn[(size_t)i * N + n];
    if (with_step) {
      T gr_t = 0, gS_t = 0;
      for_sources(I, nd.x, nd.y, [&](int j, int s) {
        const T w3 = T(3) * wgt<T>(j);
#pragma unroll
        for (int i = 0; i < 3; ++i)
          mu_b[i] += w3 * (mcx(j, ab.gm[(size_t)(2 * i) * N + s]) + mcy(j, ab.gm[(size_t)(2 * i + 1) * N + s]));
        gr_t += w3 * (mcx(j, ab.gr[s]) + mcy(j, ab.gr[(size_t)N + s]));
      });
      // grad S of the restoring flux: S reaches every phase with weight one
      if (I.sum_relax != 0 && I.phase_mode == 0)
        for_sources(I, nd.x, nd.y, [&](int j, int s) {
          gS_t += T(3) * wgt<T>(j) * (mcx(j, ab.gS[s]) + mcy(j, ab.gS[(size_t)N + s]));
        });
#pragma unroll
      for (int i = 0; i < 3; ++i) ph_b[i] += P.rho[i] * gr_t + gS_t;
      ex_b += ab.en[n];
      ey_b += ab.en[(size_t)N + n];
    }
    const T Ex = rc.En[n], Ey = rc.En[(size_t)N + n];
    const T e2 = Ex * Ex + Ey * Ey;
    T e2_b = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T ph = rc.phi[(size_t)i * N + n];
      ph_b[i] += mu_b[i] * T(24) / P.D * P.lam[i] * (T(3) * ph * ph - T(3) * ph + T(0.5));
      ab.lb[(size_t)i * N + n] = -mu_b[i] * T(0.75) * P.D * P.lam[i];
      ph_b[i] -= mu_b[i] * T(3) * P.eps[i] * (T(1) - T(2) * ph) * e2;
      e2_b -= mu_b[i] * T(3) * P.eps[i] * ph * (T(1) - ph);
      th[i] -= (double)(mu_b[i] * T(3) * ph * (T(1) - ph) * e2);
    }
    ex_b += T(2) * Ex * e2_b;
    ey_b += T(2) * Ey * e2_b;
    // E = (m + (tau_h/3) E_ext) / den with m the first moment of the final h
    const T th3 = P.tau_h / T(3), iden = T(1) / ((rc.eps[n] - P.eps_ref) + th3);
    const T mx_b = ex_b * iden, my_b = ey_b * iden;
    th[6] += ((double)mx_b * ab.dEext[0] + (double)my_b * ab.dEext[1]) * (double)th3;
    ab.eb[n] = -(ex_b * Ex + ey_b * Ey) * iden;
#pragma unroll
    for (int j = 1; j < Q; ++j) hb[(size_t)j * N + n] = hb0[j] + (mcx(j, mx_b) + mcy(j, my_b));
#pragma unroll
    for (int i = 0; i < 3; ++i) PBn[(size_t)i * N + n] = pb0[i] + ph_b[i];
  }
  add_theta(I, ab.tb, lblk, th);
}

// Local part of the adjoint of one potential sub-iteration at a node: vb
// is the adjoint of the node's post-collision populations (already pulled
// through the push), h its forward input; returns the adjoint of h and adds
// to eps_hat-bar, q-bar and the applied field's adjoint ee_b (which enters
// through grad(psi) = -(m + (tau_h/3) E_ext) iden).
//   iden: 1 / (eps_hat + tau_h / 3), as the forward collision forms it.
// Constants of the potential collision's adjoint: 1/tau_h and tau_h/3.
template <typename T> struct AdjPotK {
  T ith, tau3;
};
template <typename T> __device__ __forceinline__ AdjPotK<T> adj_pot_k(const Phys<T> &P) {
  AdjPotK<T> k;
  k.ith = T(1) / P.tau_h;
  k.tau3 = P.tau_h / T(3);
  return k;
}
// Terms with a zero lattice coefficient are left out (they are exact zeros).
template <typename T>
__device__ __forceinline__ void adj_poisson_local(const T (&vb)[Q], const T (&h)[Q], T eh, T iden, const Phys<T> &P,
                                                  const AdjPotK<T> &K, T (&hb)[Q], T &eh_b, T &q_b, T (&ee_b)[2]) {
  T mx = K.tau3 * P.Eext[0], my = K.tau3 * P.Eext[1];
#pragma unroll
  for (int j = 1; j < Q; ++j) {
    if (cx(j)) mx += T(cx(j)) * h[j];
    if (cy(j)) my += T(cy(j)) * h[j];
  }
  const T gx = -mx * iden, gy = -my * iden;
  const T ith = K.ith;
  T pot_b = 0, gx_b = 0, gy_b = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    pot_b += vb[j] * ith * (j == 0 ? wgt<T>(0) - T(1) : wgt<T>(j));
    if (j == 0) continue;
    const T c3 = vb[j] * T(3) * wgt<T>(j) * ith;
    if (cx(j)) gx_b -= c3 * eh * T(cx(j));
    if (cy(j)) gy_b -= c3 * eh * T(cy(j));
    const T cg = cx(j) && cy(j) ? T(cx(j)) * gx + T(cy(j)) * gy : (cx(j) ? T(cx(j)) * gx : T(cy(j)) * gy);
    eh_b -= c3 * cg;
    q_b += T(0.125) * vb[j];
  }
  // g = -M iden, M = m + (tau_h/3) E_ext, iden = 1 / (eps_hat + tau_h / 3):
  // dg/d eps_hat = M iden^2
  const T mx_b = -gx_b * iden, my_b = -gy_b * iden;
  eh_b += (gx_b * mx + gy_b * my) * (iden * iden);
  ee_b[0] += mx_b * K.tau3;
  ee_b[1] += my_b * K.tau3;
  const T ps_b = pot_b * (T(1) / (T(1) - wgt<T>(0)));
  hb[0] = vb[0] * (T(1) - ith);
#pragma unroll
  for (int j = 1; j < Q; ++j) {
    T a = vb[j] * (T(1) - ith);
    if (cx(j)) a += T(cx(j)) * mx_b;
    if (cy(j)) a += T(cy(j)) * my_b;
    hb[j] = a + ps_b;
  }
}
template <typename T>
__device__ __forceinline__ void adj_poisson_local(const T (&vb)[Q], const T (&h)[Q], T eh, T iden, const Phys<T> &P,
                                                  T (&hb)[Q], T &eh_b, T &q_b, T (&ee_b)[2]) {
  adj_poisson_local(vb, h, eh, iden, P, adj_pot_k(P), hb, eh_b, q_b, ee_b);
}
template <typename T>
__device__ __forceinline__ void adj_poisson_local(const T (&vb)[Q], const T (&h)[Q], T eh, const Phys<T> &P,
                                                  T (&hb)[Q], T &eh_b, T &q_b, T (&ee_b)[2]) {
  adj_poisson_local(vb, h, eh, poisson_iden(eh, P), P, hb, eh_b, q_b, ee_b);
}
// Whether an instance has an applied field (its sub-iterations then carry a
// d/d E0 term at every node, not only at the electrodes).
template <typename T> __device__ __forceinline__ bool has_eext(const Phys<T> &P) {
  return P.Eext[0] != T(0) || P.Eext[1] != T(0);
}

// Adjoint of one potential sub-iteration (Eqs. 43-45 with anti-bounce-back
// electrodes): hb[src] holds the adjoint of the output level, h_in the
// forward input level; writes the adjoint of the input level to hb[src ^ 1]
// and adds to eps-bar and q-bar (qb may alias a scratch plane).
template <typename T>
__global__ __launch_bounds__(NT) void k_adj_poisson(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                    const T *__restrict__ h_in, const T *__restrict__ eps,
                                                    AdjBufs<T> ab, int src, T *qb) {
  const Inst *Ip;
  int lblk;
  const Node nd = locate(insts, b2i, Ip, lblk);
  const Inst &I = *Ip;
  double th[TB_SLOTS] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (nd.valid) {
    const Phys<T> &P = phys<T>(I);
    const int N = I.N, n = nd.n;
    const T *Hs = ab.hb[src];
    T vb[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      size_t slot;
      int dn;
      bool top;
      const bool in = push_slot(I, nd.x, nd.y, n, j, slot, dn, top);
      const T a = Hs[slot];
      if (in) {
        vb[j] = a;
      } else {
        vb[j] = -a;
        th[6] += 2.0 * (double)(wgt<T>(j) * a) * ab.dwall[top ? 1 : 0];
      }
    }
    T h[Q], hb[Q], eh_b = 0, q_b = 0, ee_b[2] = {T(0), T(0)};
#pragma unroll
    for (int j = 0; j < Q; ++j) h[j] = h_in[(size_t)j * N + n];
    adj_poisson_local(vb, h, eps[n] - P.eps_ref, P, hb, eh_b, q_b, ee_b);
    th[6] += (double)ee_b[0] * ab.dEext[0] + (double)ee_b[1] * ab.dEext[1];
    T *Hd = ab.hb[src ^ 1];
#pragma unroll
    for (int j = 0; j < Q; ++j) Hd[(size_t)j * N + n] = hb[j];
    ab.eb[n] += eh_b;
    qb[n] += q_b;
  }
  // only blocks holding a wall row carry a d/d E0 term (uniform per block),
  // or every block under an applied field
  if (has_eext(phys<T>(I)) || (I.bc_y && (lblk * NT < I.nx || (lblk + 1) * NT > (I.ny - 1) * I.nx)))
    add_theta(I, ab.tb, lblk, th);
}

// Adjoints of two potential sub-iterations in one launch, the transpose of
// k_poisson2: a block owns the same tiles, loads the adjoint of the output
// level for the extended tile into LDS, pulls and transforms it on the ring
// of width 1 (forward input level h1 there), writes that level back to LDS,
// pulls and transforms it on the interior (input level h0) and writes the
// adjoint of h0 to hb[src ^ 1].  eps-bar and q-bar of both iterations are
// added on the interior; wall tiles add their d/d E0 terms to slot
// blockIdx.x of tb.
template <typename T>
__global__ __launch_bounds__(P2NT) void k_adj_poisson2(const Inst *__restrict__ insts, const int4 *__restrict__ tiles,
                                                      const T *__restrict__ h1, const T *__restrict__ h0,
                                                      const T *__restrict__ eps, AdjBufs<T> ab, int src, T *qb) {
  __shared__ T buf[Q * P2EW * P2ER];
  __shared__ double red[P2NT / 64];
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  const Phys<T> &P = phys<T>(I);
  const int nx = I.nx, ny = I.ny, N = I.N, walls = I.bc_y;
  // one extended node per thread (P2RPT == 1); a wave covers one row
  const int tx = threadIdx.x & 63, r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gx = wrapx(((t.y - 2 + tx) % nx + nx) % nx, nx);
  int gy = t.z - 2 + r;
  bool inside = true;
  if (walls) inside = gy >= 0 && gy < ny;
  else gy = ((gy % ny) + ny) % ny;
  const int n = gy * nx + gx;
  const int e = r * P2EW + tx;
  const T *Hs = ab.hb[src];
  const bool ring1 = inside && r >= 1 && r < P2ER - 1 && tx >= 1 && tx < P2EW - 1;
  const bool interior = inside && r >= 2 && r < 2 + P2H && tx >= 2 && tx < 2 + P2W && t.y + tx - 2 < nx &&
                        t.z + r - 2 < ny;
  // the adjoint level, and the first iteration's forward level and eps
  // where they are used, in one burst of loads ahead of the first barrier
  T hv[Q], h1v[Q], epsv = T(0);
#pragma unroll
  for (int j = 0; j < Q; ++j) hv[j] = h1v[j] = T(0);
  if (inside)
#pragma unroll
    for (int j = 0; j < Q; ++j) hv[j] = Hs[(size_t)j * N + n];
  if (ring1) {
#pragma unroll
    for (int j = 0; j < Q; ++j) h1v[j] = h1[(size_t)j * N + n];
    epsv = eps[n];
  }
#pragma unroll
  for (int j = 0; j < Q; ++j) buf[j * (P2EW * P2ER) + e] = hv[j];
  __syncthreads();
  double th = 0.0;
  T eh_b = 0, q_b = 0, ee_b[2] = {T(0), T(0)};
  const T eh = ring1 ? epsv - P.eps_ref : T(0);
  const T iden = poisson_iden(eh, P);
  const AdjPotK<T> pk = adj_pot_k(P);
  const bool wall_row = walls && (gy == 0 || gy == ny - 1);
  // pull of the adjoint through the push of node (r, tx); wall slots at the
  // node itself (rows next to an electrode only)
  auto pull = [&](T (&vb)[Q]) {
    if (wall_row) {
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const int yd = gy + cy(j);
        if (yd < 0 || yd >= ny) {
          const T a = buf[opp(j) * (P2EW * P2ER) + e];
          vb[j] = -a;
          if (interior) th += 2.0 * (double)(wgt<T>(j) * a) * ab.dwall[yd >= ny ? 1 : 0];
        } else {
          vb[j] = buf[j * (P2EW * P2ER) + e + cy(j) * P2EW + cx(j)];
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < Q; ++j) vb[j] = buf[j * (P2EW * P2ER) + e + cy(j) * P2EW + cx(j)];
    }
  };
  T hb[Q];
  if (ring1) {
    T vb[Q];
    pull(vb);
    T eb1 = 0, qb1 = 0, ee1[2] = {T(0), T(0)};
    adj_poisson_local(vb, h1v, eh, iden, P, pk, hb, eb1, qb1, ee1);
    if (interior) {
      eh_b += eb1;
      q_b += qb1;
      ee_b[0] += ee1[0];
      ee_b[1] += ee1[1];
    }
  }
  __syncthreads();
  if (ring1)
#pragma unroll
    for (int j = 0; j < Q; ++j) buf[j * (P2EW * P2ER) + e] = hb[j];
  __syncthreads();
  if (interior) {
    T vb[Q], h[Q];
    pull(vb);
#pragma unroll
    for (int j = 0; j < Q; ++j) h[j] = h0[(size_t)j * N + n];
    adj_poisson_local(vb, h, eh, iden, P, pk, hb, eh_b, q_b, ee_b);
    T *Hd = ab.hb[src ^ 1];
#pragma unroll
    for (int j = 0; j < Q; ++j) Hd[(size_t)j * N + n] = hb[j];
    ab.eb[n] += eh_b;
    qb[n] += q_b;
    th += (double)ee_b[0] * ab.dEext[0] + (double)ee_b[1] * ab.dEext[1];
  }
  if (has_eext(P) || (walls && (t.z == 0 || t.z + P2H >= ny))) {
    for (int o = 32; o > 0; o >>= 1) th += __shfl_down(th, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = th;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0;
      for (int w = 0; w < P2NT / 64; ++w) s += red[w];
      ab.tb[(size_t)blockIdx.x * TB_SLOTS + 6] += s;
    }
  }
}

// Adjoints of four potential sub-iterations in one launch, the transpose of
// the four-iteration k_poisson2 on 64 x 32 tiles (two extended rows per
// thread): the adjoint of the output level is loaded for the extended tile
// into LDS; sub-iterations 4, 3, 2, 1 are reversed in turn on the nodes at
// least 1, 2, 3, 4 nodes inside the tile (their push targets hold the
// adjoint of the next level there), each with its forward input level
// lv[3], lv[2], lv[1], lv[0], writing the level's adjoint back to LDS.  The
// interior's adjoint of the input level goes to hb[src ^ 1] and its eps-bar
// and q-bar of all four sub-iterations are added; wall tiles add their
// d/d E0 terms to slot blockIdx.x of tb.
template <typename T>
__global__ __launch_bounds__(P2NT) void k_adj_poisson4(const Inst *__restrict__ insts, const int4 *__restrict__ tiles,
                                                      const T *__restrict__ lv0, const T *__restrict__ lv1,
                                                      const T *__restrict__ lv2, const T *__restrict__ lv3,
                                                      const T *__restrict__ eps, AdjBufs<T> ab, int src, T *qb) {
  constexpr int RPT = 2, IT = 4, ER = P2Shape<RPT, IT>::ER, H4 = P2Shape<RPT, IT>::H, W4 = P2Shape<RPT, IT>::W;
  constexpr int PL = P2EW * ER;  // LDS plane
  __shared__ T buf[Q * PL];
  __shared__ double red[P2NT / 64];
  const int4 t = tiles[blockIdx.x];
  const Inst &I = insts[t.x];
  const Phys<T> &P = phys<T>(I);
  const int nx = I.nx, ny = I.ny, N = I.N, walls = I.bc_y;
  // a 64-lane wave covers one row of the tile: row tests are uniform branches
  const int tx = threadIdx.x & 63, ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gx = wrapx(((t.y - IT + tx) % nx + nx) % nx, nx);
  int gy[RPT], n[RPT], e[RPT], dist[RPT];
  bool inside[RPT], interior[RPT], wall_row[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = ty + (P2NT / 64) * k;
    int y = t.z - IT + r;
    bool in = true;
    if (walls) in = y >= 0 && y < ny;
    else y = ((y % ny) + ny) % ny;
    gy[k] = y;
    inside[k] = in;
    n[k] = y * nx + gx;
    e[k] = r * P2EW + tx;
    const int dr = r < ER - 1 - r ? r : ER - 1 - r, dc = tx < P2EW - 1 - tx ? tx : P2EW - 1 - tx;
    dist[k] = dr < dc ? dr : dc;  // 0 on the tile's outermost ring
    interior[k] = in && dist[k] >= IT && r - IT < H4 && tx - IT < W4 && t.y + tx - IT < nx && t.z + r - IT < ny;
    wall_row[k] = walls && (y == 0 || y == ny - 1);
  }
  // the adjoint of the output level and eps, in one burst of loads
  const T *Hs = ab.hb[src];
  T hv[RPT][Q], epsv[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
#pragma unroll
    for (int j = 0; j < Q; ++j) hv[k][j] = inside[k] ? Hs[(size_t)j * N + n[k]] : T(0);
    epsv[k] = inside[k] && dist[k] >= 1 ? eps[n[k]] : T(0);
  }
#pragma unroll
  for (int k = 0; k < RPT; ++k)
#pragma unroll
    for (int j = 0; j < Q; ++j) buf[j * PL + e[k]] = hv[k][j];
  __syncthreads();
  double th = 0.0;
  T eh[RPT], iden[RPT], eh_b[RPT], q_b[RPT], ee_b[2] = {T(0), T(0)};
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    eh[k] = inside[k] && dist[k] >= 1 ? epsv[k] - P.eps_ref : T(0);
    iden[k] = poisson_iden(eh[k], P);
    eh_b[k] = q_b[k] = T(0);
  }
  const T *lvs[IT] = {lv0, lv1, lv2, lv3};
  const AdjPotK<T> pk = adj_pot_k(P);
  T hb[RPT][Q];
#pragma unroll 1
  for (int i = IT; i >= 1; --i) {
    const int need = IT - i + 1;  // nodes this reversal reaches: at least `need` inside the tile
    const T *lv = lvs[i - 1];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      if (!inside[k] || dist[k] < need) continue;
      T vb[Q], h[Q];
      // pull of the adjoint through the push of this node; wall slots at the
      // node itself (rows next to an electrode only)
      if (wall_row[k]) {
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          const int yd = gy[k] + cy(j);
          if (yd < 0 || yd >= ny) {
            const T a = buf[opp(j) * PL + e[k]];
            vb[j] = -a;
            if (interior[k]) th += 2.0 * (double)(wgt<T>(j) * a) * ab.dwall[yd >= ny ? 1 : 0];
          } else {
            vb[j] = buf[j * PL + e[k] + cy(j) * P2EW + cx(j)];
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < Q; ++j) vb[j] = buf[j * PL + e[k] + cy(j) * P2EW + cx(j)];
      }
#pragma unroll
      for (int j = 0; j < Q; ++j) h[j] = lv[(size_t)j * N + n[k]];
      T eb1 = 0, qb1 = 0, ee1[2] = {T(0), T(0)};
      adj_poisson_local(vb, h, eh[k], iden[k], P, pk, hb[k], eb1, qb1, ee1);
      if (interior[k]) {
        eh_b[k] += eb1;
        q_b[k] += qb1;
        ee_b[0] += ee1[0];
        ee_b[1] += ee1[1];
      }
    }
    if (i > 1) {
      __syncthreads();
#pragma unroll
      for (int k = 0; k < RPT; ++k)
        if (inside[k] && dist[k] >= need)
#pragma unroll
          for (int j = 0; j < Q; ++j) buf[j * PL + e[k]] = hb[k][j];
      __syncthreads();
    }
  }
  T *Hd = ab.hb[src ^ 1];
#pragma unroll
  for (int k = 0; k < RPT; ++k)
    if (interior[k]) {
#pragma unroll
      for (int j = 0; j < Q; ++j) Hd[(size_t)j * N + n[k]] = hb[k][j];
      ab.eb[n[k]] += eh_b[k];
      qb[n[k]] += q_b[k];
    }
  th += (double)ee_b[0] * ab.dEext[0] + (double)ee_b[1] * ab.dEext[1];
  if (has_eext(P) || (walls && (t.z == 0 || t.z + H4 >= ny))) {
    for (int o = 32; o > 0; o >>= 1) th += __shfl_down(th, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = th;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0;
      for (int w = 0; w < P2NT / 64; ++w) s += red[w];
      ab.tb[(size_t)blockIdx.x * TB_SLOTS + 6] += s;
    }
  }
}

// Adjoint-bar of the Ohmic source of Eq. (47) at node s (R' = (sigma/eps)
// grad(eps).E - grad(sigma).E with the previous step's field): a function of
// values at s alone (phi, the previous field, R-bar and q-bar there), so the
// last kernel of a step's adjoint forms it at every source of its
// transposed gradient stencils instead of reading it from a plane.
//   se: sigma / eps at s (Eq. 30 and the conductivity of Eq. 29).
template <typename T> __device__ __forceinline__ T pre_rp_from(T se, T R_b, T qb) {
  return R_b + T(0.5) * ((qb - se * R_b) / (T(1) + T(0.5) * se));
}
template <typename T>
__device__ __forceinline__ T pre_rp_bar(const Phys<T> &P, T p1, T p2, T p3, T R_b, T qb, T &se) {
  se = (P.sig[0] * p1 + P.sig[1] * p2 + P.sig[2] * p3) / (P.eps[0] * herm(p1) + P.eps[1] * herm(p2) + P.eps[2] * herm(p3));
  return pre_rp_from(se, R_b, qb);
}

// Last kernel of a step's adjoint: charge recovery (Eq. 47 with the
// previous step's field) and the permittivity and conductivity fields.
// Gathers the Laplacian-bar of the mu adjoint, and transposes the eps and
// sigma gradient stencils of Eq. (47) onto phi-bar (their gradient-bars
// recomputed at each source node).  Writes phi-bar, the lsum-bar and the
// previous field's adjoint (state).
template <typename T>
__global__ __launch_bounds__(NT) void k_adj_pre(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                Rec<T> rc, AdjBufs<T> ab, int cur) {
  const Inst *Ip;
  int lblk;
  const Node nd = locate(insts, b2i, Ip, lblk);
  const Inst &I = *Ip;
  double th[TB_SLOTS] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (nd.valid) {
    const Phys<T> &P = phys<T>(I);
    const int N = I.N, nx = I.nx, n = nd.n;
    // the accumulator this node adds to, read before any store
    T *PBn = ab.pb[cur ^ 1];
    T pb0[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) pb0[i] = PBn[(size_t)i * N + n];
    T ph_b[3] = {T(0), T(0), T(0)};
    // transpose of the Laplacian in mu: 6 sum_j w_j v(m + c_j) - 6 v(m)
    for_sources(I, nd.x, nd.y, [&](int j, int s) {
#pragma unroll
      for (int i = 0; i < 3; ++i) ph_b[i] += T(6) * wgt<T>(j) * ab.lb[(size_t)i * N + s];
    });
#pragma unroll
    for (int i = 0; i < 3; ++i) ph_b[i] -= T(6) * ab.lb[(size_t)i * N + n];
    // forward values
    T ev[Q], sv[Q], ph[3];
    int mm[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int m = fdrow(nd.y + cy(j), I.ny, I.bc_y) * nx + wrapx(nd.x + cx(j), nx);
      mm[j] = m;
      const T p1 = rc.phi[m], p2 = rc.phi[(size_t)N + m], p3 = rc.phi[(size_t)2 * N + m];
      ev[j] = P.eps[0] * herm(p1) + P.eps[1] * herm(p2) + P.eps[2] * herm(p3);
      sv[j] = P.sig[0] * p1 + P.sig[1] * p2 + P.sig[2] * p3;
      if (j == 0) {
        ph[0] = p1;
        ph[1] = p2;
        ph[2] = p3;
      }
    }
    T gex, gey, gsx, gsy, dummy;
    fd9(ev, gex, gey, dummy);
    fd9(sv, gsx, gsy, dummy);
    const T ex = rc.Eo[n], ey = rc.Eo[(size_t)N + n];
    const T q = rc.q[n];
    // adjoints
    const T R_b = ab.rb[n], qb = ab.qb[n];
    T se;
    const T Rp_b = pre_rp_bar(P, ph[0], ph[1], ph[2], R_b, qb, se);
    const T B = T(1) + T(0.5) * se;
    const T q_b = qb - se * R_b;
    const T A_b = q_b / B, B_b = -q_b * q / B;
    const T Ls_b = A_b;
    T se_b = -q * R_b + T(0.5) * B_b;
    se_b += Rp_b * (gex * ex + gey * ey);
    const T ex_b = Rp_b * (se * gex - gsx), ey_b = Rp_b * (se * gey - gsy);
    const T sv_b = se_b / ev[0];
    const T ev_b = -se_b * se / ev[0] + ab.eb[n];
    // transposed gradients of eps and sigma: the sources' grad-bars,
    // (Rp-bar se E) for eps and (-Rp-bar E) for sigma
    T te = 0, ts = 0;
    auto source = [&](int j, int s, T ses) {
      const T rp = pre_rp_from(ses, ab.rb[s], ab.qb[s]);
      const T w3 = T(3) * wgt<T>(j);
      const T exs = rp * rc.Eo[s], eys = rp * rc.Eo[(size_t)N + s];
      te += w3 * (mcx(j, ses * exs) + mcy(j, ses * eys));
      ts -= w3 * (mcx(j, exs) + mcy(j, eys));
    };
    if (!I.bc_y || (nd.y > 0 && nd.y < I.ny - 1)) {
      // away from the wall rows the source x - c_j is the stencil point
      // x + c_opp(j) above, whose eps and sigma are at hand (the order and
      // the arithmetic of the general form below)
#pragma unroll
      for (int j = 0; j < Q; ++j) source(j, mm[opp(j)], sv[opp(j)] / ev[opp(j)]);
    } else {
      for_sources(I, nd.x, nd.y, [&](int j, int s) {
        T ses;
        pre_rp_bar(P, rc.phi[s], rc.phi[(size_t)N + s], rc.phi[(size_t)2 * N + s], T(0), T(0), ses);
        source(j, s, ses);
      });
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const T e_b = ev_b + te, s_b = sv_b + ts;
      ph_b[i] += e_b * P.eps[i] * T(6) * ph[i] * (T(1) - ph[i]) + s_b * P.sig[i];
      th[i] += (double)(e_b * herm(ph[i]));
      th[3 + i] += (double)(s_b * ph[i]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) PBn[(size_t)i * N + n] = pb0[i] + ph_b[i];
    PBn[(size_t)3 * N + n] = Ls_b;
    T *An = ab.a[cur ^ 1];
    An[(size_t)AO_E * N + n] = ex_b;
    An[(size_t)(AO_E + 1) * N + n] = ey_b;
  }
  add_theta(I, ab.tb, lblk, th);
}

// Seed of the sweep: phi-bar of the last step's moments from the FP64
// seed planes (plane k belongs to phase sel[k]).
template <typename T>
__global__ __launch_bounds__(NT) void k_adj_seed(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                 const double *__restrict__ seed, int3 sel, int count, T *pb) {
  const Inst *Ip;
  int lblk;
  const Node nd = locate(insts, b2i, Ip, lblk);
  if (!nd.valid) return;
  const int N = Ip->N, n = nd.n;
  const int s[3] = {sel.x, sel.y, sel.z};
  // seed planes are dense ([count][nn]); pb has the state's plane stride
  for (int k = 0; k < count; ++k) pb[(size_t)s[k] * N + n] += (T)seed[(size_t)k * Ip->nn + n];
}

// Create-time populations are the equilibria of the initial fields (Eq. 35):
// their adjoint reaches mu only.  The state's f-bar is the stored part plus
// the moments part phi-bar.
template <typename T>
__global__ __launch_bounds__(NT) void k_adj_init_pops(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                      AdjBufs<T> ab, int cur) {
  const Inst *Ip;
  int lblk;
  const Node nd = locate(insts, b2i, Ip, lblk);
  if (!nd.valid) return;
  const int N = Ip->N, n = nd.n;
  const T *A = ab.a[cur];
  const T *PB = ab.pb[cur];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T pb = PB[(size_t)i * N + n];
    T mb = -(T(1) - wgt<T>(0)) * (A[(size_t)(i * Q) * N + n] + pb);
#pragma unroll
    for (int j = 1; j < Q; ++j) mb += wgt<T>(j) * (A[(size_t)(i * Q + j) * N + n] + pb);
    ab.muL[(size_t)i * N + n] = Ip->phase_mode == 0 ? mb : T(0);
  }
}

// One potential sub-iteration on explicit buffers (the cold start of
// create, recomputed during the sweep): same collision and push as the
// forward potential kernels.
template <typename T>
__global__ __launch_bounds__(NT) void k_poisson_buf(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                    const T *__restrict__ src, T *__restrict__ dst,
                                                    const T *__restrict__ eps, const T *__restrict__ q,
                                                    T *rec_in) {
  const Inst *Ip;
  int lblk;
  const Node nd = locate(insts, b2i, Ip, lblk);
  if (!nd.valid) return;
  const Inst &I = *Ip;
  const Phys<T> &P = phys<T>(I);
  const int N = I.N, n = nd.n;
  T h[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) h[j] = src[(size_t)j * N + n];
  if (rec_in)
#pragma unroll
    for (int j = 0; j < Q; ++j) rec_in[(size_t)j * N + n] = h[j];
  T v[Q];
  poisson_collide<D2Q9>(h, eps[n] - P.eps_ref, q[n], P, v);
  push_potential<D2Q9>(dst, v, I, nd, P);
}

// Equilibrium potential populations of a potential plane (Eq. 44), the
// cold start's first level (stored as the deviation from the reference
// potential's equilibrium).
template <typename T>
__global__ __launch_bounds__(NT) void k_h_equilibrium(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                      const T *__restrict__ psi, T *__restrict__ h) {
  const Inst *Ip;
  int lblk;
  const Node nd = locate(insts, b2i, Ip, lblk);
  if (!nd.valid) return;
  const int N = Ip->N, n = nd.n;
  const T v = psi[n] - psi_ref<T>(phys<T>(*Ip), nd.y);
#pragma unroll
  for (int j = 0; j < Q; ++j) h[(size_t)j * N + n] = j == 0 ? (wgt<T>(0) - T(1)) * v : wgt<T>(j) * v;
}

// End of the sweep: the initial potential guess and the create-time
// permittivity.  psi0_b = adjoint of the equilibrium h of psi0 (d/d E0 via
// (psi0 - mean) / E0); eps-bar of create reaches eps_i through Eq. (30).
template <typename T>
__global__ __launch_bounds__(NT) void k_adj_create_tail(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                        AdjBufs<T> ab, int hsel, const T *__restrict__ phi0,
                                                        const T *__restrict__ psi0, double mean, double inv_e0) {
  const Inst *Ip;
  int lblk;
  const Node nd = locate(insts, b2i, Ip, lblk);
  const Inst &I = *Ip;
  double th[TB_SLOTS] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (nd.valid) {
    const int N = I.N, n = nd.n;
    const T *hb = ab.hb[hsel];
    T pb = (wgt<T>(0) - T(1)) * hb[n];
#pragma unroll
    for (int j = 1; j < Q; ++j) pb += wgt<T>(j) * hb[(size_t)j * N + n];
    th[6] += (double)pb * ((double)psi0[n] - mean) * inv_e0;
    const T eb = ab.eb[n];
#pragma unroll
    for (int i = 0; i < 3; ++i) th[i] += (double)(eb * herm(phi0[(size_t)i * N + n]));
  }
  add_theta(I, ab.tb, lblk, th);
}

// Sum of the per-block parameter adjoints (one block, fixed order).
__global__ __launch_bounds__(NT) void k_adj_reduce(const double *__restrict__ tb, int nblk, double *__restrict__ out) {
  double v[TB_SLOTS];
  reduce_partials<TB_SLOTS>(tb, nblk, v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < TB_SLOTS; ++k) out[k] = v[k];
}

}  // namespace lbm
