// Device-side data structures and kernels of the three-phase EHD LB step for
// gfx950.  Included once, by lbm_ehd.hip.
//
// The step kernels are templates on the lattice: D2Q9 (Eq. 31) on an
// nx x ny plane or D3Q15 (Eq. 32) on an nx x ny x nz box, periodic in x (and
// z), y periodic or bounded by half-way walls.  Vector fields carry D planes.
//
// Layout: every plane is [nz][ny][nx] with x fastest (structure of arrays), so
// a wave of 64 lanes reads 64 consecutive nodes of one row.  Populations are
// double-buffered; which buffer is current lives in a per-instance control
// block in device memory, so the host launch sequence (and a captured graph)
// does not depend on the step parity or on how many potential sub-iterations
// ran.
#pragma once
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

// Forward-mode (tangent) arithmetic: a value and its derivative along one
// parameter direction.  Instantiating the kernels with Dual<double> runs the
// exact tangent-linear step next to the FP64 step.
template <typename R> struct Dual {
  R v, d;
  __host__ __device__ constexpr Dual() : v(0), d(0) {}
  __host__ __device__ constexpr Dual(R a) : v(a), d(0) {}
  __host__ __device__ constexpr Dual(int a) : v(R(a)), d(0) {}
  __host__ __device__ constexpr Dual(R a, R b) : v(a), d(b) {}
  __host__ __device__ constexpr explicit operator double() const { return (double)v; }
  __host__ __device__ constexpr explicit operator float() const { return (float)v; }
  friend __host__ __device__ constexpr Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
  friend __host__ __device__ constexpr Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
  friend __host__ __device__ constexpr Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
  friend __host__ __device__ constexpr Dual operator/(Dual a, Dual b) {
    return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
  }
  __host__ __device__ constexpr Dual operator-() const { return Dual(-v, -d); }
  __host__ __device__ Dual &operator+=(Dual b) { v += b.v; d += b.d; return *this; }
  __host__ __device__ Dual &operator-=(Dual b) { v -= b.v; d -= b.d; return *this; }
  __host__ __device__ Dual &operator*=(Dual b) { *this = *this * b; return *this; }
};
using DualD = Dual<double>;

constexpr int NT = 256;  // threads per block (4 waves of 64)
constexpr int Q = 9;

// D2Q9 velocities and weights, Eq. (31).
__host__ __device__ constexpr int cx(int j) { return j == 1 || j == 5 || j == 8 ? 1 : (j == 3 || j == 6 || j == 7 ? -1 : 0); }
__host__ __device__ constexpr int cy(int j) { return j == 2 || j == 5 || j == 6 ? 1 : (j == 4 || j == 7 || j == 8 ? -1 : 0); }
__host__ __device__ constexpr int opp(int j) { return j == 0 ? 0 : (j <= 4 ? ((j + 1) & 3) + 1 : ((j - 3) & 3) + 5); }
template <typename T> __host__ __device__ constexpr T wgt(int j) {
  return j == 0 ? T(4) / T(9) : (j <= 4 ? T(1) / T(9) : T(1) / T(36));
}

// Velocity sets as compile-time traits: c(j, d), weights w, opposite
// direction, and the source weights of the potential scheme (Eq. 43:
// 0 at rest, equal on the moving directions, summing to one).
struct D2Q9 {
  static constexpr int Q = 9, D = 2;
  __host__ __device__ static constexpr int c(int j, int d) { return d == 0 ? cx(j) : (d == 1 ? cy(j) : 0); }
  __host__ __device__ static constexpr int op(int j) { return opp(j); }
  template <typename T> __host__ __device__ static constexpr T w(int j) { return wgt<T>(j); }
  template <typename T> __host__ __device__ static constexpr T varpi(int j) { return j ? T(1) / T(8) : T(0); }
};
struct D3Q15 {
  static constexpr int Q = 15, D = 3;
  __host__ __device__ static constexpr int c(int j, int d) {
    constexpr int X[15] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
    constexpr int Y[15] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1};
    constexpr int Z[15] = {0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, 1, -1, 1, -1};
    return d == 0 ? X[j] : (d == 1 ? Y[j] : Z[j]);
  }
  __host__ __device__ static constexpr int op(int j) { return j == 0 ? 0 : (j & 1 ? j + 1 : j - 1); }
  template <typename T> __host__ __device__ static constexpr T w(int j) {
    return j == 0 ? T(2) / T(9) : (j <= 6 ? T(1) / T(9) : T(1) / T(72));
  }
  template <typename T> __host__ __device__ static constexpr T varpi(int j) { return j ? T(1) / T(14) : T(0); }
};
template <class L, typename T> __host__ __device__ constexpr T lw(int j) { return L::template w<T>(j); }
template <class L, typename T> __host__ __device__ constexpr T lc(int j, int d) { return T(L::c(j, d)); }

// Per-instance control words (device memory).  The f/g/l buffer parity is
// known to the host (one flip per step) and passed to the kernels; the
// potential buffer parity depends on how many sub-iterations ran, so it lives
// here.  Hot kernels never use atomics: reductions go through per-block
// partials and a separate one-block-per-instance pass (fixed order).
struct Ctl {
  int hcur;          // current potential buffer at the start of a step
  int done;          // potential loop converged in this step (adaptive mode)
  int k_used;        // sub-iterations run in this step
  int status;        // latched conditions: ST_DIVERGED, ST_NOCONV
  double res_prev;   // relative potential change of the previous sub-iteration
  double res_last;   // relative potential change of the last sub-iteration
  long long k_total; // sub-iterations summed over steps
  long long steps;
  // diagnostics: [0..15] the outputs of lbm_ehd_diagnostics, [16..21] the
  // indicator centroids (outer x, y, z; inner x, y, z), [22] the seeded
  // directional derivative of a tangent run
  double diag[24];
};
// Status bits, set by the kernels and read (and partly cleared) by the host
// at its next synchronising call.
constexpr int ST_DIVERGED = 1;  // a non-finite velocity or pressure was formed
constexpr int ST_NOCONV = 2;    // a residual-controlled potential loop reached sub_max

// ref_a, ref_b: the fixed reference potential psi_ref(y) = ref_a + ref_b y
// of the potential populations' storage (see push_potential); hwall: the
// electrode potentials less psi_ref at the walls (zero unless a tangent run
// moves the electrodes).
template <typename T> struct Phys {
  T lam[3];
  T m0, tau_f, tau_l, tau_h, eps_ref, D;
  T rho[3], visc[3], eps[3], sig[3];
  T Eext[3], wall_u[2], wall_phi[2], wall_q[2];
  T ion_tau, ion_beta, ion_e;  // Nernst-Planck charge model
  T ref_a, ref_b, hwall[2];
};

// Instance descriptor (device memory, read with uniform loads).
// N is the plane stride: the node count nn rounded up to 64 nodes (every
// plane 256-byte aligned) plus a fixed skew against HBM address-mapping
// conflicts between planes.  Node n of a plane sits at offset n < nn; the
// tail up to N is padding no kernel reads.
struct Inst {
  int nx, ny, N, bc_y;
  int wall_q_mode, phase_mode, nblk, nz;
  int charge_model, nn, blk0, sum_relax;  // charge model: 0 leaky dielectric, 1 two-ion Nernst-Planck (l holds
                                          // [2][Q][N]); blk0: node blocks of the instances before this one;
                                          // sum_relax: restoring flux of phi_1 + phi_2 + phi_3
  void *f[2], *g[2], *l[2], *h[2];
  float *f0[2];  // FP16S only: FP32 rest populations f^i_0, [3][N]
  // planes: phi 3 (two buffers), lsum, eps, q (two buffers), R, psi, E D,
  // mu 3, u D, p, rho.  The order parameters and the charge formed in step n
  // are in buffer n & 1 (create's initial fields in buffer 1), so the
  // collide kernel finds the previous step's at its node for the time
  // derivatives of phi_i u and q u.
  void *phi[2], *lsum, *eps, *q[2], *R, *psi, *E, *mu, *u, *p, *rho;
  void *ion;  // Nernst-Planck: n_+, n_- [2][N] (null otherwise)
  double *part_p;   // potential residual partials, nblk x 2
  double *part_mu;  // last-iteration residual partials, nblk x 2
  double *part_d;   // diagnostics partials, nblk x 16
  Ctl *ctl;
  Phys<float> pf;
  Phys<double> pd;
  Phys<DualD> pt;  // tangent mode: parameters with their derivatives along one direction
};

// Global-memory view of a state pointer.  The pointers live in the instance
// descriptor, so the compiler cannot tell their address space and would emit
// flat loads and stores, whose completion it can only wait for all at once;
// global instructions complete in order and let loads stay in flight.
// Arithmetic element types only: the tangent type keeps generic pointers
// (its copy constructor cannot bind a global-memory reference), and FP16
// storage is viewed as raw 16-bit words (PopIO converts).
template <typename T>
using gptr = typename std::conditional<std::is_arithmetic<typename std::remove_cv<T>::type>::value,
                                       __attribute__((address_space(1))) T *, T *>::type;
template <typename T> __device__ __forceinline__ gptr<T> gbl(T *p) { return (gptr<T>)p; }
// Element i of a plane with a uniform base, addressed with a 32-bit byte
// offset (scalar base + vector offset addressing instead of a 64-bit vector
// address per load); a plane's byte offsets stay below 2^32 (fewer than 2^30
// nodes of 4 bytes, 2^29 of 8).
template <typename T>
__device__ __forceinline__ T ld_plane(const __attribute__((address_space(1))) T *base, unsigned i) {
  using cb = const __attribute__((address_space(1))) char *;
  return *(const __attribute__((address_space(1))) T *)((cb)base + i * (unsigned)sizeof(T));
}
template <typename T> __device__ __forceinline__ T ld_plane(const T *base, unsigned i) { return base[i]; }
// A pointer the caller knows to be uniform, materialised in scalar registers
// (keeps the compiler from folding a plane offset into every lane's address).
template <typename P> __device__ __forceinline__ P uniform_ptr(P p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (P)(((unsigned long long)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ void st_plane(__attribute__((address_space(1))) T *base, unsigned i, T v) {
  using bp = __attribute__((address_space(1))) char *;
  *(__attribute__((address_space(1))) T *)((bp)base + i * (unsigned)sizeof(T)) = v;
}
template <typename T> __device__ __forceinline__ void st_plane(T *base, unsigned i, T v) { base[i] = v; }
using gwords = __attribute__((address_space(1))) unsigned short *;
using gcwords = const __attribute__((address_space(1))) unsigned short *;
__device__ __forceinline__ gwords gbl(__half *p) { return (gwords)p; }
__device__ __forceinline__ gcwords gbl(const __half *p) { return (gcwords)p; }
__device__ __forceinline__ __half ld_half(const __half *p, size_t i) { return p[i]; }
__device__ __forceinline__ __half ld_half(gcwords p, size_t i) { return __ushort_as_half(p[i]); }
__device__ __forceinline__ __half ld_half(gwords p, size_t i) { return __ushort_as_half(p[i]); }
__device__ __forceinline__ void st_half(__half *p, size_t i, __half v) { p[i] = v; }
__device__ __forceinline__ void st_half(gwords p, size_t i, __half v) { p[i] = __half_as_ushort(v); }
// Read-only view in the constant address space, for descriptors no thread
// writes while the kernel runs (instance and tile tables, the control word
// outside the kernels that update it): uniform reads through it are scalar
// loads, off the vector-memory queue the population loads wait on.
template <typename T> using cptr = const T __attribute__((address_space(4))) *;
template <typename T> __device__ __forceinline__ cptr<T> cst(const T *p) { return (cptr<T>)p; }

template <typename T> __device__ __forceinline__ const Phys<T> &phys(const Inst &I);
template <> __device__ __forceinline__ const Phys<float> &phys<float>(const Inst &I) { return I.pf; }
template <> __device__ __forceinline__ const Phys<double> &phys<double>(const Inst &I) { return I.pd; }
template <> __device__ __forceinline__ const Phys<DualD> &phys<DualD>(const Inst &I) { return I.pt; }

// ------------------------------------------------------------ helpers

// Population storage.  FP32 and FP64 store the populations as they are.
// FP16S stores each population as a half-precision value scaled by a power
// of two per family (its deviation from the rest state, where g, l and the
// moving f populations vanish), and keeps the three rest populations f^i_0 in
// FP32: the colliding node writes f^i_0 = (its post-collision total) - (sum of
// the rounded moving populations it sends), so sum_x phi_i stays exact to
// FP32 rounding.  Arithmetic is FP32 in both FP32 and FP16S.
constexpr float SC_F = 16384.f;  // |f^i_j| < 4 for j >= 1
constexpr float SC_G = 65536.f;  // |g_j| < 1
constexpr float SC_L = 65536.f;  // |l_j| < 1

template <typename S, typename T> struct PopIO {
  static constexpr bool split = false;
  template <typename P> __device__ static __forceinline__ T ld(P p, size_t i, T) { return (T)p[i]; }
  template <typename P> __device__ static __forceinline__ void put(P p, size_t i, S v) { p[i] = v; }
  __device__ static __forceinline__ S cv(T v, T) { return (S)v; }
  __device__ static __forceinline__ T back(S s, T) { return (T)s; }
};
template <> struct PopIO<__half, float> {
  static constexpr bool split = true;
  template <typename P> __device__ static __forceinline__ float ld(P p, size_t i, float sc) {
    return __half2float(ld_half(p, i)) / sc;
  }
  template <typename P> __device__ static __forceinline__ void put(P p, size_t i, __half v) { st_half(p, i, v); }
  __device__ static __forceinline__ __half cv(float v, float sc) { return __float2half_rn(v * sc); }
  __device__ static __forceinline__ float back(__half s, float sc) { return __half2float(s) / sc; }
};

// Order-parameter populations are not evolved when the phases are frozen,
// so they stay in buffer 0 instead of alternating with the other families.
__device__ __forceinline__ int fbuf(const Inst &I, int pc) { return I.phase_mode ? 0 : pc; }

struct Node {
  int inst, n, x, y, z;
  bool valid;
};

// Forward values that the reverse (adjoint) sweep needs from one step, as
// written by the step's own kernels when the pointers are set (recording
// runs); null in ordinary steps.  Planes of N values each: phi 3, q, R, eps,
// E of the previous step 2, mu 3, E of this step 2, the pre-collision flow
// populations 9; the potential populations of each sub-iteration's input
// level go to the separate pointers of the potential kernels.
template <typename T> struct Rec {
  T *phi, *q, *R, *eps, *Eo, *mu, *En, *g;
};

// The block table maps each launched block to (instance, block within the
// instance).  The host orders it so that the blocks one XCD receives
// (consecutive block ids go round-robin over the 8 XCDs) cover a contiguous
// range of rows: stencil neighbours then hit that XCD's own L2.
//   bid, tid: the table entry and the thread within its NT nodes (a
//   launched block and its thread, or a persistent block's share of them).
template <class L = D2Q9>
__device__ __forceinline__ Node locate_at(const Inst *__restrict__ insts, const int2 *__restrict__ b2i, int bid,
                                          int tid, const Inst *&Ip, int &lblk) {
  __builtin_assume(tid >= 0 && tid < NT);
  // the tables are written by the host only: read through the constant
  // address space (scalar loads where bid is uniform, in every kernel)
  Node nd;
  const cptr<int> t = cst((const int *)b2i) + 2 * (size_t)bid;
  nd.inst = t[0];
  lblk = t[1];
  Ip = insts + nd.inst;
  const cptr<Inst> Ic = cst(Ip);
  const int nx = Ic->nx;
  const int local = lblk * NT + tid;
  nd.valid = local < Ic->nn;
  nd.n = nd.valid ? local : 0;
  int r = nd.n;
  nd.z = 0;
  if (L::D == 3) {
    const int plane = nx * Ic->ny;
    nd.z = r / plane;
    r -= nd.z * plane;
  }
  nd.y = r / nx;
  nd.x = r - nd.y * nx;
  return nd;
}
template <class L = D2Q9>
__device__ __forceinline__ Node locate(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                       const Inst *&Ip, int &lblk) {
  return locate_at<L>(insts, b2i, (int)blockIdx.x, (int)threadIdx.x, Ip, lblk);
}

__device__ __forceinline__ int wrapx(int x, int nx) { return x < 0 ? x + nx : (x >= nx ? x - nx : x); }
// x mod n; one: x is known to lie in [-n, 2n) (a uniform test), which
// takes one conditional add instead of the integer remainder
__device__ __forceinline__ int wrapn(int x, int n, bool one) { return one ? wrapx(x, n) : ((x % n) + n) % n; }
// finite-difference neighbour row: wrap (periodic) or mirror ghost (walls)
// (both forms computed and selected: no branch between the stencil loads)
__device__ __forceinline__ int fdrow(int y, int ny, int walls) {
  const int mirror = y < 0 ? 0 : (y >= ny ? ny - 1 : y);
  const int wrap = y < 0 ? y + ny : (y >= ny ? y - ny : y);
  return walls ? mirror : wrap;
}

// Node index of the Eq. (33) stencil point x + c_j (periodic wrap in x and
// z; mirror ghost rows at walls in y).
template <class L>
__device__ __forceinline__ int nbr(int nx, int ny, int nz, int bc_y, const Node &nd, int j) {
  const int row = fdrow(nd.y + L::c(j, 1), ny, bc_y);
  const int col = wrapx(nd.x + L::c(j, 0), nx);
  if (L::D == 2) return row * nx + col;
  return (wrapx(nd.z + L::c(j, 2), nz) * ny + row) * nx + col;
}
template <class L> __device__ __forceinline__ int nbr(const Inst &I, const Node &nd, int j) {
  return nbr<L>(I.nx, I.ny, I.nz, I.bc_y, nd, j);
}

// Eq. (33) gradient g[D] and Laplacian from the Q stencil values v[j]
// (v[j] = chi(x + c_j)).
// Terms whose lattice coefficient is zero are left out (they add exact
// zeros, which IEEE arithmetic would otherwise have to compute).
template <class L, typename T>
__device__ __forceinline__ void fdq(const T *v, T (&g)[L::D], T &lap) {
  T sg[L::D], sl = 0;
#pragma unroll
  for (int d = 0; d < L::D; ++d) sg[d] = 0;
#pragma unroll
  for (int j = 1; j < L::Q; ++j) {
#pragma unroll
    for (int d = 0; d < L::D; ++d)
      if (L::c(j, d) != 0) sg[d] += lw<L, T>(j) * lc<L, T>(j, d) * v[j];
    sl += T(2) * lw<L, T>(j) * (v[j] - v[0]);
  }
#pragma unroll
  for (int d = 0; d < L::D; ++d) g[d] = sg[d] * T(3);
  lap = sl * T(3);
}

// D2Q9 form of fdq with named components (used by the reverse-mode kernels).
template <typename T>
__device__ __forceinline__ void fd9(const T *v, T &gx, T &gy, T &lap) {
  T g[2];
  fdq<D2Q9, T>(v, g, lap);
  gx = g[0];
  gy = g[1];
}

// c_j . a for a D-vector a, over the nonzero components of c_j (the
// components are -1, 0 or 1: the products are exact).
template <class L, typename T>
__device__ __forceinline__ T cdot(int j, const T (&a)[L::D]) {
  T r = T(0);
  bool any = false;
#pragma unroll
  for (int d = 0; d < L::D; ++d) {
    const int c = L::c(j, d);
    if (c == 0) continue;
    const T t = c > 0 ? a[d] : -a[d];
    r = any ? r + t : t;
    any = true;
  }
  return r;
}

template <typename T> __device__ __forceinline__ T herm(T p) { return p * p * (T(3) - T(2) * p); }

// Block-wide sum of K doubles; result valid in thread 0.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K]) {
  __shared__ double red[NT / 64][K];
#pragma unroll
  for (int k = 0; k < K; ++k)
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_down(v[k], o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[w][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0;
      for (int i = 0; i < NT / 64; ++i) s += red[i][k];
      v[k] = s;
    }
}

// Second pass of a reduction, run by one block per instance: sums the K
// partials of nblk blocks in a fixed order (strided per thread, then the
// block tree), so results are bitwise reproducible.  Valid in thread 0.
template <int K>
__device__ __forceinline__ void reduce_partials(const double *__restrict__ part, int nblk, double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += NT)
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] += part[(size_t)b * K + k];
  block_sum<K>(v);
}

// Push-stream one family from node nd with half-way walls (y).
// mode 0: bounce-back with moving-wall term -2 w_j psi (c_j . u_w) / cs2
//         (walls move along x);
// mode 1: anti-bounce-back toward Dirichlet values (vb bottom, vt top).
// sc: storage scale (FP16S); skip0: do not store the rest population.
// Returns the sum of the moving populations as stored (after rounding).
template <class L, typename T, typename S, typename P>
__device__ __forceinline__ T push(P dst, const T (&v)[L::Q], const Inst &I, const Node &nd,
                                  int mode, T psi, T ub, T ut, T vb, T vt, T sc, bool skip0) {
  using IO = PopIO<S, T>;
  const int nx = I.nx, ny = I.ny, N = I.N, n = nd.n;
  T moved = 0;
#pragma unroll
  for (int j = 0; j < L::Q; ++j) {
    const int xd = wrapx(nd.x + L::c(j, 0), nx);
    int yd = nd.y + L::c(j, 1);
    const int zoff = L::D == 3 ? wrapx(nd.z + L::c(j, 2), I.nz) * ny : 0;
    T out = v[j];
    size_t idx;
    if (!I.bc_y) {
      yd = yd < 0 ? yd + ny : (yd >= ny ? yd - ny : yd);
      idx = (size_t)j * N + (zoff + yd) * nx + xd;
    } else if (yd >= 0 && yd < ny) {
      idx = (size_t)j * N + (zoff + yd) * nx + xd;
    } else {
      const bool top = yd >= ny;
      if (mode == 0)
        out = v[j] - T(2) * lw<L, T>(j) * psi * (lc<L, T>(j, 0) * (top ? ut : ub)) * T(3);
      else
        out = -v[j] + T(2) * lw<L, T>(j) * (top ? vt : vb);
      idx = (size_t)L::op(j) * N + n;
    }
    if (j == 0 && skip0) continue;
    const S st = IO::cv(out, sc);
    IO::put(dst, idx, st);
    if (j) moved += IO::back(st, sc);
  }
  return moved;
}

// Potential populations are stored as deviations from the equilibrium
// (Eq. 44) of a fixed reference potential, psi_ref(y) = ref_a + ref_b y: the
// linear profile between the electrodes (zero in a periodic box).  The
// reference equilibrium has no first moment, so the collision of Eqs. 43-45
// applies unchanged to the deviation (its potential is psi - psi_ref, its
// first moment that of h), and streaming it adds
// w_j (psi_ref(y - c_jy) - psi_ref(y)) = -w_j c_jy ref_b; at an electrode
// the anti-bounce-back value becomes phi_w - psi_ref(wall) (hwall).  Stored
// values are then O(psi - psi_ref) instead of O(psi): at 1024^2 with 5.12
// between the electrodes that keeps ~40x more of E = -grad(psi), formed from
// the cancelling first moment, in FP32 storage.
template <typename T, class PP> __device__ __forceinline__ T psi_ref(const PP &P, int y) {
  return P.ref_a + P.ref_b * T(y);
}
template <class L, typename T, class PP, typename Ptr>
__device__ __forceinline__ void push_potential(Ptr dst, T (&v)[L::Q], const Inst &I, const Node &nd, const PP &P) {
#pragma unroll
  for (int j = 0; j < L::Q; ++j)
    if (L::c(j, 1) != 0) v[j] -= lw<L, T>(j) * lc<L, T>(j, 1) * P.ref_b;
  push<L, T, T>(dst, v, I, nd, 1, T(0), T(0), T(0), P.hwall[0], P.hwall[1], T(1), false);
}

// ------------------------------------------------------------ kernels

// a1: order-parameter moments phi_i = sum_j f^i_j and the charge-population
// sum; resets the per-step potential control words.
template <class L, typename T, typename S>
__global__ __launch_bounds__(NT) void k_moments(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                int pc, Rec<T> rc = Rec<T>{}) {
  constexpr int Q = L::Q;
  const Inst *Ip;
  int lblk;
  const Node nd = locate<L>(insts, b2i, Ip, lblk);
  const Inst &I = *Ip;
  if (lblk == 0 && threadIdx.x == 0) {
    I.ctl->done = 0;
    I.ctl->k_used = 0;
  }
  if (!nd.valid) return;
  const int N = I.N, n = nd.n;
  using IO = PopIO<S, T>;
  const int fb = fbuf(I, pc);
  auto f = gbl((const S *)I.f[fb]);
  auto l = gbl((const S *)I.l[pc]);
  auto phi = gbl((T *)I.phi[pc]);
  // Every load before the first store: a store to a plane the compiler
  // cannot tell apart from the loaded ones would hold back the later loads.
  const bool ions = I.charge_model == 1;
  T fv[3][Q], lv[2][Q];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < Q; ++j)
      fv[i][j] = (IO::split && j == 0) ? (T)gbl(I.f0[fb])[(size_t)i * N + n]
                                       : IO::ld(f, (size_t)(i * Q + j) * N + n, T(SC_F));
#pragma unroll
  for (int j = 0; j < Q; ++j) lv[0][j] = IO::ld(l, (size_t)j * N + n, T(SC_L));
  if (ions)
#pragma unroll
    for (int j = 0; j < Q; ++j) lv[1][j] = IO::ld(l, (size_t)(Q + j) * N + n, T(SC_L));
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T a = IO::split ? fv[i][0] : T(0);
#pragma unroll
    for (int j = IO::split ? 1 : 0; j < Q; ++j) a += fv[i][j];
    phi[(size_t)i * N + n] = a;
    if (rc.phi) rc.phi[(size_t)i * N + n] = a;
  }
  if (ions) {
    // ion concentrations and the charge they carry (Eq. 52 model)
    T c[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      c[k] = 0;
#pragma unroll
      for (int j = 0; j < Q; ++j) c[k] += lv[k][j];
      (gbl((T *)I.ion))[(size_t)k * N + n] = c[k];
    }
    (gbl((T *)I.lsum))[n] = phys<T>(I).ion_e * (c[0] - c[1]);
    return;
  }
  T b = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) b += lv[0][j];
  (gbl((T *)I.lsum))[n] = b;
}

// a1 four nodes per thread (leaky-dielectric charge model): the same
// sums as k_moments, read and written as vectors of W nodes (16-byte loads
// and stores for four FP32 nodes, 8-byte half loads in FP16S): a quarter (or
// half) of the memory instructions of the node-per-thread form for a kernel
// that only streams.  Plane strides and block bases are multiples of 4
// nodes; the last vector of an instance may run into the plane's padding,
// which no kernel reads.
//   b2i4: (instance, block of 4 NT nodes within it) per table entry; with
//         W = 2 two consecutive launched blocks share an entry, one half each
//         (D3Q15 in FP32: 60 vectors of four floats would fill every VGPR).
constexpr int M4 = 4 * NT;  // nodes per block-table entry of k_moments4
template <typename T, int W> struct VecN {
  typedef T v __attribute__((ext_vector_type(W)));
};
//   rc: when rc.phi is set, the order parameters also go there (recording runs).
//   bid, tid: launched block (PER per table entry) and thread (k_moments4
//   passes its own; the persistent step its blocks' shares).
template <class L, typename T, typename S, int W = 4, bool CST = false>
__device__ __forceinline__ void moments4_body(const Inst *__restrict__ insts, const int2 *__restrict__ b2i4, int pc,
                                              const Rec<T> &rc, int bid, int tid) {
  static_assert(W == 4 || W == 2, "four or two nodes per thread");
  constexpr int Q = L::Q, PER = 4 / W;  // launched blocks per table entry
  using V = typename VecN<T, W>::v;
  using GV = const V __attribute__((address_space(1))) *;
  using GVW = V __attribute__((address_space(1))) *;
  // CST: the table and the descriptor (written by the host only) read
  // through the constant address space, scalar loads where the caller's
  // pointers come from memory (the persistent step; a launch's restrict
  // arguments give scalar loads already, and its code stays as it is)
  int2 t;
  if constexpr (CST) {
    const cptr<int> te = cst((const int *)b2i4) + 2 * (size_t)(bid / PER);
    t = make_int2(te[0], te[1]);
  } else {
    t = b2i4[bid / PER];
  }
  const int sub = bid % PER;
  const Inst &I = CST ? *(const Inst *)(cst(insts) + t.x) : insts[t.x];
  if (t.y == 0 && sub == 0 && tid == 0) {
    I.ctl->done = 0;
    I.ctl->k_used = 0;
  }
  const int base = t.y * M4 + sub * (W * NT) + W * tid;
  if (base >= I.nn) return;
  const size_t bv = (size_t)base / W, NV = (size_t)I.N / W;
  const int fb = fbuf(I, pc);
  V fv[3][Q], lv[Q];
  if constexpr (std::is_same<S, __half>::value) {
    // W half words per vector: f^i_0 in its FP32 plane, the rest as stored deviations
    typedef unsigned short hv __attribute__((ext_vector_type(W)));
    using GH = const hv __attribute__((address_space(1))) *;
    const GH f = (GH)I.f[fb], l = (GH)I.l[pc];
    const GV f0 = (GV)I.f0[fb];
    auto cvt = [](hv w, float sc) {
      V r;
#pragma unroll
      for (int c = 0; c < W; ++c) r[c] = __half2float(__ushort_as_half(w[c])) / sc;
      return r;
    };
    hv fw[3][Q], lw[Q];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 1; j < Q; ++j) fw[i][j] = f[(size_t)(i * Q + j) * NV + bv];
#pragma unroll
    for (int i = 0; i < 3; ++i) fv[i][0] = f0[(size_t)i * NV + bv];
#pragma unroll
    for (int j = 0; j < Q; ++j) lw[j] = l[(size_t)j * NV + bv];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 1; j < Q; ++j) fv[i][j] = cvt(fw[i][j], T(SC_F));
#pragma unroll
    for (int j = 0; j < Q; ++j) lv[j] = cvt(lw[j], T(SC_L));
  } else {
    const GV f = (GV)I.f[fb], l = (GV)I.l[pc];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < Q; ++j) fv[i][j] = f[(size_t)(i * Q + j) * NV + bv];
#pragma unroll
    for (int j = 0; j < Q; ++j) lv[j] = l[(size_t)j * NV + bv];
  }
  constexpr bool split = PopIO<S, T>::split;
  const GVW phi = (GVW)I.phi[pc];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    V a = split ? fv[i][0] : V(T(0));
#pragma unroll
    for (int j = split ? 1 : 0; j < Q; ++j) a += fv[i][j];
    phi[(size_t)i * NV + bv] = a;
    if (rc.phi) ((V *)rc.phi)[(size_t)i * NV + bv] = a;
  }
  V b = V(T(0));
#pragma unroll
  for (int j = 0; j < Q; ++j) b += lv[j];
  ((GVW)I.lsum)[bv] = b;
}
template <class L, typename T, typename S, int W = 4>
__global__ __launch_bounds__(NT) void k_moments4(const Inst *__restrict__ insts, const int2 *__restrict__ b2i4,
                                                 int pc, Rec<T> rc = Rec<T>{}) {
  moments4_body<L, T, S, W>(insts, b2i4, pc, rc, (int)blockIdx.x, (int)threadIdx.x);
}

// a2 + a3: permittivity/conductivity stencils (Eq. 33 on the eps and sigma
// fields of Eqs. 29-30), charge recovery q = (sum l + R'/2)/(1 + sigma/(2 eps))
// and the Ohmic source R of Eq. (47) with the previous step's field.
//   pc: the step's field buffer.
template <class L, typename T>
__global__ __launch_bounds__(NT) void k_pre(const Inst *__restrict__ insts, const int2 *__restrict__ b2i, int pc,
                                            Rec<T> rc = Rec<T>{}) {
  constexpr int Q = L::Q, D = L::D;
  const Inst *Ip;
  int lblk;
  const Node nd = locate<L>(insts, b2i, Ip, lblk);
  if (!nd.valid) return;
  const Inst &I = *Ip;
  const Phys<T> &P = phys<T>(I);
  const int N = I.N, n = nd.n;
  auto phi = gbl((const T *)I.phi[pc]);
  // the node's own loads first: issued with the stencil's, one memory
  // round trip for the whole kernel
  auto E = gbl((const T *)I.E);
  T e[D];
#pragma unroll
  for (int d = 0; d < D; ++d) e[d] = E[(size_t)d * N + n];
  const T lsum = (gbl((const T *)I.lsum))[n];
  // uniform plane bases and 32-bit node offsets (scalar base + vector offset
  // addressing instead of a 64-bit vector address per load)
  decltype(phi) pl[3] = {uniform_ptr(phi), uniform_ptr(phi + N), uniform_ptr(phi + 2 * (size_t)N)};
  T pv[3][Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int m = nbr<L>(I, nd, j);
#pragma unroll
    for (int i = 0; i < 3; ++i) pv[i][j] = ld_plane(pl[i], (unsigned)m);
  }
  T ev[Q], sv[Q];
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    ev[j] = P.eps[0] * herm(pv[0][j]) + P.eps[1] * herm(pv[1][j]) + P.eps[2] * herm(pv[2][j]);
    sv[j] = P.sig[0] * pv[0][j] + P.sig[1] * pv[1][j] + P.sig[2] * pv[2][j];
  }
  T ge[D], gs[D], dummy;
  fdq<L>(ev, ge, dummy);
  fdq<L>(sv, gs, dummy);
  const T se = sv[0] / ev[0];
  T gee = ge[0] * e[0], gse = gs[0] * e[0];
#pragma unroll
  for (int d = 1; d < D; ++d) {
    gee += ge[d] * e[d];
    gse += gs[d] * e[d];
  }
  const T Rp = se * gee - gse;
  const T q = (lsum + T(0.5) * Rp) / (T(1) + T(0.5) * se);
  (gbl((T *)I.q[pc]))[n] = q;
  (gbl((T *)I.R))[n] = -se * q + Rp;
  (gbl((T *)I.eps))[n] = ev[0];
  if (rc.q) {
    rc.q[n] = q;
    rc.R[n] = -se * q + Rp;
    rc.eps[n] = ev[0];
#pragma unroll
    for (int d = 0; d < D; ++d) rc.Eo[(size_t)d * N + n] = e[d];
  }
}

// Potential LB at one node (Eqs. 43-45): potential and gradient from the
// pre-collision h, then the collision with the eps_hat first-moment source
// and the charge source.  Returns the potential of the input h.
//   iden: 1 / (eps_hat + tau_h / 3), the node's gradient denominator, which
//   does not change between the sub-iterations of a step.
// An applied field E_ext is an imposed mean gradient: the populations carry
// the periodic part psi' of the potential psi = psi' - E_ext . x, and the
// eps_hat source and Eq. (45) take the gradient of the full psi, so the first
// moment m = -(tau_h/3) grad(psi') - eps_hat grad(psi) gives
// grad(psi) = -(m + (tau_h/3) E_ext) iden.
// Per-instance constants of the potential collision: 1/tau_h, 1 - 1/tau_h
// and the applied-field term (tau_h/3) E_ext of Eq. (45).
template <typename T, int D> struct PotK {
  T ith, omi, ge[D];
};
template <int D, typename T, class PP> __device__ __forceinline__ PotK<T, D> pot_k(const PP &P) {
  PotK<T, D> k;
  k.ith = T(1) / P.tau_h;
  k.omi = T(1) - k.ith;
#pragma unroll
  for (int d = 0; d < D; ++d) k.ge[d] = P.tau_h / T(3) * P.Eext[d];
  return k;
}

// Collision of one node's potential populations (Eqs. 43-45); returns the
// local potential.  BGK relaxation towards Eq. (44) with the eps_hat
// first-moment source of Eq. (43):
//   v_j = h_j (1 - 1/tau_h) + heq_j / tau_h - 3 w_j eps_hat c_j . grad(psi) / tau_h + varpi_j q,
// grad(psi) = -(m + (tau_h/3) E_ext) iden, iden = 1 / (eps_hat + tau_h/3)
// (Eq. 45); the factor 3 eps_hat / tau_h is folded into the gradient once.
template <class L, typename T>
__device__ __forceinline__ T poisson_collide(const T (&h)[L::Q], T epshat, T iden, T q, const PotK<T, L::D> &K,
                                             T (&v)[L::Q]) {
  constexpr int Q = L::Q, D = L::D;
  T s1 = h[1], m[D];
#pragma unroll
  for (int d = 0; d < D; ++d) m[d] = 0;
#pragma unroll
  for (int j = 2; j < Q; ++j) s1 += h[j];
#pragma unroll
  for (int j = 1; j < Q; ++j)
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (L::c(j, d) != 0) m[d] += lc<L, T>(j, d) * h[j];
  const T pot = s1 * (T(1) / (T(1) - lw<L, T>(0)));
  const T sc = -T(3) * epshat * K.ith * iden;
  T gs[D];
#pragma unroll
  for (int d = 0; d < D; ++d) gs[d] = (m[d] + K.ge[d]) * sc;
  const T pb = pot * K.ith;
  v[0] = h[0] * K.omi + (lw<L, T>(0) - T(1)) * pb;
#pragma unroll
  for (int j = 1; j < Q; ++j)
    v[j] = h[j] * K.omi + (lw<L, T>(j) * pb - lw<L, T>(j) * cdot<L>(j, gs) + L::template varpi<T>(j) * q);
  return pot;
}
template <typename T, class PP> __device__ __forceinline__ T poisson_iden(T epshat, const PP &P) {
  return T(1) / (epshat + P.tau_h / T(3));
}
template <class L, typename T, class PP>
__device__ __forceinline__ T poisson_collide(const T (&h)[L::Q], T epshat, T q, const PP &P, T (&v)[L::Q]) {
  return poisson_collide<L>(h, epshat, poisson_iden(epshat, P), q, pot_k<L::D, T>(P), v);
}

// a4: one potential sub-iteration (Eqs. 43-45): local potential and gradient
// from the pre-collision h, collision with the eps_hat first-moment source
// and the charge source, push with anti-bounce-back electrodes.
//   k: 1-based iteration index; K: iterations this step; hpar: parity of the
//   input buffer relative to ctl->hcur (fixed count: the launch index).
//   Fixed count (adaptive == 0): the last iteration stores the potential of
//   its input for the final residual.
//   Adaptive: skipped once the loop has converged; stores the potential of
//   its input and, from k = 2 on, the residual partials of the previous
//   iteration for k_reduce_poisson.
//   fb: the field buffer holding the charge (the step's; 1 at create).
//   rec_in: when set, receives the input level (recording runs).
template <class L, typename T>
__global__ __launch_bounds__(NT) void k_poisson(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                int k, int K, int adaptive, int hpar, int fb, T *rec_in = nullptr) {
  constexpr int Q = L::Q;
  const Inst *Ip;
  int lblk;
  const Node nd = locate<L>(insts, b2i, Ip, lblk);
  const Inst &I = *Ip;
  const cptr<Ctl> ctl = cst(I.ctl);  // written only by the control pass between launches
  if (adaptive && ctl->done) return;  // uniform over the instance
  const Phys<T> &P = phys<T>(I);
  const int hc = adaptive ? ctl->hcur : (ctl->hcur ^ hpar);
  const bool write_psi = adaptive || k == K;
  const bool resid = adaptive && k >= 2;
  double red[2] = {0.0, 0.0};
  if (nd.valid) {
    const int N = I.N, n = nd.n;
    auto src = gbl((const T *)I.h[hc]);
    auto dst = gbl((T *)I.h[hc ^ 1]);
    // every load before the first store (a later load would wait for it)
    T h[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) h[j] = src[(size_t)j * N + n];
    const T epshat = (gbl((const T *)I.eps))[n] - P.eps_ref;
    const T q = (gbl((const T *)I.q[fb]))[n];
    auto psi = gbl((T *)I.psi);
    const T psi_prev = resid ? psi[n] : T(0);
    if (rec_in)
#pragma unroll
      for (int j = 0; j < Q; ++j) rec_in[(size_t)j * N + n] = h[j];
    T v[Q];
    const T pot = poisson_collide<L>(h, epshat, q, P, v) + psi_ref<T>(P, nd.y);
    if (write_psi) {
      if (resid) {
        const double d = (double)pot - (double)psi_prev;
        red[0] = d * d;
        red[1] = (double)pot * (double)pot;
      }
      psi[n] = pot;
    }
    push_potential<L>(dst, v, I, nd, P);
  }
  if (resid) {
    block_sum<2>(red);
    if (threadIdx.x == 0) {
      I.part_p[(size_t)lblk * 2] = red[0];
      I.part_p[(size_t)lblk * 2 + 1] = red[1];
    }
  }
}

// Several potential sub-iterations in one launch (fixed count, D2Q9).  A
// block owns a tile and recomputes a ring of width IT (the sub-iterations
// per launch, 2 or 4) around it: it loads h, eps_hat and q of the extended
// tile (neighbour rows come from L2), collides every extended node, streams
// inside LDS (pull, with anti-bounce-back where the source lies beyond an
// electrode), and repeats on the region still valid, then writes the
// interior's pre-collision values to the other buffer: 80 B/node of HBM
// traffic per launch instead of 80 per sub-iteration.
//   tiles: (instance, x0, y0, -) per block; hpar: input parity relative to
//   ctl->hcur; write_psi: store the potential of the last sub-iteration's
//   input (the last launch of the step).
constexpr int P2NT = 1024;  // threads per block of the LDS-tiled potential kernel
constexpr int P2EW = 64, P2ER = 16, P2W = P2EW - 4, P2H = P2ER - 4, P2RPT = P2ER / (P2NT / 64);
// Tile shapes: RPT extended rows per thread, so a 64 x 16 RPT extended tile
// with a (16 RPT - 2 IT)-row, (64 - 2 IT)-column interior (RPT = 1, IT = 2:
// 60 x 12, 70% of the loaded nodes written; RPT = 2, IT = 2: 60 x 28, 82%,
// twice the LDS and half the blocks; RPT = 2, IT = 4: 56 x 24, 66%, one HBM
// round trip for four sub-iterations).  The launch configuration picks one.
//   IT: sub-iterations per launch (the width of the recomputed ring); the
//   interior is (64 - 2 IT) x (16 RPT - 2 IT).
template <int RPT, int IT = 2> struct P2Shape {
  static constexpr int ER = 16 * RPT, H = ER - 2 * IT, W = P2EW - 2 * IT;
};

// Per-tile values of the LDS-tiled potential kernel, read with scalar loads
// before the tile's population loads are issued.
template <typename T> struct P2Meta {
  const T *src, *eps, *q;
  T *dst, *psi;
  int nx, ny, N, walls;
  T tau_h, eps_ref, hwall[2], Eext[2], ref_a, ref_b;
  // the charge step folded into the launch (PRE): its inputs and outputs
  const T *phi, *Eo, *lsum;
  T *q_out, *R_out, *eps_out;
  T pe[3], ps[3];  // phase permittivities and conductivities (Eqs. 29-30)
};

//   COH: read the control word with a coherent load (the persistent step,
//   where an earlier stage of the same launch rewrote it) instead of
//   through the scalar cache.
template <typename T, bool PRE = false, bool COH = false>
__device__ __forceinline__ P2Meta<T> p2_meta(const Inst *insts, const int4 *tiles, int ti, int hpar, int fb, int4 &t) {
  const cptr<int> tp = cst((const int *)tiles) + 4 * (size_t)ti;
  t = make_int4(tp[0], tp[1], tp[2], 0);
  const cptr<Inst> I = cst(insts) + t.x;
  int hcur;
  if constexpr (COH)
    hcur = __hip_atomic_load(&I->ctl->hcur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    hcur = cst(I->ctl)->hcur;
  const int hc = hcur ^ hpar;
  P2Meta<T> m;
  m.src = (const T *)I->h[hc];
  m.dst = (T *)I->h[hc ^ 1];
  m.eps = (const T *)I->eps;
  m.q = (const T *)I->q[fb];
  m.psi = (T *)I->psi;
  m.nx = I->nx;
  m.ny = I->ny;
  m.N = I->N;
  m.walls = I->bc_y;
  if constexpr (sizeof(T) == 4) {
    m.tau_h = I->pf.tau_h;
    m.eps_ref = I->pf.eps_ref;
    m.hwall[0] = I->pf.hwall[0];
    m.hwall[1] = I->pf.hwall[1];
    m.ref_a = I->pf.ref_a;
    m.ref_b = I->pf.ref_b;
    m.Eext[0] = I->pf.Eext[0];
    m.Eext[1] = I->pf.Eext[1];
  } else {
    m.tau_h = I->pd.tau_h;
    m.eps_ref = I->pd.eps_ref;
    m.hwall[0] = I->pd.hwall[0];
    m.hwall[1] = I->pd.hwall[1];
    m.ref_a = I->pd.ref_a;
    m.ref_b = I->pd.ref_b;
    m.Eext[0] = I->pd.Eext[0];
    m.Eext[1] = I->pd.Eext[1];
  }
  if constexpr (PRE) {
    m.phi = (const T *)I->phi[fb];
    m.Eo = (const T *)I->E;
    m.lsum = (const T *)I->lsum;
    m.q_out = (T *)I->q[fb];
    m.R_out = (T *)I->R;
    m.eps_out = (T *)I->eps;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if constexpr (sizeof(T) == 4) {
        m.pe[i] = I->pf.eps[i];
        m.ps[i] = I->pf.sig[i];
      } else {
        m.pe[i] = I->pd.eps[i];
        m.ps[i] = I->pd.sig[i];
      }
    }
  }
  return m;
}

// Registers of one tile of the LDS-tiled potential kernel: this thread's RPT
// extended-tile nodes (h, eps, q; zeros beyond an electrode wall).  eps_hat
// = eps - eps_ref is formed after the loads, not between them.
template <typename T, int RPT> struct P2Regs {
  T h[RPT][Q], eh[RPT], qq[RPT], id[RPT];
  int gy[RPT];
  bool inside[RPT];
};

template <typename T, int RPT, int IT>
__device__ __forceinline__ void p2_load(const P2Meta<T> &m, const int4 t, P2Regs<T, RPT> &s) {
  const int nx = m.nx, ny = m.ny, N = m.N;
  auto src = gbl(m.src);
  // a 64-lane wave covers one row of the tile: the row index is uniform
  const int tx = threadIdx.x & 63, ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gx = wrapn(t.y - IT + tx, nx, nx >= P2EW);
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = ty + (P2NT / 64) * k;  // extended row of this thread's k-th node
    int y = t.z - IT + r;
    bool in = true;
    if (m.walls) in = (y >= 0 && y < ny);
    else y = wrapn(y, ny, ny >= 16 * RPT);
    s.gy[k] = y;
    s.inside[k] = in;
    if (in) {
      const int n = y * nx + gx;
#pragma unroll
      for (int j = 0; j < Q; ++j) s.h[k][j] = src[(size_t)j * N + n];
      s.eh[k] = (gbl(m.eps))[n];
      s.qq[k] = (gbl(m.q))[n];
    } else {
#pragma unroll
      for (int j = 0; j < Q; ++j) s.h[k][j] = T(0);
      s.eh[k] = T(0);
      s.qq[k] = T(0);
    }
  }
}

// Record outputs of the LDS-tiled kernel (recording runs): lev[i], when
// set, receives the input level of the launch's i-th sub-iteration on the
// tile's interior.
//   q, R, eps, Eo: when set, the charge step of a PRE launch records what
//   k_pre records (its charge, source, permittivity and the field it read).
template <typename T, int IT> struct P2Rec {
  T *lev[IT];
  T *q = nullptr, *R = nullptr, *eps = nullptr, *Eo = nullptr;
};

// Interior node of a tile (the nodes a launch writes) for this thread's k-th
// extended row: its node index in n.
template <typename T, int RPT, int IT>
__device__ __forceinline__ bool p2_interior(const P2Meta<T> &m, const int4 t, const P2Regs<T, RPT> &s, int k,
                                            int tx, int ty, int gx, int &n) {
  constexpr int H2 = P2Shape<RPT, IT>::H, W2 = P2Shape<RPT, IT>::W;
  const int r = ty + (P2NT / 64) * k;
  if (r < IT || r >= IT + H2 || tx < IT || tx >= IT + W2 || !s.inside[k]) return false;
  if (t.y + tx - IT >= m.nx || t.z + r - IT >= m.ny) return false;
  n = s.gy[k] * m.nx + gx;
  return true;
}

// a2 + a3 folded into the first potential launch of a step: the charge q,
// the Ohmic source R and the permittivity eps of k_pre, formed on the tile
// instead of in a launch of their own.  The permittivity and conductivity
// (Eqs. 29-30) of the extended tile and of a one-node ring around it (the
// reach of the Eq. 33 stencil) are formed once per node into LDS (the
// buffer the streaming uses afterwards); every extended node then takes its
// Eq. 33 gradients from there and forms q and R with the previous step's
// field, in k_pre's arithmetic; the interior stores q, R and eps for the
// later kernels of the step.
template <typename T, int RPT, int IT>
__device__ __forceinline__ void p2_load_pre(const P2Meta<T> &m, const int4 t, const P2Rec<T, IT> &rec,
                                            P2Regs<T, RPT> &s, T *buf) {
  constexpr int ER = P2Shape<RPT, IT>::ER, SW = P2EW + 2, SN = SW * (ER + 2), SP = (SN + P2NT - 1) / P2NT;
  static_assert(2 * SN <= (Q - 1) * P2EW * ER, "the ring fits the streaming buffer");
  const int nx = m.nx, ny = m.ny, N = m.N;
  auto src = gbl(m.src);
  auto phi = gbl(m.phi);
  const int tx = threadIdx.x & 63, ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gx = wrapn(t.y - IT + tx, nx, nx >= P2EW);
  // the ring's order parameters first (needed first), then this thread's
  // nodes: every load of the launch in flight at once
  T pv[SP][3];
#pragma unroll
  for (int u = 0; u < SP; ++u) {
    const int i = (int)threadIdx.x + u * P2NT;
    if (i < SN) {
      const int rr = i / SW, cc = i - rr * SW;
      int y = t.z - IT - 1 + rr;  // mirror ghost rows at walls
      y = m.walls ? (y < 0 ? 0 : (y >= ny ? ny - 1 : y)) : wrapn(y, ny, ny >= ER + 2);
      const int n = y * nx + wrapn(t.y - IT - 1 + cc, nx, nx >= SW);
#pragma unroll
      for (int c = 0; c < 3; ++c) pv[u][c] = phi[(size_t)c * N + n];
    }
  }
  T e[RPT][2], ls[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    const int r = ty + (P2NT / 64) * k;
    int y = t.z - IT + r;
    bool in = true;
    if (m.walls) in = (y >= 0 && y < ny);
    else y = wrapn(y, ny, ny >= 16 * RPT);
    s.gy[k] = y;
    s.inside[k] = in;
    if (in) {
      const int n = y * nx + gx;
#pragma unroll
      for (int j = 0; j < Q; ++j) s.h[k][j] = src[(size_t)j * N + n];
      e[k][0] = (gbl(m.Eo))[n];
      e[k][1] = (gbl(m.Eo))[(size_t)N + n];
      ls[k] = (gbl(m.lsum))[n];
    } else {
#pragma unroll
      for (int j = 0; j < Q; ++j) s.h[k][j] = T(0);
      e[k][0] = e[k][1] = ls[k] = T(0);
    }
  }
  // eps and sigma of the ring's nodes
  T *sev = buf, *ssv = buf + SN;
#pragma unroll
  for (int u = 0; u < SP; ++u) {
    const int i = (int)threadIdx.x + u * P2NT;
    if (i < SN) {
      sev[i] = m.pe[0] * herm(pv[u][0]) + m.pe[1] * herm(pv[u][1]) + m.pe[2] * herm(pv[u][2]);
      ssv[i] = m.ps[0] * pv[u][0] + m.ps[1] * pv[u][1] + m.ps[2] * pv[u][2];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    if (!s.inside[k]) {
      s.eh[k] = T(0);
      s.qq[k] = T(0);
      continue;
    }
    const int c = (ty + (P2NT / 64) * k + 1) * SW + tx + 1;
    T ev[Q], sv[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      ev[j] = sev[c + cy(j) * SW + cx(j)];
      sv[j] = ssv[c + cy(j) * SW + cx(j)];
    }
    T ge[2], gs[2], dummy;
    fdq<D2Q9>(ev, ge, dummy);
    fdq<D2Q9>(sv, gs, dummy);
    const T se = sv[0] / ev[0];
    T gee = ge[0] * e[k][0], gse = gs[0] * e[k][0];
    gee += ge[1] * e[k][1];
    gse += gs[1] * e[k][1];
    const T Rp = se * gee - gse;
    const T q = (ls[k] + T(0.5) * Rp) / (T(1) + T(0.5) * se);
    s.eh[k] = ev[0];
    s.qq[k] = q;
    int n;
    if (p2_interior<T, RPT, IT>(m, t, s, k, tx, ty, gx, n)) {
      (gbl(m.q_out))[n] = q;
      (gbl(m.R_out))[n] = -se * q + Rp;
      (gbl(m.eps_out))[n] = ev[0];
      if (rec.q) {
        rec.q[n] = q;
        rec.R[n] = -se * q + Rp;
        rec.eps[n] = ev[0];
        rec.Eo[n] = e[k][0];
        rec.Eo[(size_t)N + n] = e[k][1];
      }
    }
  }
  __syncthreads();  // the ring's LDS is the streaming buffer from here on
}

// The IT sub-iterations of one loaded tile and the store of its interior.

template <typename T, int RPT, int IT>
__device__ __forceinline__ void p2_run(const P2Meta<T> &m, const int4 t, int write_psi, const P2Rec<T, IT> &rec,
                                       P2Regs<T, RPT> &s, T *buf) {
  constexpr int ER = P2Shape<RPT, IT>::ER;
  const int nx = m.nx, ny = m.ny, N = m.N, walls = m.walls;
  auto dst = gbl(m.dst);
  // a 64-lane wave covers one row of the tile: row tests are uniform branches
  const int tx = threadIdx.x & 63, ty = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int gx = wrapn(t.y - IT + tx, nx, nx >= P2EW);
  // interior node of this tile (the nodes the launch writes)
  auto interior = [&](int k, int &n) { return p2_interior<T, RPT, IT>(m, t, s, k, tx, ty, gx, n); };
  // rows next to an electrode pull some values through the wall
  bool wall_row[RPT];
#pragma unroll
  for (int k = 0; k < RPT; ++k) wall_row[k] = walls && (s.gy[k] == 0 || s.gy[k] == ny - 1);
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    if (s.inside[k]) s.eh[k] -= m.eps_ref;
    s.id[k] = poisson_iden(s.eh[k], m);
  }
  const PotK<T, 2> pk = pot_k<2, T>(m);
  for (int it = 0; it < IT; ++it) {
    if (T *lev = rec.lev[it])
#pragma unroll
      for (int k = 0; k < RPT; ++k) {
        int n;
        if (interior(k, n))
#pragma unroll
          for (int j = 0; j < Q; ++j) lev[(size_t)j * N + n] = s.h[k][j];
      }
    // collide the rows this iteration can still use (rows outside the valid
    // ring hold no streamed values; the skip is uniform over a wave), post
    // the moving values to LDS; the rest value stays in a register
    T rest[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = ty + (P2NT / 64) * k, e = r * P2EW + tx;
      rest[k] = T(0);
      if (r < it || r >= ER - it) continue;
      T v[Q];
      const T pot = poisson_collide<D2Q9>(s.h[k], s.eh[k], s.id[k], s.qq[k], pk, v);
      int n;
      if (it == IT - 1 && write_psi && interior(k, n)) (gbl(m.psi))[n] = pot + psi_ref<T>(m, s.gy[k]);
      rest[k] = v[0];
#pragma unroll
      for (int j = 1; j < Q; ++j) buf[(j - 1) * (P2EW * ER) + e] = v[j];
    }
    __syncthreads();
    // pull streaming inside the tile; sources beyond an electrode reflect;
    // every pulled deviation takes the reference's shift -w_j c_jy ref_b
    const int lo = it + 1;  // ring still valid after this streaming
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int r = ty + (P2NT / 64) * k, e = r * P2EW + tx;
      if (r < lo || r >= ER - lo || tx < lo || tx >= P2EW - lo || !s.inside[k]) continue;
      s.h[k][0] = rest[k];
      if (wall_row[k]) {
#pragma unroll
        for (int j = 1; j < Q; ++j) {
          const int sy = s.gy[k] - cy(j);
          const T shift = -wgt<T>(j) * T(cy(j)) * m.ref_b;
          if (sy < 0 || sy >= ny)
            s.h[k][j] = -buf[(opp(j) - 1) * (P2EW * ER) + e] + T(2) * wgt<T>(j) * (sy < 0 ? m.hwall[0] : m.hwall[1]) + shift;
          else
            s.h[k][j] = buf[(j - 1) * (P2EW * ER) + e - cy(j) * P2EW - cx(j)] + shift;
        }
      } else {
#pragma unroll
        for (int j = 1; j < Q; ++j)
          s.h[k][j] = buf[(j - 1) * (P2EW * ER) + e - cy(j) * P2EW - cx(j)] - wgt<T>(j) * T(cy(j)) * m.ref_b;
      }
    }
    __syncthreads();
  }
  // interior pre-collision values of the next level
#pragma unroll
  for (int k = 0; k < RPT; ++k) {
    int n;
    if (interior(k, n))
#pragma unroll
      for (int j = 0; j < Q; ++j) dst[(size_t)j * N + n] = s.h[k][j];
  }
}

//   tiles: (instance, x0, y0, -) per block.
//   fb: the field buffer holding the charge (the step's; 1 at create).
//   rec: the input levels of the sub-iterations, for recording runs.
//   PRE: the launch also forms the step's charge, source and permittivity
//   (p2_load_pre; the first launch of a step, k_pre not launched).
//   ti: the tile (the launched block, or a persistent block's current one);
//   buf: the block's LDS of (Q - 1) P2EW ER values.
template <typename T, int RPT, int IT, bool PRE, bool COH = false>
__device__ __forceinline__ void p2_body(const Inst *__restrict__ insts, const int4 *__restrict__ tiles, int ti,
                                        int hpar, int write_psi, int fb, const P2Rec<T, IT> &rec, T *buf) {
  int4 t;
  const P2Meta<T> m = p2_meta<T, PRE, COH>(insts, tiles, ti, hpar, fb, t);
  P2Regs<T, RPT> s;
  if constexpr (PRE)
    p2_load_pre<T, RPT, IT>(m, t, rec, s, buf);
  else
    p2_load<T, RPT, IT>(m, t, s);
  p2_run<T, RPT, IT>(m, t, write_psi, rec, s, buf);
}
template <typename T, int RPT = 1, int IT = 2, bool PRE = false>
__global__ __launch_bounds__(P2NT, (sizeof(T) == 8 && RPT == 2) ? 4 : 8) void k_poisson2(const Inst *__restrict__ insts, const int4 *__restrict__ tiles,
                                                 int hpar, int write_psi, int fb, P2Rec<T, IT> rec = P2Rec<T, IT>{}) {
  constexpr int ER = P2Shape<RPT, IT>::ER;
  __shared__ T buf[(Q - 1) * P2EW * ER];  // the moving values; the rest value never leaves its node
  p2_body<T, RPT, IT, PRE>(insts, tiles, (int)blockIdx.x, hpar, write_psi, fb, rec, buf);
}

// Adaptive potential loop control, one block per instance, after iteration
// k: residual of iteration k-1, stopping test, buffer flip.
//   kcap: when > 0, reaching iteration kcap without stopping latches
//   ST_NOCONV (time steps; the cold start of create passes 0).
__global__ __launch_bounds__(NT) void k_reduce_poisson(const Inst *__restrict__ insts, int k, int kmin,
                                                       double tol, int kcap = 0) {
  const Inst &I = insts[blockIdx.x];
  Ctl *ctl = I.ctl;
  if (ctl->done) return;  // iteration k did not run
  double v[2];
  if (k >= 2) reduce_partials<2>(I.part_p, I.nblk, v);
  if (threadIdx.x == 0) {
    if (k >= 2) {
      const double na = sqrt(v[1]);
      const double r = sqrt(v[0]) / (na > 1e-30 ? na : 1e-30);
      ctl->res_prev = r;
      if (k >= (kmin > 2 ? kmin : 2) && r < tol) ctl->done = 1;
    }
    if (k == kcap && !ctl->done) ctl->status |= ST_NOCONV;
    ctl->k_used = k;
    ctl->hcur ^= 1;
  }
}

// a5: field E = -grad(psi) of the full potential from the converged h
// (Eq. 45 with the applied field: E = (m + (tau_h/3) E_ext) / den), the
// potential plane and last-iteration residual, and the chemical potentials
// of Eq. (20) with eps'(phi_i) = 6 eps_i phi_i (1 - phi_i).
// In three phases, so that a caller (the persistent step's field stage) can
// issue the loads of several node blocks before it waits for any: mu_locate (the node, the control word
// that names the final h buffer, and every plane address the node reads:
// all the reads a plane load depends on), mu_fetch (the plane loads alone:
// h, eps, the previous potential and the phi stencils) and mu_finish (the
// arithmetic and the stores).
template <class L, typename T> struct MuIn {
  Node nd;
  const Inst *Ip;
  int lblk, N, nx, ny, nz, bc_y;
  const T *h, *eps, *psi, *phi;
  T hv[L::Q], epsv, psi0, pv[3][L::Q];
};

//   bid, tid: node block and thread (see locate_at).  hofs: buffer offset
//   of the final h relative to ctl->hcur (fixed count: parity of the
//   potential launches; adaptive: 0, the control pass already flipped it).
//   pc: the step's field buffer (1 at create).  COH: the control word
//   through a coherent load (see p2_meta).
template <class L, typename T, bool COH = false>
__device__ __forceinline__ void mu_locate(const Inst *__restrict__ insts, const int2 *__restrict__ b2i, int bid,
                                          int tid, int hofs, int pc, MuIn<L, T> &in) {
  in.nd = locate_at<L>(insts, b2i, bid, tid, in.Ip, in.lblk);
  // a lane outside the grid fetches node 0 (in bounds; its values are not
  // used), so that the fetch is free of branches
  if (!in.nd.valid) in.nd.n = in.nd.x = in.nd.y = in.nd.z = 0;
  // the block's instance values (one node block is one instance: wave-
  // uniform values, kept in scalar registers; the descriptor is written by
  // the host only and read through the constant address space)
  const cptr<Inst> I = cst(in.Ip);
  // (the control word through a plain pointer: a scalar read here staggers
  // less and measured slower)
  const Ctl *ctl = I->ctl;
  int hcur;
  if constexpr (COH)
    hcur = __hip_atomic_load(&ctl->hcur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    hcur = ctl->hcur;
  in.N = __builtin_amdgcn_readfirstlane(I->N);
  in.nx = __builtin_amdgcn_readfirstlane(I->nx);
  in.ny = __builtin_amdgcn_readfirstlane(I->ny);
  in.nz = __builtin_amdgcn_readfirstlane(I->nz);
  in.bc_y = __builtin_amdgcn_readfirstlane(I->bc_y);
  in.h = uniform_ptr((const T *)I->h[hcur ^ hofs]);
  in.eps = uniform_ptr((const T *)I->eps);
  in.psi = uniform_ptr((const T *)I->psi);
  in.phi = uniform_ptr((const T *)I->phi[pc]);
}

template <class L, typename T>
__device__ __forceinline__ void mu_fetch(MuIn<L, T> &in) {
  constexpr int Q = L::Q;
  const int N = in.N, n = in.nd.n;
  auto h = gbl(in.h);
#pragma unroll
  for (int j = 0; j < Q; ++j) in.hv[j] = ld_plane(uniform_ptr(h + (size_t)j * N), (unsigned)n);
  in.epsv = (gbl(in.eps))[n];
  auto phi = gbl(in.phi);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const int m = nbr<L>(in.nx, in.ny, in.nz, in.bc_y, in.nd, j);
#pragma unroll
    for (int i = 0; i < 3; ++i) in.pv[i][j] = ld_plane(uniform_ptr(phi + (size_t)i * N), (unsigned)m);
  }
  in.psi0 = (gbl(in.psi))[n];
}

//   red receives this thread's residual terms.
template <class L, typename T>
__device__ __forceinline__ void mu_finish(const MuIn<L, T> &in, const Rec<T> &rc, double (&red)[2]) {
  constexpr int Q = L::Q, D = L::D;
  red[0] = red[1] = 0.0;
  if (!in.nd.valid) return;
  const Inst &I = *(const Inst *)cst(in.Ip);  // host-written: constant-space reads
  const Phys<T> &P = phys<T>(I);
  // every descriptor value the node uses, read before its first store (as
  // far as the compiler can tell a plane store may alias the descriptor, so
  // a read after one would be issued, and waited for, after it)
  const int N = in.N, n = in.nd.n;
  T *const psi = (T *)in.psi, *const E = (T *)I.E, *const mu = (T *)I.mu;
  const T pref = psi_ref<T>(P, in.nd.y), tau_h = P.tau_h, eps_ref = P.eps_ref, width = P.D;
  T Eext[D], lam[3], epsi[3];
#pragma unroll
  for (int d = 0; d < D; ++d) Eext[d] = P.Eext[d];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    lam[i] = P.lam[i];
    epsi[i] = P.eps[i];
  }
  T s1 = 0, m[D];
#pragma unroll
  for (int d = 0; d < D; ++d) m[d] = 0;
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const T v = in.hv[j];
    if (j) s1 += v;
#pragma unroll
    for (int d = 0; d < D; ++d)
      if (L::c(j, d) != 0) m[d] += lc<L, T>(j, d) * v;
  }
  const T pot = s1 * (T(1) / (T(1) - lw<L, T>(0))) + pref;
  const T th3 = tau_h / T(3), iden = T(1) / ((in.epsv - eps_ref) + th3);
  T e[D];
#pragma unroll
  for (int d = 0; d < D; ++d) e[d] = (m[d] + th3 * Eext[d]) * iden;
  const double dd = (double)pot - (double)in.psi0;
  red[0] = dd * dd;
  red[1] = (double)pot * (double)pot;
  (gbl(psi))[n] = pot;
  auto Eg = gbl(E);
  T e2 = e[0] * e[0];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    st_plane(uniform_ptr(Eg + (size_t)d * N), (unsigned)n, e[d]);
    if (rc.En) rc.En[(size_t)d * N + n] = e[d];
    if (d) e2 += e[d] * e[d];
  }
  auto mug = gbl(mu);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    T gg[D], lap;
    fdq<L>(in.pv[i], gg, lap);
    const T ph = in.pv[i][0];
    const T bulk = T(24) / width * lam[i] * ph * (ph - T(0.5)) * (ph - T(1));
    const T grad = T(0.75) * width * lam[i] * lap;
    const T elec = T(0.5) * (T(6) * epsi[i] * ph * (T(1) - ph)) * e2;
    st_plane(uniform_ptr(mug + (size_t)i * N), (unsigned)n, bulk - grad - elec);
    if (rc.mu) rc.mu[(size_t)i * N + n] = bulk - grad - elec;
  }
}

// The same arithmetic in one pass, for the separate launch (loads and
// arithmetic interleaved as the compiler schedules them: 0.4 us faster at
// 1024^2 than the three phases above; the two agree bitwise, which the
// persistent-step tests check against ordinary steps).
//   hofs: buffer offset of the final h relative to ctl->hcur (fixed count:
//   parity of the potential launches; adaptive: 0, the control pass already
//   flipped it).
//   pc: the step's field buffer (1 at create).
//   bid, tid: node block and thread (see locate_at); red receives this
//   thread's residual terms, Ip and lblk the block's instance.  COH: the
//   control word through a coherent load (see p2_meta).
template <class L, typename T, bool COH = false>
__device__ __forceinline__ void mu_body(const Inst *__restrict__ insts, const int2 *__restrict__ b2i, int hofs, int pc,
                                        const Rec<T> &rc, int bid, int tid, double (&red)[2], const Inst *&Ip,
                                        int &lblk) {
  constexpr int Q = L::Q, D = L::D;
  const Node nd = locate_at<L>(insts, b2i, bid, tid, Ip, lblk);
  const Inst &I = *Ip;
  // (the control word through a plain pointer: a scalar read here staggers
  // less and measured slower)
  const Ctl *ctl = I.ctl;
  const Phys<T> &P = phys<T>(I);
  red[0] = red[1] = 0.0;
  if (nd.valid) {
    const int N = I.N, n = nd.n;
    int hcur;
    if constexpr (COH)
      hcur = __hip_atomic_load(&ctl->hcur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
      hcur = ctl->hcur;
    auto h = gbl((const T *)I.h[hcur ^ hofs]);
    T s1 = 0, m[D];
#pragma unroll
    for (int d = 0; d < D; ++d) m[d] = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const T v = ld_plane(uniform_ptr(h + (size_t)j * N), (unsigned)n);
      if (j) s1 += v;
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (L::c(j, d) != 0) m[d] += lc<L, T>(j, d) * v;
    }
    const T eps = (gbl((const T *)I.eps))[n];
    const T pot = s1 * (T(1) / (T(1) - lw<L, T>(0))) + psi_ref<T>(P, nd.y);
    const T th3 = P.tau_h / T(3), iden = T(1) / ((eps - P.eps_ref) + th3);
    T e[D];
#pragma unroll
    for (int d = 0; d < D; ++d) e[d] = (m[d] + th3 * P.Eext[d]) * iden;
    auto psi = gbl((T *)I.psi);
    // the phi stencils and the previous potential, loaded before the first
    // store (later loads would wait for it: the compiler cannot tell the
    // planes apart)
    auto phi = gbl((const T *)I.phi[pc]);
    T pv[3][Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const int m = nbr<L>(I, nd, j);
#pragma unroll
      for (int i = 0; i < 3; ++i) pv[i][j] = ld_plane(uniform_ptr(phi + (size_t)i * N), (unsigned)m);
    }
    const double dd = (double)pot - (double)psi[n];
    red[0] = dd * dd;
    red[1] = (double)pot * (double)pot;
    psi[n] = pot;
    auto E = gbl((T *)I.E);
    T e2 = e[0] * e[0];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      st_plane(uniform_ptr(E + (size_t)d * N), (unsigned)n, e[d]);
      if (rc.En) rc.En[(size_t)d * N + n] = e[d];
      if (d) e2 += e[d] * e[d];
    }
    auto mu = gbl((T *)I.mu);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T gg[D], lap;
      fdq<L>(pv[i], gg, lap);
      const T ph = pv[i][0];
      const T bulk = T(24) / P.D * P.lam[i] * ph * (ph - T(0.5)) * (ph - T(1));
      const T grad = T(0.75) * P.D * P.lam[i] * lap;
      const T elec = T(0.5) * (T(6) * P.eps[i] * ph * (T(1) - ph)) * e2;
      st_plane(uniform_ptr(mu + (size_t)i * N), (unsigned)n, bulk - grad - elec);
      if (rc.mu) rc.mu[(size_t)i * N + n] = bulk - grad - elec;
    }
  }
}
template <class L, typename T>
__global__ __launch_bounds__(NT) void k_mu(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                           int hofs, int pc, Rec<T> rc = Rec<T>{}) {
  double red[2];
  const Inst *Ip;
  int lblk;
  mu_body<L, T>(insts, b2i, hofs, pc, rc, (int)blockIdx.x, (int)threadIdx.x, red, Ip, lblk);
  block_sum<2>(red);
  if (threadIdx.x == 0) {
    Ip->part_mu[(size_t)lblk * 2] = red[0];
    Ip->part_mu[(size_t)lblk * 2 + 1] = red[1];
  }
}

// a6-a11: grad(mu_i) (Eq. 33), force -sum phi_i grad mu_i + q E (Eq. 27b),
// flow moments (Eq. 41), degenerate mobility (Eq. 28), the three CH
// collisions (Eqs. 34-36), the flow collision (Eqs. 37-40) and the charge
// collision (Eqs. 48-50), each pushed to its neighbours with wall rules.
//   pc: current f/g/l buffer; write_macro: store u, p, rho for output;
//   fixedK: sub-iterations of a fixed-count step (0 in adaptive mode) and
//   hflip the buffer parity of its launches, which block 0 folds into
//   ctl->hcur (no other kernel of the step reads it any more).
//   EARLY: load schedule (see below; a launch-configuration choice, both
//   give bitwise the same results).  The per-family D2Q9 FP32/FP16S form is
//   held to 128 VGPRs (4 waves per SIMD), which it fits without spilling.
//   bid, tid: node block and thread (see locate_at).
template <class L, typename T, typename S, bool EARLY, bool CST = false>
__device__ __forceinline__ void collide_body(const Inst *__restrict__ insts, const int2 *__restrict__ b2i, int pc,
                                             int write_macro, int fixedK, int hflip, const Rec<T> &rc, int bid,
                                             int tid) {
  constexpr int Q = L::Q, D = L::D;
  const Inst *Ip;
  int lblk;
  const Node nd = locate_at<L>(insts, b2i, bid, tid, Ip, lblk);
  // CST: the descriptor (written by the host only) read through the
  // constant address space, for callers whose pointers come from memory
  // (the persistent step); a launch keeps its code as it is
  const Inst &I = CST ? *(const Inst *)cst(Ip) : *Ip;
  if (lblk == 0 && tid == 0) {
    // device-scope atomics: in the persistent step an earlier stage of the
    // same launch, on another CU, wrote these words
    Ctl *ctl = I.ctl;
    int ku;
    if (fixedK > 0) {
      __hip_atomic_fetch_xor(&ctl->hcur, hflip, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctl->k_used, fixedK, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ku = fixedK;
    } else {
      ku = __hip_atomic_load(&ctl->k_used, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __hip_atomic_fetch_add(&ctl->k_total, (long long)ku, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_add(&ctl->steps, 1LL, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (nd.valid) {
    const Phys<T> &P = phys<T>(I);
    const int N = I.N, n = nd.n;
    auto phi = gbl((const T *)I.phi[pc]);
    auto mu = gbl((const T *)I.mu);
    int m[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) m[j] = nbr<L>(I, nd, j);

    // density stencil (Eq. 33 on rho of Eq. 29) and mu gradients
    T ph[3], rv[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const T p1 = phi[m[j]], p2 = phi[(size_t)N + m[j]], p3 = phi[(size_t)2 * N + m[j]];
      rv[j] = P.rho[0] * p1 + P.rho[1] * p2 + P.rho[2] * p3;
      if (j == 0) {
        ph[0] = p1;
        ph[1] = p2;
        ph[2] = p3;
      }
    }
    T gr[D], dummy;
    fdq<L>(rv, gr, dummy);
    T gS[D];  // gradient of S = phi_1 + phi_2 + phi_3 (restoring flux of the sum)
#pragma unroll
    for (int d = 0; d < D; ++d) gS[d] = T(0);
    if (I.sum_relax) {
      T sv[Q];
#pragma unroll
      for (int j = 0; j < Q; ++j) sv[j] = phi[m[j]] + phi[(size_t)N + m[j]] + phi[(size_t)2 * N + m[j]];
      fdq<L>(sv, gS, dummy);
    }
    T gm[3][D], muc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      T v[Q];
#pragma unroll
      for (int j = 0; j < Q; ++j) v[j] = mu[(size_t)i * N + m[j]];
      fdq<L>(v, gm[i], dummy);
      muc[i] = v[0];
    }
    const T rho = rv[0];
    const T q = (gbl((const T *)I.q[pc]))[n];
    auto E = gbl((const T *)I.E);

    // force and flow moments
    T F[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      F[d] = q * E[(size_t)d * N + n];
#pragma unroll
      for (int i = 0; i < 3; ++i) F[d] -= ph[i] * gm[i][d];
    }
    // Load schedule.  EARLY: every population and previous-step value is loaded
    // before the first store (the stores, to buffers the compiler cannot
    // tell apart from the loaded ones, would otherwise hold back the loads
    // issued after them): most loads in flight, ~160 VGPRs.  Otherwise each
    // family is loaded next to its use: fewer registers, higher occupancy,
    // which wins when the state sits in the Infinity Cache.  8-byte values
    // always use the second form (the early copy would halve the occupancy).
    using IO = PopIO<S, T>;
    constexpr bool early = EARLY && sizeof(T) <= 4;
    const bool ch = I.phase_mode == 0;
    const int fbs = fbuf(I, pc);
    auto gs = gbl((const S *)I.g[pc]);
    auto fs = gbl((const S *)I.f[fbs]);
    auto ls = gbl((const S *)I.l[pc]);
    // the previous step's phi_i, q (the other field buffer) and u at this node
    auto php = gbl((const T *)I.phi[pc ^ 1]);
    auto qp = gbl((const T *)I.q[pc ^ 1]);
    auto uu = gbl((T *)I.u);
    T g[Q], fin[3][Q], lin[Q], ph0[3], u0[D], q0 = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) g[j] = IO::ld(gs, (size_t)j * N + n, T(SC_G));
    auto ldf = [&](int i, int j) -> T {
      return (IO::split && j == 0) ? (T)gbl(I.f0[fbs])[(size_t)i * N + n]
                                   : IO::ld(fs, (size_t)(i * Q + j) * N + n, T(SC_F));
    };
    if (early && ch)
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < Q; ++j) fin[i][j] = ldf(i, j);
    const bool ions = I.charge_model == 1;
    if (early && !ions)
#pragma unroll
      for (int j = 0; j < Q; ++j) lin[j] = IO::ld(ls, (size_t)j * N + n, T(SC_L));
    const T R = (gbl((const T *)I.R))[n];
    auto ld_prev = [&]() {
#pragma unroll
      for (int i = 0; i < 3; ++i) ph0[i] = php[(size_t)i * N + n];
#pragma unroll
      for (int d = 0; d < D; ++d) u0[d] = uu[(size_t)d * N + n];
      q0 = qp[n];
    };
    if (early) ld_prev();
    if (rc.g)
#pragma unroll
      for (int j = 0; j < Q; ++j) rc.g[(size_t)j * N + n] = g[j];
    T mg[D], s1 = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) mg[d] = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
#pragma unroll
      for (int d = 0; d < D; ++d)
        if (L::c(j, d) != 0) mg[d] += lc<L, T>(j, d) * g[j];
      if (j) s1 += g[j];
    }
    T u[D];
#pragma unroll
    for (int d = 0; d < D; ++d) u[d] = (mg[d] + T(0.5) * F[d]) / rho;
    T udr = u[0] * gr[0], usq = u[0] * u[0];
#pragma unroll
    for (int d = 1; d < D; ++d) {
      udr += u[d] * gr[d];
      usq += u[d] * u[d];
    }
    const T s0 = lw<L, T>(0) * (-usq * T(1.5));
    const T pp = (s1 + T(0.5) * udr + rho * s0) / (T(3) * (T(1) - lw<L, T>(0)));
    // divergence watch: a non-finite population, order parameter, charge,
    // field or chemical potential reaches u or p within a step; latched for
    // the host (an atomic only on that rare path)
    {
      bool ok = isfinite((double)pp);
#pragma unroll
      for (int d = 0; d < D; ++d) ok = ok && isfinite((double)u[d]);
      if (!ok) atomicOr(&I.ctl->status, ST_DIVERGED);
    }
    if (!early) ld_prev();
    // first-order time derivatives of phi_i u and q u against the previous
    // step's values (the products formed as the previous step formed them)
    T dp[3][D], dq[D];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const T b = ph0[i] * u0[d];
        dp[i][d] = ph[i] * u[d] - b;
      }
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const T b = q0 * u0[d];
      dq[d] = q * u[d] - b;
    }
    // u every step (the next step's previous velocity); p and rho for output
#pragma unroll
    for (int d = 0; d < D; ++d) uu[(size_t)d * N + n] = u[d];
    if (write_macro) {
      (gbl((T *)I.p))[n] = pp;
      (gbl((T *)I.rho))[n] = rho;
    }

    const int nc = pc ^ 1;
    // three CH families
    if (ch) {
      const T m0 = P.m0, itf = T(1) / P.tau_f, cf = T(1) - T(0.5) * itf;
      // optional restoring flux m0 (phi_i / S) grad S of the constraint S = 1
      const T wsum = I.sum_relax ? m0 / (ph[0] + ph[1] + ph[2]) : T(0);
      const int fbd = fbuf(I, nc);
      auto fd = gbl((S *)I.f[fbd]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        // degenerate mobility row i: M_ik = -m0 phi_i phi_k, M_ii = -sum_k M_ik
        T X[D], mii = 0;
#pragma unroll
        for (int d = 0; d < D; ++d) X[d] = 0;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
          if (kk != i) {
            const T mik = -m0 * ph[i] * ph[kk];
            mii -= mik;
#pragma unroll
            for (int d = 0; d < D; ++d) X[d] += mik * gm[kk][d];
          }
        T dt[D], pu[D];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          X[d] += (mii - m0) * gm[i][d] + wsum * ph[i] * gS[d];
          dt[d] = dp[i][d] * T(3) - X[d] / m0;
          pu[d] = ph[i] * u[d];
        }
        T v[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          const T fj = early ? fin[i][j] : ldf(i, j);
          const T cu = cdot<L>(j, pu);
          const T feq = j == 0 ? ph[i] - (T(1) - lw<L, T>(0)) * muc[i] : lw<L, T>(j) * muc[i] + lw<L, T>(j) * cu * T(3);
          const T Fj = lw<L, T>(j) * cdot<L>(j, dt);
          v[j] = fj - (fj - feq) * itf + cf * Fj;
        }
        const T moved = push<L, T, S>(fd + (size_t)i * Q * N, v, I, nd, 0, ph[i], P.wall_u[0], P.wall_u[1], T(0),
                                      T(0), T(SC_F), IO::split);
        if (IO::split) {
          T tot = 0;
#pragma unroll
          for (int j = 0; j < Q; ++j) tot += v[j];
          gbl(I.f0[fbd])[(size_t)i * N + n] = (float)(tot - moved);
        }
      }
    }

    // flow family
    {
      const T tg = T(0.5) + (P.visc[0] * ph[0] + P.visc[1] * ph[1] + P.visc[2] * ph[2]) * T(3) / rho;
      const T itg = T(1) / tg, cg = T(1) - T(0.5) * itg;
      T v[Q];
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const T cu = cdot<L>(j, u);
        const T sj = lw<L, T>(j) * (cu * T(3) + cu * cu * T(4.5) - usq * T(1.5));
        const T geq = (j == 0 ? (lw<L, T>(0) - T(1)) * pp * T(3) : lw<L, T>(j) * pp * T(3)) + rho * sj;
        const T cF = cdot<L>(j, F);
        const T cgr = cdot<L>(j, gr);
        const T Gb = lw<L, T>(j) * (udr + cF * T(3) + (cu * cgr - udr / T(3)) * T(3));
        v[j] = g[j] - (g[j] - geq) * itg + cg * Gb;
      }
      push<L, T, S>(gbl((S *)I.g[nc]), v, I, nd, 0, rho, P.wall_u[0], P.wall_u[1], T(0), T(0), T(SC_G), false);
    }

    // two ion families (Nernst-Planck model): BGK advection-diffusion with
    // the drift z beta D E of this step's field, no-flux walls
    if (ions) {
      const T itn = T(1) / P.ion_tau, Dn = (P.ion_tau - T(0.5)) / T(3);
      auto E = gbl((const T *)I.E);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const T z = k == 0 ? T(1) : T(-1);
        T m[Q], ns = 0;
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          m[j] = IO::ld(ls, (size_t)(k * Q + j) * N + n, T(SC_L));
          ns += m[j];
        }
        T w[D];
#pragma unroll
        for (int d = 0; d < D; ++d) w[d] = u[d] + z * P.ion_beta * Dn * E[(size_t)d * N + n];
        T v[Q];
#pragma unroll
        for (int j = 0; j < Q; ++j) {
          const T meq = lw<L, T>(j) * ns * (T(1) + cdot<L>(j, w) * T(3));
          v[j] = m[j] - (m[j] - meq) * itn;
        }
        push<L, T, S>(gbl((S *)I.l[nc]) + (size_t)k * Q * N, v, I, nd, 0, ns, P.wall_u[0], P.wall_u[1], T(0), T(0),
                      T(SC_L), false);
      }
    }

    // charge family
    if (!ions) {
      const T itl = T(1) / P.tau_l, cl = T(1) - T(0.5) * itl;
      T v[Q];
#pragma unroll
      for (int j = 0; j < Q; ++j) {
        const T lj = early ? lin[j] : IO::ld(ls, (size_t)j * N + n, T(SC_L));
        const T cu = cdot<L>(j, u);
        const T leq = lw<L, T>(j) * q * (T(1) + cu * T(3));
        const T Sj = cl * lw<L, T>(j) * R;
        const T Tj = cl * lw<L, T>(j) * cdot<L>(j, dq) * T(3);
        v[j] = lj - (lj - leq) * itl + Sj + Tj;
      }
      const int mode = I.wall_q_mode == 1 ? 1 : 0;
      push<L, T, S>(gbl((S *)I.l[nc]), v, I, nd, mode, q, P.wall_u[0], P.wall_u[1], P.wall_q[0], P.wall_q[1],
                    T(SC_L), false);
    }
  }
}
template <class L, typename T, typename S, bool EARLY = (sizeof(T) <= 4)>
__global__ __launch_bounds__(NT, (EARLY || sizeof(T) > 4 || L::Q > 9) ? 1 : 4) void k_collide(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                int pc, int write_macro, int fixedK, int hflip,
                                                Rec<T> rc = Rec<T>{}) {
  collide_body<L, T, S, EARLY>(insts, b2i, pc, write_macro, fixedK, hflip, rc, (int)blockIdx.x, (int)threadIdx.x);
}

// ------------------------------------------------------------ create-time

// Permittivity of the initial order parameters and the potential
// populations at the equilibrium of the initial guess (Eq. 44).
template <class L, typename T>
__global__ __launch_bounds__(NT) void k_init_potential(const Inst *__restrict__ insts, const int2 *__restrict__ b2i) {
  constexpr int Q = L::Q;
  const Inst *Ip;
  int lblk;
  const Node nd = locate<L>(insts, b2i, Ip, lblk);
  if (!nd.valid) return;
  const Inst &I = *Ip;
  const Phys<T> &P = phys<T>(I);
  const int N = I.N, n = nd.n;
  auto phi = gbl((const T *)I.phi[1]);  // create's fields: buffer 1
  (gbl((T *)I.eps))[n] = P.eps[0] * herm(phi[n]) + P.eps[1] * herm(phi[(size_t)N + n]) + P.eps[2] * herm(phi[(size_t)2 * N + n]);
  const T v = (gbl((const T *)I.psi))[n] - psi_ref<T>(P, nd.y);  // stored as the deviation
  auto h = gbl((T *)I.h[I.ctl->hcur]);
#pragma unroll
  for (int j = 0; j < Q; ++j) h[(size_t)j * N + n] = j == 0 ? (lw<L, T>(0) - T(1)) * v : lw<L, T>(j) * v;
}

// Equilibria of the initial fields (p = 0) into population buffer 0 (the
// initial fields in field buffer 1 and u serve as the first step's previous
// values); block 0 folds the cold start's buffer parity hofs into ctl->hcur.
template <class L, typename T, typename S>
__global__ __launch_bounds__(NT) void k_init_pops(const Inst *__restrict__ insts, const int2 *__restrict__ b2i,
                                                  int hofs) {
  constexpr int Q = L::Q, D = L::D;
  const Inst *Ip;
  int lblk;
  const Node nd = locate<L>(insts, b2i, Ip, lblk);
  const Inst &I = *Ip;
  if (lblk == 0 && threadIdx.x == 0) I.ctl->hcur ^= hofs;
  if (!nd.valid) return;
  const Phys<T> &P = phys<T>(I);
  const int N = I.N, n = nd.n, pc = 0;
  auto phi = gbl((const T *)I.phi[1]);
  auto mu = gbl((const T *)I.mu);
  T u[D], usq = 0;
#pragma unroll
  for (int d = 0; d < D; ++d) {
    u[d] = (gbl((const T *)I.u))[(size_t)d * N + n];
    usq += u[d] * u[d];
  }
  const T q = (gbl((const T *)I.q[1]))[n];
  T rho = 0;
  using IO = PopIO<S, T>;
  auto f = gbl((S *)I.f[pc]);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const T ph = phi[(size_t)i * N + n], m = mu[(size_t)i * N + n];
    rho += P.rho[i] * ph;
    T moved = 0;
#pragma unroll
    for (int j = 0; j < Q; ++j) {
      const T cu = ph * cdot<L>(j, u);
      const T feq = j == 0 ? ph - (T(1) - lw<L, T>(0)) * m : lw<L, T>(j) * m + lw<L, T>(j) * cu * T(3);
      if (IO::split && j == 0) continue;
      const S st = IO::cv(feq, T(SC_F));
      IO::put(f, (size_t)(i * Q + j) * N + n, st);
      moved += IO::back(st, T(SC_F));
    }
    if (IO::split) gbl(I.f0[pc])[(size_t)i * N + n] = (float)(ph - moved);
  }
  auto g = gbl((S *)I.g[pc]);
  auto l = gbl((S *)I.l[pc]);
#pragma unroll
  for (int j = 0; j < Q; ++j) {
    const T cu = cdot<L>(j, u);
    IO::put(g, (size_t)j * N + n, IO::cv(rho * lw<L, T>(j) * (cu * T(3) + cu * cu * T(4.5) - usq * T(1.5)), T(SC_G)));
    if (I.charge_model == 0) IO::put(l, (size_t)j * N + n, IO::cv(lw<L, T>(j) * q * (T(1) + cu * T(3)), T(SC_L)));
  }
  if (I.charge_model == 1) {
    // ion equilibria with the drift of the cold-start field
    const T Dn = (P.ion_tau - T(0.5)) / T(3);
    auto E = gbl((const T *)I.E);
    auto ion = gbl((const T *)I.ion);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const T z = k == 0 ? T(1) : T(-1), ns = ion[(size_t)k * N + n];
      T w[D];
#pragma unroll
      for (int d = 0; d < D; ++d) w[d] = u[d] + z * P.ion_beta * Dn * E[(size_t)d * N + n];
#pragma unroll
      for (int j = 0; j < Q; ++j)
        IO::put(l, (size_t)(k * Q + j) * N + n, IO::cv(lw<L, T>(j) * ns * (T(1) + cdot<L>(j, w) * T(3)), T(SC_L)));
    }
  }
  (gbl((T *)I.p))[n] = T(0);
  (gbl((T *)I.rho))[n] = rho;
  (gbl((T *)I.R))[n] = T(0);
}

// ------------------------------------------------------------ output / diag

// Copy (and convert) `nplanes` planes of element type Tin to Tout.
template <typename Tin, typename Tout>
__global__ __launch_bounds__(NT) void k_convert(const Tin *__restrict__ src, Tout *__restrict__ dst, size_t count) {
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  if (i < count) dst[i] = (Tout)src[i];
}

// Populations of the current level of instance `inst`, family fam (0 f,
// 1 g, 2 l, 3 h), as plain numbers [planes][N] of type Tout.
template <class L, typename T, typename S, typename Tout>
__global__ __launch_bounds__(NT) void k_export_pops(const Inst *__restrict__ insts, int inst, int fam, int pc,
                                                    Tout *__restrict__ dst) {
  constexpr int Q = L::Q;
  using IO = PopIO<S, T>;
  const Inst &I = insts[inst];
  const int n = blockIdx.x * NT + threadIdx.x;
  if (n >= I.nn) return;
  const size_t N = I.N, M = I.nn;  // plane stride of the state, of the dense output
  if (fam == 0) {
    const int fb = fbuf(I, pc);
    auto f = gbl((const S *)I.f[fb]);
    for (int j = 0; j < 3 * Q; ++j) {
      const T v = (IO::split && j % Q == 0) ? (T)gbl(I.f0[fb])[(j / Q) * N + n] : IO::ld(f, j * N + n, T(SC_F));
      dst[j * M + n] = (Tout)v;
    }
  } else if (fam == 3) {
    // stored deviation plus the reference potential's equilibrium
    auto h = gbl((const T *)I.h[I.ctl->hcur]);
    const T pr = psi_ref<T>(phys<T>(I), (n / I.nx) % I.ny);
    for (int j = 0; j < Q; ++j)
      dst[j * M + n] = (Tout)(h[j * N + n] + (j == 0 ? lw<L, T>(0) - T(1) : lw<L, T>(j)) * pr);
  } else {
    const S *p = (const S *)(fam == 1 ? I.g[pc] : I.l[pc]);
    const T sc = fam == 1 ? T(SC_G) : T(SC_L);
    const int nq = (fam == 2 && I.charge_model == 1) ? 2 * Q : Q;
    for (int j = 0; j < nq; ++j) dst[j * M + n] = (Tout)IO::ld(p, j * N + n, sc);
  }
}

// Indicator of a drop for the deformation moments: the order parameter with
// its far-field tail removed (weight 0 below 0.005, full weight from 0.02,
// cubic blend between).  Whole-box moments would weigh a 1e-5 background by
// (y - y_c)^2 ~ 1e5 and drown the drop's own shape.
__device__ __forceinline__ double drop_indicator(double w) {
  const double a = 0.005, b = 0.02;
  if (w <= a) return 0.0;
  if (w >= b) return w;
  const double s = (w - a) / (b - a);
  return w * s * s * (3.0 - 2.0 * s);
}

// Tangent parts of `count` dual values.
template <typename Tout>
__global__ __launch_bounds__(NT) void k_tangent(const DualD *__restrict__ src, Tout *__restrict__ dst, size_t count) {
  const size_t i = (size_t)blockIdx.x * NT + threadIdx.x;
  if (i < count) dst[i] = (Tout)src[i].d;
}

// Seeded directional derivative, first pass: per block, sum over the
// selected planes of seed * tangent (planes: pointers to [N] dual planes).
struct SeedPlanes {
  const DualD *plane[20];
  int count;
};
__global__ __launch_bounds__(NT) void k_seed_dot(const Inst *__restrict__ insts, SeedPlanes sp,
                                                 const double *__restrict__ seed) {
  const Inst &I = insts[0];
  const int n = blockIdx.x * NT + threadIdx.x;
  double v[1] = {0.0};
  if (n < I.nn)  // seed planes are dense ([count][nn])
    for (int k = 0; k < sp.count; ++k) v[0] += seed[(size_t)k * I.nn + n] * sp.plane[k][n].d;
  block_sum<1>(v);
  if (threadIdx.x == 0) I.part_p[(size_t)blockIdx.x * 2] = v[0];
}
__global__ __launch_bounds__(NT) void k_reduce_seed_dot(const Inst *__restrict__ insts) {
  const Inst &I = insts[0];
  double s = 0.0;
  for (int b = threadIdx.x; b < I.nblk; b += NT) s += I.part_p[(size_t)b * 2];
  double v[1] = {s};
  block_sum<1>(v);
  if (threadIdx.x == 0) I.ctl->diag[22] = v[0];
}

// Diagnostics, first pass: masses, charge, max |sum phi - 1|, non-finite
// populations, the raw second moments of the outer (1 - phi1) and inner
// (phi3) windowed indicators and the sums that locate each indicator's
// centroid (weights max(w, 0)), per block: DIAG_SUMS sums and the maximum.
constexpr int DIAG_SUMS = 23, DIAG_PART = DIAG_SUMS + 1;
//   part: where the per-block results go: null for the instance's own
//   partials in the workspace, else a buffer of DIAG_PART doubles per node
//   block of the handle (block blk0 + lblk of instance I).
template <class L, typename T, typename S>
__global__ __launch_bounds__(NT) void k_diag(const Inst *__restrict__ insts, const int2 *__restrict__ b2i, int pc,
                                             double *part = nullptr) {
  constexpr int Q = L::Q;
  const Inst *Ip;
  int lblk;
  const Node nd = locate<L>(insts, b2i, Ip, lblk);
  const Inst &I = *Ip;
  double v[DIAG_SUMS];
#pragma unroll
  for (int k = 0; k < DIAG_SUMS; ++k) v[k] = 0.0;
  double mx = 0.0;
  if (nd.valid) {
    const int N = I.N, n = nd.n;
    // pc: the next step's population buffer; the last step's fields are in pc ^ 1
    auto phi = gbl((const T *)I.phi[pc ^ 1]);
    const double p1 = (double)phi[n], p2 = (double)phi[(size_t)N + n], p3 = (double)phi[(size_t)2 * N + n];
    v[0] = p1;
    v[1] = p2;
    v[3] = (double)(gbl((const T *)I.q[pc ^ 1]))[n];
    v[2] = p3;
    mx = fabs(p1 + p2 + p3 - 1.0);
    using IO = PopIO<S, T>;
    int bad = 0;
    const int fb = fbuf(I, pc);
    auto f = gbl((const S *)I.f[fb]);
    for (int j = 0; j < 3 * Q; ++j) {
      const T v = (IO::split && j % Q == 0) ? (T)gbl(I.f0[fb])[(size_t)(j / Q) * N + n]
                                             : IO::ld(f, (size_t)j * N + n, T(SC_F));
      bad += !isfinite((double)v);
    }
    auto g = gbl((const S *)I.g[pc]);
    auto l = gbl((const S *)I.l[pc]);
    auto h = gbl((const T *)I.h[I.ctl->hcur]);
    for (int j = 0; j < Q; ++j) {
      bad += !isfinite((double)IO::ld(g, (size_t)j * N + n, T(SC_G)));
      bad += !isfinite((double)IO::ld(l, (size_t)j * N + n, T(SC_L)));
      bad += !isfinite((double)h[(size_t)j * N + n]);
    }
    if (I.charge_model == 1)
      for (int j = Q; j < 2 * Q; ++j) bad += !isfinite((double)IO::ld(l, (size_t)j * N + n, T(SC_L)));
    v[4] = bad;
    const double xx = nd.x, yy = nd.y;
    const double wo = drop_indicator(1.0 - p1), wi = drop_indicator(p3);
    v[5] = wo; v[6] = wo * xx; v[7] = wo * yy; v[8] = wo * xx * xx; v[9] = wo * yy * yy;
    v[10] = wi; v[11] = wi * xx; v[12] = wi * yy; v[13] = wi * xx * xx; v[14] = wi * yy * yy;
    const double zz = nd.z, co = fmax(1.0 - p1, 0.0), ci = fmax(p3, 0.0);
    v[15] = co; v[16] = co * xx; v[17] = co * yy; v[18] = co * zz;
    v[19] = ci; v[20] = ci * xx; v[21] = ci * yy; v[22] = ci * zz;
  }
  block_sum<DIAG_SUMS>(v);
  __shared__ double mred[NT / 64];
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_down(mx, o, 64));
  if ((threadIdx.x & 63) == 0) mred[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = mred[0];
    for (int i = 1; i < NT / 64; ++i) m = fmax(m, mred[i]);
    double *dst = (part ? part + (size_t)I.blk0 * DIAG_PART : I.part_d) + (size_t)lblk * DIAG_PART;
    for (int k = 0; k < DIAG_SUMS; ++k) dst[k] = v[k];
    dst[DIAG_SUMS] = m;
  }
}

// Diagnostics, second pass (one block per instance, fixed order): the
// outputs of lbm_ehd_diagnostics, including the residual of the last
// potential sub-iteration from k_mu's partials.
//   part: as for k_diag.
__global__ __launch_bounds__(NT) void k_reduce_diag(const Inst *__restrict__ insts, const double *part = nullptr) {
  const Inst &I = insts[blockIdx.x];
  Ctl *ctl = I.ctl;
  const double *pd = part ? part + (size_t)I.blk0 * DIAG_PART : I.part_d;
  double s[DIAG_PART];
  reduce_partials<DIAG_PART>(pd, I.nblk, s);  // (the maximum's slot is summed too, unused)
  double r[2];
  reduce_partials<2>(I.part_mu, I.nblk, r);
  // max over blocks of |sum phi - 1|
  double m = 0.0;
  for (int b = threadIdx.x; b < I.nblk; b += NT) m = fmax(m, pd[(size_t)b * DIAG_PART + DIAG_SUMS]);
  __shared__ double mred[NT / 64];
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
  if ((threadIdx.x & 63) == 0) mred[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x != 0) return;
  for (int i = 1; i < NT / 64; ++i) mred[0] = fmax(mred[0], mred[i]);
  double *out = ctl->diag;
  const double na = sqrt(r[1]);
  ctl->res_last = sqrt(r[0]) / (na > 1e-30 ? na : 1e-30);
  out[0] = s[0]; out[1] = s[1]; out[2] = s[2]; out[3] = s[3]; out[4] = mred[0];
  out[5] = ctl->res_last; out[6] = ctl->k_used; out[7] = s[4];
  for (int d = 0; d < 2; ++d) {
    const double w = s[5 + 5 * d], sx = s[6 + 5 * d], sy = s[7 + 5 * d];
    const double sxx = s[8 + 5 * d], syy = s[9 + 5 * d];
    double val = 0.0;
    if (w > 0) {
      const double ipar = syy / w - (sy / w) * (sy / w);  // along the field (y)
      const double iper = sxx / w - (sx / w) * (sx / w);  // across it (x)
      const double a = sqrt(ipar > 0 ? ipar : 0), b = sqrt(iper > 0 ? iper : 0);
      val = (a + b) > 0 ? (a - b) / (a + b) : 0.0;
    }
    out[10 + d] = val;
    // centroid of the indicator (weights max(w, 0)) for the contour pass
    const double c0 = s[15 + 4 * d];
    for (int a = 0; a < 3; ++a) out[16 + 3 * d + a] = c0 > 0 ? s[16 + 4 * d + a] / c0 : 0.0;
  }
}

// The Sec. 4.4 deformation factor D = (r_par - r_perp) / (r_par + r_perp)
// of the outer (w = 1 - phi1) and inner (w = phi3) drops, one block per
// instance, after k_reduce_diag.  The field is along y: r_par is half the
// distance between the two w = 1/2 crossings on the y line through the
// indicator's centroid, r_perp the same on the x line.  The lines fall
// between lattice nodes: w on them is interpolated linearly in each other
// axis (periodic wrap).  From the node s nearest the centroid (which must
// have w >= 1/2), the crossing in each direction lies between the last
// line node with w >= 1/2 and the next, found as the smallest offset k with
// w(s +- (k + 1)) < 1/2 (a minimum over the block's threads), and placed by
// linear interpolation.  A line that meets a wall first, or never drops
// below 1/2, gives nan.  Outputs diag[8..9] (D) and diag[12..15] (r_par,
// r_perp of the outer drop, then of the inner).
//   fb: the field buffer of the last step.
template <class L, typename T>
__global__ __launch_bounds__(NT) void k_contour(const Inst *__restrict__ insts, int fb) {
  const Inst &I = insts[blockIdx.x];
  double *out = I.ctl->diag;
  const int nx = I.nx, ny = I.ny, nz = L::D == 3 ? I.nz : 1;
  const T *phi = (const T *)I.phi[fb];
  __shared__ int kmin[NT / 64];
  const double nan = __builtin_nan("");
  for (int d = 0; d < 2; ++d) {
    const double cxyz[3] = {out[16 + 3 * d], out[17 + 3 * d], out[18 + 3 * d]};
    const T *pl = phi + (d == 0 ? 0 : (size_t)2 * I.N);
    auto w = [&](int x, int y, int z) -> double {
      const double p = (double)pl[((size_t)z * ny + y) * nx + x];
      return d == 0 ? 1.0 - p : p;
    };
    double r[2] = {nan, nan};
    const bool finite = isfinite(cxyz[0]) && isfinite(cxyz[1]) && isfinite(cxyz[2]);
    for (int axis = 1; axis >= 0 && finite; --axis) {  // the y line (along the field), then the x line
      // the interpolation corners in the other in-plane axis (and z)
      const int other = 1 - axis;
      const int nother = other == 0 ? nx : ny, nline = axis == 0 ? nx : ny;
      const double fo = floor(cxyz[other]), fz = floor(cxyz[2]);
      const int o0 = ((int)fo % nother + nother) % nother, o1 = (o0 + 1) % nother;
      const double ao = cxyz[other] - fo;
      const int z0 = L::D == 3 ? (((int)fz % nz) + nz) % nz : 0, z1 = L::D == 3 ? (z0 + 1) % nz : 0;
      const double az = L::D == 3 ? cxyz[2] - fz : 0.0;
      auto val = [&](int t) -> double {  // w on the line at line coordinate t (wrapped)
        const int tt = ((t % nline) + nline) % nline;
        auto at = [&](int o, int z) { return axis == 1 ? w(o, tt, z) : w(tt, o, z); };
        double v = (1.0 - ao) * at(o0, z0) + ao * at(o1, z0);
        if (L::D == 3) v = (1.0 - az) * v + az * ((1.0 - ao) * at(o0, z1) + ao * at(o1, z1));
        return v;
      };
      const bool bounded = axis == 1 && I.bc_y;
      const int s = (((int)floor(cxyz[axis] + 0.5)) % nline + nline) % nline;
      double ends[2];
      bool okk = val(s) >= 0.5;
      for (int dir = 0; dir < 2 && okk; ++dir) {
        const int step = dir == 0 ? 1 : -1;
        // offsets k = 0 .. kend-1 may be tested (the target s + step (k+1) stays off the wall)
        const int kend = bounded ? (step > 0 ? ny - 1 - s : s) : nline;
        int best = 0x7fffffff;
        for (int k = threadIdx.x; k < kend; k += NT)
          if (val(s + step * (k + 1)) < 0.5) best = k < best ? k : best;
        for (int o = 32; o > 0; o >>= 1) {
          const int b = __shfl_down(best, o, 64);
          best = b < best ? b : best;
        }
        if ((threadIdx.x & 63) == 0) kmin[threadIdx.x >> 6] = best;
        __syncthreads();
        best = kmin[0];
        for (int q = 1; q < NT / 64; ++q) best = kmin[q] < best ? kmin[q] : best;
        __syncthreads();
        if (best == 0x7fffffff) {
          okk = false;
          break;
        }
        const int i = s + step * best;
        const double a = val(i), b = val(i + step);
        ends[dir] = i + step * (a - 0.5) / (a - b);
      }
      r[axis == 1 ? 0 : 1] = okk ? 0.5 * (ends[0] - ends[1]) : nan;
    }
    if (threadIdx.x == 0) {
      out[8 + d] = (r[0] - r[1]) / (r[0] + r[1]);
      out[12 + 2 * d] = r[0];
      out[13 + 2 * d] = r[1];
    }
  }
}

}  // namespace lbm
