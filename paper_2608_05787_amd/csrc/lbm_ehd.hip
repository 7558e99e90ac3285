// Host runtime and C ABI of the three-phase EHD lattice Boltzmann step
// (declared in include/lbm_ehd.h).  The caller owns all device memory; this
// file carves the caller's workspace into planes, uploads the initial fields,
// and enqueues the kernels of lbm_ehd_kernels.h on the caller's stream.
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <type_traits>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "lbm_ehd.h"
#include "lbm_ehd_kernels.h"
#include "lbm_ehd_adjoint.h"
#include "lbm_ehd_persistent.h"

using namespace lbm;

namespace {

constexpr size_t ALIGN = 256;
size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

thread_local std::string g_create_error;

// Byte offsets of one instance inside the workspace.
struct Layout {
  size_t ctl, part_p, part_mu, part_d, planes, f[2], f0[2], g[2], l[2], h[2], end;
  int nblk;
};
// Macroscopic plane groups, each [k][nz][ny][nx] contiguous with plane
// stride N: phi(2 x 3) lsum eps q(2) R psi E(D) mu(3) u(D) p rho, and the ion
// concentrations (2, Nernst-Planck model only)
constexpr int N_GROUPS = 12;
int group_planes(int g, int D, int nion) {
  const int k[N_GROUPS] = {6, 1, 1, 2, 1, 1, D, 3, D, 1, 1, nion};
  return k[g];
}
int ion_planes(const lbm_ehd_params &p) { return p.charge_model == LBM_CHARGE_NERNST_PLANCK ? 2 : 0; }
int lat_q(const lbm_ehd_params &p) { return p.lattice == LBM_LATTICE_D3Q15 ? 15 : 9; }
int lat_d(const lbm_ehd_params &p) { return p.lattice == LBM_LATTICE_D3Q15 ? 3 : 2; }
int lat_nz(const lbm_ehd_params &p) { return p.nz > 1 ? p.nz : 1; }
size_t lat_nodes(const lbm_ehd_params &p) { return (size_t)p.nx * p.ny * lat_nz(p); }
// Plane stride: the node count rounded up to 64 nodes (planes 256-byte
// aligned) plus a skew of 27 x 64 nodes.  Without a skew some sizes put the
// ~36 planes a kernel streams at relative offsets that collide in the HBM
// address mapping (1020^2: collide 27% and moments 28% slower than at
// 1024^2 per node).  Swept over skews 0 - 151 and six sizes near 1M nodes,
// 27 is within 1% of the best step time on five and 2.5% off on 1020^2; it
// costs no traffic.
size_t plane_stride(const lbm_ehd_params &p) { return (lat_nodes(p) + 63) / 64 * 64 + 64 * 27; }

size_t elem_size(int prec) { return prec == LBM_PREC_TANGENT ? 16 : (prec == LBM_PREC_FP64 ? 8 : 4); }
size_t pop_size(int prec) {
  return prec == LBM_PREC_TANGENT ? 16 : prec == LBM_PREC_FP64 ? 8 : (prec == LBM_PREC_FP16S ? 2 : 4);
}

Layout layout_one(const lbm_ehd_params &p, size_t off) {
  Layout L;
  const size_t nodes = lat_nodes(p), N = plane_stride(p);
  const size_t Q = lat_q(p);
  const int D = lat_d(p);
  const size_t te = elem_size(p.precision), se = pop_size(p.precision);
  L.nblk = (int)((nodes + NT - 1) / NT);
  L.ctl = off;
  off = align_up(off + sizeof(Ctl));
  L.part_p = off;
  off = align_up(off + (size_t)L.nblk * 2 * sizeof(double));
  L.part_mu = off;
  off = align_up(off + (size_t)L.nblk * 2 * sizeof(double));
  L.part_d = off;
  off = align_up(off + (size_t)L.nblk * DIAG_PART * sizeof(double));
  L.planes = off;
  for (int g = 0; g < N_GROUPS; ++g) off += align_up(group_planes(g, D, ion_planes(p)) * N * te);
  const size_t nl = p.charge_model == LBM_CHARGE_NERNST_PLANCK ? 2 : 1;  // families in l
  for (int b = 0; b < 2; ++b) {
    L.f[b] = off;
    off = align_up(off + 3 * Q * N * se);
    L.f0[b] = off;
    if (p.precision == LBM_PREC_FP16S) off = align_up(off + 3 * N * sizeof(float));
    L.g[b] = off;
    off = align_up(off + Q * N * se);
    L.l[b] = off;
    off = align_up(off + nl * Q * N * se);
    L.h[b] = off;
    off = align_up(off + Q * N * te);
  }
  L.end = off;
  return L;
}

// Interior size of the LDS-tiled potential kernel's tile shapes: 0 the
// 64 x 16 tile with two sub-iterations, 1 the 64 x 32 tile with two, 2 the
// 64 x 32 tile with four.
constexpr int tile_cols(int s) { return s == 2 ? P2Shape<2, 4>::W : P2Shape<1>::W; }
constexpr int tile_rows(int s) { return s == 0 ? P2Shape<1>::H : s == 1 ? P2Shape<2>::H : P2Shape<2, 4>::H; }

struct Plan {
  size_t desc_off, b2i_off, b2i4_off, t2_off, bar_off, state_off, total;
  int total_blocks4;               // blocks of the four-nodes-per-thread moments kernel
  int total_blocks, total_tiles2;  // tiles of the default shape (64 x 16, two sub-iterations)
  int total_tiles2t;               // tiles of the tall (64 x 32) shape
  int total_tiles4;                // tiles of the tall shape with four sub-iterations per launch
  std::vector<Layout> lay;
};

Plan make_plan(const lbm_ehd_params *p, int n) {
  Plan P;
  P.desc_off = 0;
  size_t off = align_up((size_t)n * sizeof(Inst));
  P.total_blocks = 0;
  for (int i = 0; i < n; ++i) P.total_blocks += (int)(((size_t)p[i].nx * p[i].ny * lat_nz(p[i]) + NT - 1) / NT);
  // block and tile tables, each in two orders (XCD-grouped, linear)
  P.b2i_off = off;
  off = align_up(off + 2 * (size_t)P.total_blocks * sizeof(int2));
  P.total_blocks4 = 0;
  for (int i = 0; i < n; ++i) P.total_blocks4 += (int)(((size_t)p[i].nx * p[i].ny * lat_nz(p[i]) + M4 - 1) / M4);
  P.b2i4_off = off;
  off = align_up(off + (size_t)P.total_blocks4 * sizeof(int2));
  P.total_tiles2 = P.total_tiles2t = P.total_tiles4 = 0;
  // LDS-tiled potential tiles (D2Q9 planes only), all three shapes
  for (int i = 0; i < n; ++i)
    if (p[i].lattice == LBM_LATTICE_D2Q9)
      for (int s = 0; s < 3; ++s) {
        const int w = tile_cols(s), h = tile_rows(s);
        (s == 0 ? P.total_tiles2 : s == 1 ? P.total_tiles2t : P.total_tiles4) +=
            ((p[i].nx + w - 1) / w) * ((p[i].ny + h - 1) / h);
      }
  // tile tables: per shape (default, tall, tall four-iteration) the
  // XCD-grouped order, then the linear order
  P.t2_off = off;
  off = align_up(off + 2 * (size_t)(P.total_tiles2 + P.total_tiles2t + P.total_tiles4) * sizeof(int4));
  // persistent step: barrier words, then its launch arguments
  P.bar_off = off;
  off = align_up(off + align_up(PS_WORDS * sizeof(unsigned)) + sizeof(PersistArgs));
  P.state_off = off;
  for (int i = 0; i < n; ++i) {
    P.lay.push_back(layout_one(p[i], off));
    off = P.lay.back().end;
  }
  P.total = off;
  return P;
}

template <typename T> void fill_phys(Phys<T> &P, const lbm_ehd_params &p) {
  const double cs2 = 1.0 / 3.0;
  // spreading coefficients, Eq. (9)
  P.lam[0] = (T)(p.gamma12 + p.gamma13 - p.gamma23);
  P.lam[1] = (T)(p.gamma12 + p.gamma23 - p.gamma13);
  P.lam[2] = (T)(p.gamma13 + p.gamma23 - p.gamma12);
  P.m0 = (T)(cs2 * (p.tau_f - 0.5));
  P.tau_f = (T)p.tau_f;
  P.tau_l = (T)p.tau_l;
  P.eps_ref = (T)p.eps[p.eps_ref_phase];
  P.tau_h = (T)(0.5 + p.eps[p.eps_ref_phase] / cs2);
  P.D = (T)p.width;
  for (int i = 0; i < 3; ++i) {
    P.rho[i] = (T)p.rho[i];
    P.visc[i] = (T)p.visc[i];
    P.eps[i] = (T)p.eps[i];
    P.sig[i] = (T)p.sigma[i];
  }
  for (int s = 0; s < 2; ++s) {
    P.Eext[s] = (T)p.E_ext[s];
    P.wall_u[s] = (T)p.wall_u[s];
    P.wall_phi[s] = (T)p.wall_phi[s];
    P.wall_q[s] = (T)p.wall_q[s];
  }
  P.Eext[2] = (T)(p.lattice == LBM_LATTICE_D3Q15 ? p.E_ext_z : 0.0);
  // reference potential of the potential populations' storage: linear
  // between the electrodes (half-way walls at y = -1/2 and ny - 1/2)
  const bool walls = p.bc_y == LBM_BC_WALL;
  const double b = walls ? (p.wall_phi[1] - p.wall_phi[0]) / p.ny : 0.0;
  const double a = walls ? p.wall_phi[0] + 0.5 * b : 0.0;
  P.ref_a = (T)a;
  P.ref_b = (T)b;
  P.hwall[0] = (T)(p.wall_phi[0] - (a - 0.5 * b));
  P.hwall[1] = (T)(p.wall_phi[1] - (a + b * (p.ny - 0.5)));
  P.ion_tau = (T)p.ion_tau;
  P.ion_beta = (T)p.ion_beta;
  P.ion_e = (T)p.ion_charge;
}

// Applied-field magnitude E0 and the mean electrode potential about which
// the E0 direction scales the electric boundary data (see dtheta).
void applied_field(const lbm_ehd_params &p, double &E0, double &mean) {
  const bool walls = p.bc_y == LBM_BC_WALL;
  const double ey = walls ? (p.wall_phi[0] - p.wall_phi[1]) / p.ny : 0.0;
  const double ez = p.lattice == LBM_LATTICE_D3Q15 ? p.E_ext_z : 0.0;
  E0 = sqrt(p.E_ext[0] * p.E_ext[0] + (p.E_ext[1] + ey) * (p.E_ext[1] + ey) + ez * ez);
  mean = walls ? 0.5 * (p.wall_phi[0] + p.wall_phi[1]) : 0.0;
}

// Tangent-mode parameters: values of fill_phys<double> plus derivatives
// along dtheta (eps2/eps1, eps3/eps1, sigma2/sigma1, sigma3/sigma1, E0).
void fill_tangent(Phys<DualD> &T, const lbm_ehd_params &p) {
  Phys<double> v;
  fill_phys(v, p);
  auto cp = [](DualD *d, const double *s, int n) {
    for (int i = 0; i < n; ++i) d[i] = DualD(s[i], 0.0);
  };
  cp(T.lam, v.lam, 3);
  T.m0 = v.m0; T.tau_f = v.tau_f; T.tau_l = v.tau_l; T.tau_h = v.tau_h; T.eps_ref = v.eps_ref; T.D = v.D;
  cp(T.rho, v.rho, 3); cp(T.visc, v.visc, 3); cp(T.eps, v.eps, 3); cp(T.sig, v.sig, 3);
  cp(T.Eext, v.Eext, 3); cp(T.wall_u, v.wall_u, 2); cp(T.wall_phi, v.wall_phi, 2); cp(T.wall_q, v.wall_q, 2);
  T.ion_tau = v.ion_tau; T.ion_beta = v.ion_beta; T.ion_e = v.ion_e;
  T.ref_a = v.ref_a; T.ref_b = v.ref_b; cp(T.hwall, v.hwall, 2);  // the reference stays fixed
  T.eps[1].d = p.eps[0] * p.dtheta[0];
  T.eps[2].d = p.eps[0] * p.dtheta[1];
  T.sig[1].d = p.sigma[0] * p.dtheta[2];
  T.sig[2].d = p.sigma[0] * p.dtheta[3];
  double E0, mean;
  applied_field(p, E0, mean);
  if (E0 > 0) {
    const double s = p.dtheta[4] / E0;
    for (int k = 0; k < 2; ++k) {
      T.Eext[k].d = p.E_ext[k] * s;
      if (p.bc_y == LBM_BC_WALL) T.wall_phi[k].d = T.hwall[k].d = (p.wall_phi[k] - mean) * s;
    }
    T.Eext[2].d = v.Eext[2] * s;
  }
  // the reference permittivity (and tau_h) belongs to one phase: if that
  // phase's eps moves along dtheta, so does eps_ref
  T.eps_ref = T.eps[p.eps_ref_phase];
}

const char *validate(const lbm_ehd_params &p, const lbm_ehd_params &p0) {
  if (p.nx < 2 || p.ny < 2) return "nx and ny must be >= 2";
  if (p.lattice != LBM_LATTICE_D2Q9 && p.lattice != LBM_LATTICE_D3Q15) return "unknown lattice";
  if (p.nz < 0 || (p.lattice == LBM_LATTICE_D2Q9 && p.nz > 1)) return "nz must be 0 or 1 on D2Q9 (>= 1 on D3Q15)";
  if (p.lattice != p0.lattice) return "all instances of a handle must share the lattice";
  if ((long long)p.nx * p.ny * lat_nz(p) > (1ll << 30)) return "too many nodes in one instance";
  if (p.bc_y != LBM_BC_PERIODIC && p.bc_y != LBM_BC_WALL) return "bc_y must be LBM_BC_PERIODIC or LBM_BC_WALL";
  if (p.wall_q_mode != 0 && p.wall_q_mode != 1) return "wall_q_mode must be 0 or 1";
  if (p.eps_ref_phase < 0 || p.eps_ref_phase > 2) return "eps_ref_phase must be 0, 1 or 2";
  if (p.phase_mode != 0 && p.phase_mode != 1) return "phase_mode must be 0 or 1";
  if (!(p.tau_f > 0.5) || !(p.tau_l > 0.5)) return "tau_f and tau_l must exceed 1/2";
  if (!(p.width > 0)) return "width must be > 0";
  const double l1 = p.gamma12 + p.gamma13 - p.gamma23, l2 = p.gamma12 + p.gamma23 - p.gamma13,
               l3 = p.gamma13 + p.gamma23 - p.gamma12;
  if (!(l1 > 0) || !(l2 > 0) || !(l3 > 0)) return "spreading coefficients lambda_i (Eq. 9) must be > 0";
  for (int i = 0; i < 3; ++i) {
    if (!(p.rho[i] > 0)) return "densities must be > 0";
    if (!(p.visc[i] > 0)) return "viscosities must be > 0";
    if (!(p.eps[i] > 0)) return "permittivities must be > 0";
    if (!(p.sigma[i] >= 0)) return "conductivities must be >= 0";
  }
  if (p.sub_min < 1 || p.sub_max < p.sub_min || p.sub_max > 4096) return "need 1 <= sub_min <= sub_max <= 4096";
  if (p.init_sub_max < 0) return "init_sub_max must be >= 0";
  if (p.precision != LBM_PREC_FP32 && p.precision != LBM_PREC_FP64 && p.precision != LBM_PREC_FP16S &&
      p.precision != LBM_PREC_TANGENT)
    return "unknown precision";
  if (p.charge_model != LBM_CHARGE_LEAKY && p.charge_model != LBM_CHARGE_NERNST_PLANCK) return "unknown charge_model";
  if (p.sum_relax != 0 && p.sum_relax != 1) return "sum_relax must be 0 or 1";
  if (p.charge_model != p0.charge_model) return "all instances of a handle must share the charge model";
  if (p.charge_model == LBM_CHARGE_NERNST_PLANCK) {
    if (p.sigma[0] != 0 || p.sigma[1] != 0 || p.sigma[2] != 0)
      return "the Nernst-Planck charge model needs sigma = 0 (the ions carry the current)";
    if (p.wall_q_mode != 0) return "the Nernst-Planck charge model needs wall_q_mode 0 (no-flux walls)";
    if (!(p.ion_tau > 0.5)) return "ion_tau must exceed 1/2";
    if (p.precision == LBM_PREC_FP16S) return "the Nernst-Planck charge model does not support FP16S storage";
  }
  if (p.precision == LBM_PREC_TANGENT && p.eps_ref_phase != 0 && (p.dtheta[0] != 0 || p.dtheta[1] != 0))
    return "tangent mode along permittivity ratios needs eps_ref_phase 0 (tau_h must stay fixed)";
  if (p.precision != p0.precision || p.sub_min != p0.sub_min || p.sub_max != p0.sub_max ||
      p.sub_tol != p0.sub_tol || p.init_sub_max != p0.init_sub_max || p.init_tol != p0.init_tol)
    return "all instances of a handle must share precision and sub-iteration settings";
  return nullptr;
}

}  // namespace

struct lbm_ehd_s {
  int n_inst = 0, prec = 0, lattice = 0;
  int device = 0;  // the device current at create
  hipStream_t stream = nullptr;
  char *ws = nullptr;
  Plan plan;
  std::vector<lbm_ehd_params> params;
  std::vector<Inst> hinst;
  Inst *d_insts = nullptr;
  int2 *d_b2i = nullptr;  // block table in the order in use
  // block table of the four-nodes-per-thread moments kernel, linear order in
  // every configuration: consecutive blocks on different XCDs spread this
  // stencil-free stream over the memory channels (30.5 against 36.4 us at
  // 1024^2 FP32 with the XCD-grouped order)
  int2 *d_b2i4 = nullptr;
  bool vec_moments = false;  // D2Q9 leaky-dielectric steps run k_moments4
  int4 *d_t2 = nullptr;   // tile table of the two-sub-iteration launches, in use
  int4 *d_t4 = nullptr;   // tile table of the four-iteration form (tall tiles), in use
  // launch configuration (lbm_ehd_set_tuning): LBM_TUNE_* bits
  int tuning = 0;
  int persist_polls = 1 << 21;  // bound of a persistent-step barrier wait (polls of ~1 us)
  int persist_timed = 0;              // run the timed persistent kernel
  double persist_us[4] = {0, 0, 0, 0};  // last persistent call: us per step of each stage
  long long persist_steps = 0;
  int n_t2 = 0;           // tiles in d_t2
  bool pairs() const { return !(tuning & LBM_TUNE_SINGLE_POTENTIAL); }
  // the tall tile shape exists for FP32, FP16S and FP64 arithmetic (in FP64
  // its 147 KB of LDS leave one block per CU: slower than pairs, kept so the
  // benchmarked tile logic can be checked against the oracle to rounding)
  bool tall() const {
    return (tuning & LBM_TUNE_TALL_TILES) != 0 &&
           (prec == LBM_PREC_FP32 || prec == LBM_PREC_FP16S || prec == LBM_PREC_FP64);
  }
  // tile table of shape s (0: 64 x 16, two sub-iterations; 1: 64 x 32, two;
  // 2: 64 x 32, four) in the block order in use
  int4 *table(int s) const {
    const size_t lin = (tuning & LBM_TUNE_LINEAR_ORDER) ? 1 : 0;
    int4 *t = (int4 *)(ws + plan.t2_off);
    if (s == 0) return t + lin * plan.total_tiles2;
    t += 2 * (size_t)plan.total_tiles2;
    if (s == 1) return t + lin * plan.total_tiles2t;
    return t + 2 * (size_t)plan.total_tiles2t + lin * plan.total_tiles4;
  }
  void apply_order() {
    const int lin = (tuning & LBM_TUNE_LINEAR_ORDER) ? 1 : 0;
    d_b2i = (int2 *)(ws + plan.b2i_off) + (size_t)lin * plan.total_blocks;

    d_t4 = table(2);
    d_t2 = table(tall() ? 1 : 0);
    n_t2 = tall() ? plan.total_tiles2t : plan.total_tiles2;
  }
  int sub_min = 1, sub_max = 1, adaptive = 0;
  double sub_tol = 0;
  long long steps = 0;
  std::string err;
  // host copies of the initial fields (gradient runs restart from them)
  std::vector<std::vector<double>> init_phi, init_u, init_q, init_psi, init_ions;
  // recording made by lbm_ehd_record (checkpoints in the caller's buffer)
  void *rec_work = nullptr;
  int64_t rec_n = -1;
  int rec_every = 0;
  // kernel timing (lbm_ehd_profile_begin/end)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;  // kind of each recorded pair
  size_t ev_used = 0;

  // Bracket one launch with events when profiling; returns the stop event.
  hipEvent_t prof_start(int kind) {
    if (!prof) return nullptr;
    if (ev_used + 2 > ev_pool.size()) {
      for (int i = 0; i < 256; ++i) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        ev_pool.push_back(e);
      }
    }
    hipEvent_t a = ev_pool[ev_used], b = ev_pool[ev_used + 1];
    ev_used += 2;
    ev_kind.push_back(kind);
    (void)hipEventRecord(a, stream);
    return b;
  }
  void prof_stop(hipEvent_t b) {
    if (b) (void)hipEventRecord(b, stream);
  }
  // captured block of steps (lbm_ehd_graph)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int glen = 0, gpar = 0;
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    glen = 0;
  }
  ~lbm_ehd_s() {
    drop_graph();
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }

  int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }
};

#define HIPC(h, call)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return (h)->fail(LBM_EHD_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// Per-block partial sums of lbm_ehd_diagnostics_static, for callers that
// cannot allocate device memory: one array per GPU the library runs on,
// held until the process ends.  Host code never passes this name to a
// kernel or a copy: it uses the address hipGetSymbolAddress returns for the
// device (static_scratch).
constexpr int DIAG_STATIC_MAX_BLOCKS = 65536;  // node blocks of 256: 16.7 M nodes, 12 MiB
static __device__ __align__(256) double scratch[(size_t)DIAG_STATIC_MAX_BLOCKS * DIAG_PART];

namespace {

std::mutex g_scratch_mu;
std::vector<double *> g_scratch_dev;  // device address of `scratch`, per device (null: not yet known)

// Address of the static scratch array on the handle's device, looked up once
// per device with that device current.
int static_scratch(lbm_ehd_s *H, double **out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  const int dev = H->device;
  if (dev >= (int)g_scratch_dev.size()) g_scratch_dev.resize(dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    int cur = 0;
    HIPC(H, hipGetDevice(&cur));
    if (cur != dev) HIPC(H, hipSetDevice(dev));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) HIPC(H, hipSetDevice(cur));
    if (e != hipSuccess || !ptr)
      return H->fail(LBM_EHD_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[dev] = (double *)ptr;
  }
  *out = g_scratch_dev[dev];
  return LBM_EHD_OK;
}

// Fixed-count potential iterations 1..K: on D2Q9 planes one
// single-iteration launch first when K is odd, then LDS-tiled launches of
// four sub-iterations (tall tiles, 4-byte arithmetic) and of two; elsewhere
// (D3Q15 boxes, 16-byte tangent values that leave no room for the tile) one
// launch per iteration.  Returns the launch count
// (its parity is the buffer flip of the whole loop).
//   fb: the field buffer holding the charge (the step's; 1 at create).
//   pre: the first launch also forms the step's charge, source and
//   permittivity (fold_pre; k_pre is then not launched).
template <class Lat, typename T>
int enqueue_fixed_potential(lbm_ehd_s *H, int K, int fb, bool pre = false) {
  const dim3 grid(H->plan.total_blocks), grid2(H->n_t2), block(NT), block2(P2NT);
  int L = 0, k = 1;
  if constexpr (sizeof(T) <= 8 && std::is_same<Lat, D2Q9>::value) {
    if (H->pairs()) {
      if (K & 1) {
        hipEvent_t e = H->prof_start(2);
        k_poisson<Lat, T><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, 1, K, 0, 0, fb);
        H->prof_stop(e);
        L = 1;
        k = 2;
      }
      // tall tiles: four sub-iterations per launch while four remain
      if constexpr (sizeof(T) <= 8) {
        if (H->tall())
          for (; k + 3 <= K; k += 4, ++L) {
            const bool fold = pre && k == 1;
            hipEvent_t e = H->prof_start(fold ? 7 : 6);
            if (fold)
              k_poisson2<T, 2, 4, true><<<dim3(H->plan.total_tiles4), block2, 0, H->stream>>>(
                  H->d_insts, H->d_t4, L & 1, k + 3 == K ? 1 : 0, fb);
            else
              k_poisson2<T, 2, 4><<<dim3(H->plan.total_tiles4), block2, 0, H->stream>>>(H->d_insts, H->d_t4, L & 1,
                                                                                        k + 3 == K ? 1 : 0, fb);
            H->prof_stop(e);
          }
      }
      for (; k + 1 <= K; k += 2, ++L) {
        hipEvent_t e = H->prof_start(6);
        const int last = k + 1 == K ? 1 : 0;
        if constexpr (sizeof(T) <= 8) {
          if (H->tall())
            k_poisson2<T, 2><<<grid2, block2, 0, H->stream>>>(H->d_insts, H->d_t2, L & 1, last, fb);
          else
            k_poisson2<T, 1><<<grid2, block2, 0, H->stream>>>(H->d_insts, H->d_t2, L & 1, last, fb);
        } else {
          k_poisson2<T, 1><<<grid2, block2, 0, H->stream>>>(H->d_insts, H->d_t2, L & 1, last, fb);
        }
        H->prof_stop(e);
      }
      return L;
    }
  }
  for (; k <= K; ++k, ++L) {
    hipEvent_t e = H->prof_start(2);
    k_poisson<Lat, T><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, k, K, 0, L & 1, fb);
    H->prof_stop(e);
  }
  return L;
}

// Whether a step folds k_pre into its first potential launch: a fixed, even
// sub-iteration count K >= 4 on tall tiles, whose first launch is then a
// four-sub-iteration one (D2Q9, FP32/FP16S/FP64 arithmetic).
template <class Lat, typename T>
bool fold_pre(const lbm_ehd_s *H, int K, int adaptive) {
  if constexpr (std::is_same<Lat, D2Q9>::value && sizeof(T) <= 8)
    return !adaptive && H->pairs() && H->tall() && K >= 4 && !(K & 1);
  return false;
}

template <class Lat, typename T, typename S>
int do_create(lbm_ehd_s *H, const lbm_ehd_init *init) {
  const dim3 grid(H->plan.total_blocks), block(NT);
  const size_t te = sizeof(T);
  // upload initial fields (converted to T on the host)
  for (int i = 0; i < H->n_inst; ++i) {
    const Inst &I = H->hinst[i];
    const size_t N = (size_t)I.nn, stride = (size_t)I.N;  // nodes (dense host arrays), plane stride
    std::vector<T> buf(N);
    // planes of N dense host values into planes of the state's stride
    auto up = [&](const double *src, void *dst, size_t planes) -> int {
      for (size_t k = 0; k < planes; ++k) {
        for (size_t m = 0; m < N; ++m) buf[m] = src ? (T)src[k * N + m] : T(0);
        HIPC(H, hipMemcpyAsync((char *)dst + k * stride * te, buf.data(), N * te, hipMemcpyHostToDevice,
                               H->stream));
        HIPC(H, hipStreamSynchronize(H->stream));
      }
      return LBM_EHD_OK;
    };
    int rc;
    // create's fields live in field buffer 1 (the first step's previous level)
    if ((rc = up(init[i].phi0, I.phi[1], 3))) return rc;
    if ((rc = up(init[i].u0, I.u, (size_t)Lat::D))) return rc;
    if (H->params[i].charge_model == LBM_CHARGE_NERNST_PLANCK) {
      // ion concentrations and the charge they carry, q = e (n_+ - n_-)
      const double *c = init[i].ions0, e = H->params[i].ion_charge;
      if ((rc = up(c, I.ion, 2))) return rc;
      std::vector<double> q0(N);
      for (size_t k = 0; k < N; ++k) q0[k] = e * (c[k] - c[N + k]);
      if ((rc = up(q0.data(), I.q[1], 1))) return rc;
    } else if ((rc = up(init[i].q0, I.q[1], 1))) {
      return rc;
    }
    if constexpr (std::is_same<T, DualD>::value) {
      // the initial potential guess scales with the applied field about the
      // electrodes' mean potential, like the electrode data
      const lbm_ehd_params &p = H->params[i];
      double E0, mean;
      applied_field(p, E0, mean);
      const double sc = E0 > 0 ? p.dtheta[4] / E0 : 0.0;
      for (size_t k = 0; k < N; ++k) {
        const double v = init[i].psi0 ? init[i].psi0[k] : 0.0;
        buf[k] = DualD(v, (v - mean) * sc);
      }
      HIPC(H, hipMemcpyAsync(I.psi, buf.data(), N * te, hipMemcpyHostToDevice, H->stream));
      HIPC(H, hipStreamSynchronize(H->stream));
    } else {
      if ((rc = up(init[i].psi0, I.psi, 1))) return rc;
    }
  }
  k_init_potential<Lat, T><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i);
  HIPC(H, hipGetLastError());
  // cold start of the potential with the initial charge
  const lbm_ehd_params &p0 = H->params[0];
  const int kmax = p0.init_sub_max;
  const bool adaptive = p0.init_tol > 0 && kmax > 1;
  const int chunk = 256;
  int nlaunch = 0;
  if (!adaptive) {
    nlaunch = enqueue_fixed_potential<Lat, T>(H, kmax, 1);
    HIPC(H, hipGetLastError());
  }
  for (int k0 = 1; adaptive && k0 <= kmax; k0 += chunk) {
    const int k1 = std::min(kmax, k0 + chunk - 1);
    for (int k = k0; k <= k1; ++k) {
      k_poisson<Lat, T><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, k, kmax, 1, 0, 1);
      k_reduce_poisson<<<H->n_inst, block, 0, H->stream>>>(H->d_insts, k, 1, p0.init_tol);
    }
    HIPC(H, hipGetLastError());
    // stop launching once every instance has converged
    HIPC(H, hipStreamSynchronize(H->stream));
    bool all = true;
    for (int i = 0; i < H->n_inst && all; ++i) {
      int done = 0;
      HIPC(H, hipMemcpy(&done, &H->hinst[i].ctl->done, sizeof(int), hipMemcpyDeviceToHost));
      all = done != 0;
    }
    if (all) break;
  }
  const int hofs = adaptive ? 0 : (nlaunch & 1);
  k_mu<Lat, T><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, hofs, 1);
  k_init_pops<Lat, T, S><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, hofs);
  HIPC(H, hipGetLastError());
  HIPC(H, hipStreamSynchronize(H->stream));
  return LBM_EHD_OK;
}

template <class Lat, typename T, typename S>
int do_step(lbm_ehd_s *H, int64_t n) {
  const dim3 grid(H->plan.total_blocks), block(NT);
  const int K = H->sub_max, ad = H->adaptive;
  for (int64_t s = 0; s < n; ++s) {
    const int pc = (int)((H->steps + s) & 1);
    hipEvent_t e = H->prof_start(0);
    bool vec = false;
    if constexpr ((std::is_same<Lat, D2Q9>::value && sizeof(T) <= 8) || sizeof(T) == 4) {
      if (H->vec_moments) {
        // D3Q15 in FP32 and D2Q9 in FP64: two nodes per thread (four would need
        // 240 or 288 VGPRs of data)
        constexpr int W = (std::is_same<Lat, D3Q15>::value && std::is_same<S, float>::value) || sizeof(T) == 8 ? 2 : 4;
        k_moments4<Lat, T, S, W>
            <<<dim3(H->plan.total_blocks4 * (4 / W)), block, 0, H->stream>>>(H->d_insts, H->d_b2i4, pc);
        vec = true;
      }
    }
    if (!vec) k_moments<Lat, T, S><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, pc);
    H->prof_stop(e);
    const bool fold = fold_pre<Lat, T>(H, K, ad);
    if (!fold) {
      e = H->prof_start(1);
      k_pre<Lat, T><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, pc);
      H->prof_stop(e);
    }
    int hflip = 0;
    if (ad) {
      for (int k = 1; k <= K; ++k) {
        e = H->prof_start(2);
        k_poisson<Lat, T><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, k, K, 1, 0, pc);
        H->prof_stop(e);
        k_reduce_poisson<<<H->n_inst, block, 0, H->stream>>>(H->d_insts, k, H->sub_min, H->sub_tol, K);
      }
    } else {
      hflip = enqueue_fixed_potential<Lat, T>(H, K, pc, fold) & 1;
    }
    e = H->prof_start(3);
    k_mu<Lat, T><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, hflip, pc);
    H->prof_stop(e);
    e = H->prof_start(4);
    if (sizeof(T) <= 4 && !(H->tuning & LBM_TUNE_COLLIDE_PER_FAMILY))
      k_collide<Lat, T, S, true><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, pc, s == n - 1 ? 1 : 0,
                                                                ad ? 0 : K, hflip);
    else
      k_collide<Lat, T, S, false><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, pc, s == n - 1 ? 1 : 0,
                                                                 ad ? 0 : K, hflip);
    H->prof_stop(e);
    HIPC(H, hipGetLastError());
  }
  H->steps += n;
  return LBM_EHD_OK;
}

//   part: null (the instances' partials in the workspace) or a buffer of
//   DIAG_PART doubles per node block of the handle.
template <class Lat, typename T, typename S>
int do_diag(lbm_ehd_s *H, double *part) {
  const dim3 grid(H->plan.total_blocks), block(NT);
  hipEvent_t e = H->prof_start(5);
  k_diag<Lat, T, S><<<grid, block, 0, H->stream>>>(H->d_insts, H->d_b2i, (int)(H->steps & 1), part);
  k_reduce_diag<<<H->n_inst, block, 0, H->stream>>>(H->d_insts, part);
  k_contour<Lat, T><<<H->n_inst, block, 0, H->stream>>>(H->d_insts, (int)((H->steps + 1) & 1));
  H->prof_stop(e);
  HIPC(H, hipGetLastError());
  return LBM_EHD_OK;
}

template <typename Tin>
int convert(lbm_ehd_s *H, const void *src, void *dst, size_t count, int dtype) {
  const dim3 grid((unsigned)((count + NT - 1) / NT)), block(NT);
  if (count == 0) return LBM_EHD_OK;
  if (dtype == LBM_DTYPE_F32)
    k_convert<Tin, float><<<grid, block, 0, H->stream>>>((const Tin *)src, (float *)dst, count);
  else
    k_convert<Tin, double><<<grid, block, 0, H->stream>>>((const Tin *)src, (double *)dst, count);
  HIPC(H, hipGetLastError());
  return LBM_EHD_OK;
}

int convert_any(lbm_ehd_s *H, int elem, const void *src, void *dst, size_t count, int dtype) {
  if (dtype == LBM_DTYPE_TANGENT_F64) {
    if (elem != 16) return H->fail(LBM_EHD_EINVAL, "tangent fields exist only in tangent mode");
    if (count == 0) return LBM_EHD_OK;
    k_tangent<double><<<dim3((unsigned)((count + NT - 1) / NT)), dim3(NT), 0, H->stream>>>((const DualD *)src,
                                                                                      (double *)dst, count);
    HIPC(H, hipGetLastError());
    return LBM_EHD_OK;
  }
  if (elem == 16) return convert<DualD>(H, src, dst, count, dtype);
  if (elem == 8) return convert<double>(H, src, dst, count, dtype);
  if (elem == 4) return convert<float>(H, src, dst, count, dtype);
  return convert<__half>(H, src, dst, count, dtype);
}

// Runs F::template run<Lattice, T, S>(args...) for the handle's lattice and
// precision.
template <class F, class... A> int dispatch(const lbm_ehd_s *H, A &&...a) {
  if (H->lattice == LBM_LATTICE_D3Q15) {
    if (H->prec == LBM_PREC_FP64) return F::template run<D3Q15, double, double>(a...);
    if (H->prec == LBM_PREC_TANGENT) return F::template run<D3Q15, DualD, DualD>(a...);
    if (H->prec == LBM_PREC_FP16S) return F::template run<D3Q15, float, __half>(a...);
    return F::template run<D3Q15, float, float>(a...);
  }
  if (H->prec == LBM_PREC_FP64) return F::template run<D2Q9, double, double>(a...);
  if (H->prec == LBM_PREC_TANGENT) return F::template run<D2Q9, DualD, DualD>(a...);
  if (H->prec == LBM_PREC_FP16S) return F::template run<D2Q9, float, __half>(a...);
  return F::template run<D2Q9, float, float>(a...);
}
struct CreateF {
  template <class L, typename T, typename S> static int run(lbm_ehd_s *H, const lbm_ehd_init *i) {
    return do_create<L, T, S>(H, i);
  }
};
struct StepF {
  template <class L, typename T, typename S> static int run(lbm_ehd_s *H, int64_t n) { return do_step<L, T, S>(H, n); }
};
struct DiagF {
  template <class L, typename T, typename S> static int run(lbm_ehd_s *H, double *part) {
    return do_diag<L, T, S>(H, part);
  }
};
struct ExportF {
  template <class L, typename T, typename S>
  static int run(lbm_ehd_s *H, dim3 grid, dim3 block, int inst, int family, int pc, void *dst, int dtype) {
    if (dtype == LBM_DTYPE_F64)
      k_export_pops<L, T, S, double><<<grid, block, 0, H->stream>>>(H->d_insts, inst, family, pc, (double *)dst);
    else
      k_export_pops<L, T, S, float><<<grid, block, 0, H->stream>>>(H->d_insts, inst, family, pc, (float *)dst);
    return 0;
  }
};

}  // namespace

// Creates a handle over the caller's workspace.  run_init: upload the
// initial fields and run the cold start; otherwise the state is left zeroed
// (a shell whose state a later restore provides).
static int create_impl(const lbm_ehd_params *params, int32_t n_inst, const lbm_ehd_init *init,
                       void *dev_workspace, void *hip_stream, lbm_ehd_t *out, bool run_init) {
  g_create_error.clear();
  if (!out) return LBM_EHD_EINVAL;
  *out = nullptr;
  if (!params || (run_init && !init) || n_inst < 1) {
    g_create_error = "params, init and n_inst >= 1 are required";
    return LBM_EHD_EINVAL;
  }
  for (int i = 0; i < n_inst; ++i) {
    if (const char *m = validate(params[i], params[0])) {
      char buf[256];
      snprintf(buf, sizeof buf, "instance %d: %s", i, m);
      g_create_error = buf;
      return LBM_EHD_EINVAL;
    }
    if (run_init && !init[i].phi0) {
      g_create_error = "init.phi0 is required";
      return LBM_EHD_EINVAL;
    }
    if (run_init && params[i].charge_model == LBM_CHARGE_NERNST_PLANCK && !init[i].ions0) {
      g_create_error = "init.ions0 is required under the Nernst-Planck charge model";
      return LBM_EHD_EINVAL;
    }
  }
  if (!dev_workspace || ((uintptr_t)dev_workspace % ALIGN) != 0) {
    g_create_error = "workspace must be non-NULL and 256-byte aligned";
    return LBM_EHD_ENOMEM;
  }
  lbm_ehd_s *H = new lbm_ehd_s();
  if (hipGetDevice(&H->device) != hipSuccess) {
    delete H;
    g_create_error = "hipGetDevice failed";
    return LBM_EHD_EHIP;
  }
  H->n_inst = n_inst;
  H->prec = params[0].precision;
  H->lattice = params[0].lattice;
  // the vector moments kernel serves leaky-dielectric handles: D2Q9 in FP32,
  // FP16S and FP64, D3Q15 in FP32 and FP16S (60 vectors of doubles would spill)
  H->vec_moments = H->prec != LBM_PREC_TANGENT &&
                   (H->lattice == LBM_LATTICE_D2Q9 || H->prec != LBM_PREC_FP64);
  for (int i = 0; i < n_inst; ++i)
    if (params[i].charge_model != LBM_CHARGE_LEAKY) H->vec_moments = false;
  H->stream = (hipStream_t)hip_stream;
  H->ws = (char *)dev_workspace;
  H->params.assign(params, params + n_inst);
  H->plan = make_plan(params, n_inst);
  H->sub_min = params[0].sub_min;
  H->sub_max = params[0].sub_max;
  H->sub_tol = params[0].sub_tol;
  H->adaptive = (H->sub_tol > 0 && H->sub_max > H->sub_min) ? 1 : 0;
  H->d_insts = (Inst *)(H->ws + H->plan.desc_off);
  H->d_b2i4 = (int2 *)(H->ws + H->plan.b2i4_off);
  H->apply_order();

  const size_t te = elem_size(H->prec);
  // logical block order: instances one after another, blocks in row order
  std::vector<int2> logical, logical4;
  for (int i = 0; i < n_inst; ++i) {
    const lbm_ehd_params &p = params[i];
    const Layout &L = H->plan.lay[i];
    Inst I{};
    I.nx = p.nx;
    I.ny = p.ny;
    I.nz = lat_nz(p);
    I.nn = (int)lat_nodes(p);
    I.N = (int)plane_stride(p);
    I.bc_y = p.bc_y;
    I.wall_q_mode = p.wall_q_mode;
    I.phase_mode = p.phase_mode;
    I.charge_model = p.charge_model;
    I.sum_relax = p.sum_relax;
    I.nblk = L.nblk;
    I.blk0 = (int)logical.size();  // node blocks of the instances before this one
    for (int b = 0; b < 2; ++b) {
      I.f[b] = H->ws + L.f[b];
      I.f0[b] = p.precision == LBM_PREC_FP16S ? (float *)(H->ws + L.f0[b]) : nullptr;
      I.g[b] = H->ws + L.g[b];
      I.l[b] = H->ws + L.l[b];
      I.h[b] = H->ws + L.h[b];
    }
    char *base = H->ws + L.planes;
    void **group[N_GROUPS] = {&I.phi[0], &I.lsum, &I.eps, &I.q[0], &I.R, &I.psi, &I.E,
                              &I.mu, &I.u, &I.p, &I.rho, &I.ion};
    for (int g = 0; g < N_GROUPS; ++g) {
      *group[g] = base;
      base += align_up(group_planes(g, lat_d(p), ion_planes(p)) * (size_t)I.N * te);
    }
    I.phi[1] = (char *)I.phi[0] + 3 * (size_t)I.N * te;
    I.q[1] = (char *)I.q[0] + (size_t)I.N * te;
    if (!ion_planes(p)) I.ion = nullptr;
    I.part_p = (double *)(H->ws + L.part_p);
    I.part_mu = (double *)(H->ws + L.part_mu);
    I.part_d = (double *)(H->ws + L.part_d);
    I.ctl = (Ctl *)(H->ws + L.ctl);
    fill_phys(I.pf, p);
    fill_phys(I.pd, p);
    fill_tangent(I.pt, p);
    H->hinst.push_back(I);
    for (int b = 0; b < L.nblk; ++b) logical.push_back(make_int2(i, b));
    for (int b = 0; b < (I.nn + M4 - 1) / M4; ++b) logical4.push_back(make_int2(i, b));
  }
  // XCD-aware order: launched block b runs on XCD b % 8; give XCD x the
  // contiguous logical range [off(x), off(x) + count(x)).
  auto xcd_order = [](int B, int b) {
    const int q8 = B / 8, r8 = B % 8, x = b % 8, i = b / 8;
    return x * q8 + std::min(x, r8) + i;
  };
  const int B = (int)logical.size();
  std::vector<int2> b2i(2 * (size_t)B);  // XCD-grouped order, then linear order
  for (int b = 0; b < B; ++b) {
    b2i[b] = logical[xcd_order(B, b)];
    b2i[B + b] = logical[b];
  }
  const std::vector<int2> &b2i4 = logical4;
  // tiles of the LDS-tiled potential kernel, rows of tiles in order
  std::vector<int4> t2;  // per shape: XCD-grouped order, then linear order
  for (int shape = 0; shape < 3; ++shape) {
    const int rows = tile_rows(shape), cols = tile_cols(shape);
    std::vector<int4> tl;
    for (int i = 0; i < n_inst; ++i)
      if (params[i].lattice == LBM_LATTICE_D2Q9)
        for (int y0 = 0; y0 < params[i].ny; y0 += rows)
          for (int x0 = 0; x0 < params[i].nx; x0 += cols) tl.push_back(make_int4(i, x0, y0, 0));
    const int T2 = (int)tl.size();
    for (int b = 0; b < T2; ++b) t2.push_back(tl[xcd_order(T2, b)]);
    t2.insert(t2.end(), tl.begin(), tl.end());
  }
  int rc = LBM_EHD_OK;
  auto bad = [&](int code) {
    g_create_error = H->err;
    delete H;
    return code;
  };
  hipError_t e;
  if ((e = hipMemsetAsync(H->ws + H->plan.state_off, 0, H->plan.total - H->plan.state_off, H->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(H->d_insts, H->hinst.data(), sizeof(Inst) * n_inst, hipMemcpyHostToDevice, H->stream)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(H->ws + H->plan.b2i_off, b2i.data(), sizeof(int2) * b2i.size(), hipMemcpyHostToDevice,
                          H->stream)) != hipSuccess ||
      (e = hipMemcpyAsync(H->ws + H->plan.b2i4_off, b2i4.data(), sizeof(int2) * b2i4.size(), hipMemcpyHostToDevice,
                          H->stream)) !=
          hipSuccess ||
      (e = hipMemcpyAsync(H->ws + H->plan.t2_off, t2.data(), sizeof(int4) * t2.size(), hipMemcpyHostToDevice,
                          H->stream)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(H->stream)) != hipSuccess) {
    H->err = std::string("workspace setup: ") + hipGetErrorString(e);
    return bad(LBM_EHD_EHIP);
  }
  if (!run_init) {
    *out = H;
    return LBM_EHD_OK;
  }
  for (int i = 0; i < n_inst; ++i) {
    const size_t N = (size_t)params[i].nx * params[i].ny * lat_nz(params[i]);
    auto keep = [&](std::vector<std::vector<double>> &dst, const double *src, size_t cnt) {
      dst.emplace_back(src ? std::vector<double>(src, src + cnt) : std::vector<double>());
    };
    keep(H->init_phi, init[i].phi0, 3 * N);
    keep(H->init_u, init[i].u0, (size_t)lat_d(params[i]) * N);
    keep(H->init_q, init[i].q0, N);
    keep(H->init_psi, init[i].psi0, N);
    keep(H->init_ions, params[i].charge_model == LBM_CHARGE_NERNST_PLANCK ? init[i].ions0 : nullptr, 2 * N);
  }
  rc = dispatch<CreateF>(H, H, init);
  if (rc) return bad(rc);
  *out = H;
  return LBM_EHD_OK;
}


// ------------------------------------------------------------ reverse mode

namespace {

constexpr int REC_FIXED = 22;    // planes of a step record before the potential levels
constexpr int ADJ_AREA = 176;    // planes of the adjoint buffers (see rev_bufs)

// Layout of the buffer shared by lbm_ehd_record and lbm_ehd_adjoint (byte
// offsets from its start, 256-byte aligned): a private handle's workspace,
// the checkpoints (one per segment of `every` steps), the step records of
// one segment (reused for the cold start's potential levels), the adjoint
// buffers, the per-block parameter partials and the cold start's chunk
// checkpoints.
struct AdjLayout {
  size_t shell, ckpt, ckpt_stride, seg, slot_stride, adj, tb, out, cold_ck, total;
  int64_t rev;     // steps whose adjoint runs in full (the last step's is its seed)
  int nseg, nck, slots, rec_planes, cold_len, cold_chunks, tb_slots;
};

AdjLayout adj_layout(const lbm_ehd_s *H, int64_t n_steps, int every) {
  AdjLayout L{};
  const lbm_ehd_params &p = H->params[0];
  const size_t N = plane_stride(p), te = elem_size(H->prec);
  L.rev = n_steps > 1 ? n_steps - 1 : 0;
  L.nseg = (int)((L.rev + every - 1) / every);
  L.nck = L.nseg > 0 ? L.nseg : 1;
  L.slots = (int)std::min<int64_t>(every, L.rev > 0 ? L.rev : 1);
  L.rec_planes = REC_FIXED + 9 * H->sub_max;
  size_t off = 0;
  L.shell = off;
  off = align_up(off + H->plan.total);
  L.ckpt = off;
  L.ckpt_stride = align_up(H->plan.total - H->plan.state_off);
  off = align_up(off + (size_t)L.nck * L.ckpt_stride);
  L.seg = off;
  L.slot_stride = align_up((size_t)L.rec_planes * N * te);
  off = align_up(off + (size_t)L.slots * L.slot_stride);
  L.adj = off;
  off = align_up(off + (size_t)ADJ_AREA * N * te);
  L.tb = off;
  L.tb_slots = std::max(H->hinst[0].nblk, H->plan.total_tiles2);
  off = align_up(off + (size_t)L.tb_slots * TB_SLOTS * sizeof(double));
  L.out = off;
  off = align_up(off + TB_SLOTS * sizeof(double));
  L.cold_len = std::max(1, (int)(((size_t)L.slots * L.slot_stride) / (9 * N * te)));
  L.cold_chunks = p.init_sub_max > 0 ? (p.init_sub_max + L.cold_len - 1) / L.cold_len : 0;
  L.cold_ck = off;
  off = align_up(off + (size_t)L.cold_chunks * 9 * N * te);
  L.total = off;
  return L;
}

const char *adjoint_unsupported(const lbm_ehd_s *H) {
  if (H->n_inst != 1) return "gradients need a single-instance handle";
  if (H->lattice != LBM_LATTICE_D2Q9) return "reverse mode is built for D2Q9 (forward mode covers D3Q15)";
  if (H->prec != LBM_PREC_FP32 && H->prec != LBM_PREC_FP64) return "reverse mode needs FP32 or FP64 precision";
  if (H->adaptive) return "reverse mode needs a fixed number of potential sub-iterations";
  const lbm_ehd_params &p = H->params[0];
  if (p.init_tol > 0 && p.init_sub_max > 1) return "reverse mode needs a fixed-count cold start (init_tol <= 0)";
  if (p.eps_ref_phase != 0) return "gradients along permittivity ratios need eps_ref_phase 0";
  if (p.charge_model != LBM_CHARGE_LEAKY) return "reverse mode is built for the leaky-dielectric charge model";
  return nullptr;
}

// Pointers of one step record: phi 3, q, R, eps, E_prev 2, mu 3, E 2, g 9,
// then the input level of each potential sub-iteration (9 planes each).
template <typename T> Rec<T> rec_slot(char *slot, size_t N) {
  T *b = (T *)slot;
  Rec<T> r;
  r.phi = b;
  r.q = b + 3 * N;
  r.R = b + 4 * N;
  r.eps = b + 5 * N;
  r.Eo = b + 6 * N;
  r.mu = b + 8 * N;
  r.En = b + 11 * N;
  r.g = b + 13 * N;
  return r;
}
template <typename T> T *rec_level(char *slot, size_t N, int k) { return (T *)slot + (REC_FIXED + 9 * (size_t)k) * N; }

// One forward step that also writes its record: the launches of an
// ordinary fixed-count step in the handle's launch configuration, the
// potential kernels storing the input level of every sub-iteration.
template <typename T>
void step_record(lbm_ehd_s *W, char *slot) {
  const dim3 grid(W->plan.total_blocks), block(NT), block2(P2NT);
  const size_t N = (size_t)W->hinst[0].N;
  const int K = W->sub_max, pc = (int)(W->steps & 1);
  const Rec<T> rc = rec_slot<T>(slot, N);
  constexpr int MW = sizeof(T) == 8 ? 2 : 4;  // nodes per thread, as in the plain step
  if (W->vec_moments)
    k_moments4<D2Q9, T, T, MW>
        <<<dim3(W->plan.total_blocks4 * (4 / MW)), block, 0, W->stream>>>(W->d_insts, W->d_b2i4, pc, rc);
  else
    k_moments<D2Q9, T, T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, pc, rc);
  // the charge step rides on the first four-sub-iteration launch where the
  // plain step folds it (same arithmetic, same record)
  const bool fold = sizeof(T) <= 8 && W->tall() && K >= 4 && !(K & 1);
  if (!fold) k_pre<D2Q9, T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, pc, rc);
  int L = 0, k = 1;
  if (K & 1) {
    k_poisson<D2Q9, T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, 1, K, 0, 0, pc, rec_level<T>(slot, N, 0));
    L = 1;
    k = 2;
  }
  auto lev = [&](int i) { return rec_level<T>(slot, N, i); };
  if constexpr (sizeof(T) <= 8) {
    if (W->tall()) {
      // four sub-iterations per launch while four remain, then tall pairs
      for (; k + 3 <= K; k += 4, ++L) {
        P2Rec<T, 4> pr{{lev(k - 1), lev(k), lev(k + 1), lev(k + 2)}};
        if (fold && k == 1) {
          pr.q = rc.q;
          pr.R = rc.R;
          pr.eps = rc.eps;
          pr.Eo = rc.Eo;
          k_poisson2<T, 2, 4, true><<<dim3(W->plan.total_tiles4), block2, 0, W->stream>>>(
              W->d_insts, W->table(2), L & 1, k + 3 == K ? 1 : 0, pc, pr);
        } else {
          k_poisson2<T, 2, 4><<<dim3(W->plan.total_tiles4), block2, 0, W->stream>>>(
              W->d_insts, W->table(2), L & 1, k + 3 == K ? 1 : 0, pc, pr);
        }
      }
      for (; k + 1 <= K; k += 2, ++L)
        k_poisson2<T, 2><<<dim3(W->plan.total_tiles2t), block2, 0, W->stream>>>(
            W->d_insts, W->table(1), L & 1, k + 1 == K ? 1 : 0, pc, P2Rec<T, 2>{{lev(k - 1), lev(k)}});
    }
  }
  for (; k + 1 <= K; k += 2, ++L)
    k_poisson2<T><<<dim3(W->plan.total_tiles2), block2, 0, W->stream>>>(
        W->d_insts, W->table(0), L & 1, k + 1 == K ? 1 : 0, pc, P2Rec<T, 2>{{lev(k - 1), lev(k)}});
  const int hflip = L & 1;
  k_mu<D2Q9, T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, hflip, pc, rc);
  if (sizeof(T) <= 4 && (W->tuning & LBM_TUNE_COLLIDE_PER_FAMILY))
    k_collide<D2Q9, T, T, false><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, pc, 0, K, hflip, rc);
  else
    k_collide<D2Q9, T, T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, pc, 0, K, hflip, rc);
  W->steps += 1;
}

// Adjoint of one recorded step: a[cur], pb[cur], hb[hs] hold the adjoint of
// the next level on entry; on return cur and hs name this level's.
template <typename T>
void step_adjoint(lbm_ehd_s *W, char *slot, const AdjBufs<T> &ab, int &cur, int &hs) {
  const dim3 grid(W->plan.total_blocks), block(NT);
  const size_t N = (size_t)W->hinst[0].N;
  const int K = W->sub_max;
  const Rec<T> rc = rec_slot<T>(slot, N);
  k_adj_collide<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, rc, ab, cur);
  k_adj_mu<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, rc, ab, cur, hs, 1);
  // sub-iterations K, K-1, ... on LDS tiles: in fours on the tall tiles
  // (in that launch configuration), then in pairs, a single one last when K
  // is odd
  int k = K;
  if constexpr (sizeof(T) <= 8)
    if (W->tall())
      for (; k >= 4; k -= 4) {
        k_adj_poisson4<T><<<dim3(W->plan.total_tiles4), dim3(P2NT), 0, W->stream>>>(
            W->d_insts, W->table(2), rec_level<T>(slot, N, k - 4), rec_level<T>(slot, N, k - 3),
            rec_level<T>(slot, N, k - 2), rec_level<T>(slot, N, k - 1), rc.eps, ab, hs, ab.qb);
        hs ^= 1;
      }
  for (; k >= 2; k -= 2) {
    k_adj_poisson2<T><<<dim3(W->plan.total_tiles2), dim3(P2NT), 0, W->stream>>>(
        W->d_insts, W->table(0), rec_level<T>(slot, N, k - 1), rec_level<T>(slot, N, k - 2), rc.eps, ab, hs, ab.qb);
    hs ^= 1;
  }
  if (k == 1) {
    k_adj_poisson<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, rec_level<T>(slot, N, 0), rc.eps, ab, hs,
                                                    ab.qb);
    hs ^= 1;
  }
  k_adj_pre<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, rc, ab, cur);
  cur ^= 1;
}

// Steps handle R from its create state through n_steps, writing a
// checkpoint at the start of every segment of `every` steps.
int record_run(lbm_ehd_s *R, char *work, const AdjLayout &L, int64_t n_steps, int every) {
  int64_t t = 0;
  int ck = 0;
  for (;;) {
    if (ck < L.nck && t == (int64_t)ck * every) {
      const int rc = lbm_ehd_checkpoint(R, work + L.ckpt + (size_t)ck * L.ckpt_stride);
      if (rc) return rc;
      ++ck;
    }
    if (t >= n_steps) break;
    const int64_t next = std::min<int64_t>(n_steps, (t / every + 1) * every);
    const int rc = lbm_ehd_step(R, next - t);
    if (rc) return rc;
    t = next;
  }
  return LBM_EHD_OK;
}

// The reverse sweep over a recording: segments last to first (restore the
// segment's checkpoint into W, re-run it writing step records, then the
// step adjoints last to first), then the adjoint of create (equilibrium
// populations, field and chemical potential, the cold-start potential
// iterations in recomputed chunks, the initial potential guess).
template <typename T>
int reverse_sweep(lbm_ehd_s *H, lbm_ehd_s *W, char *work, const AdjLayout &L, int64_t n_steps, int every,
                  const double *seed, uint32_t mask, double grad[5]) {
  const dim3 grid(W->plan.total_blocks), block(NT);
  const Inst &I = W->hinst[0];
  const size_t N = (size_t)I.N;
  const lbm_ehd_params &p = W->params[0];
  T *base = (T *)(work + L.adj);
  AdjBufs<T> ab;
  ab.a[0] = base;
  ab.a[1] = base + 55 * N;
  ab.hb[0] = base + 110 * N;
  ab.hb[1] = base + 119 * N;
  ab.pb[0] = base + 128 * N;
  ab.pb[1] = base + 132 * N;
  ab.muL = base + 136 * N;
  ab.gm = base + 139 * N;
  ab.gr = base + 145 * N;
  ab.qb = base + 147 * N;
  ab.rb = base + 148 * N;
  ab.en = base + 149 * N;
  ab.eb = base + 151 * N;
  ab.lb = base + 152 * N;
  ab.gS = base + 155 * N;
  T *psi0 = base + 157 * N;
  T *cold[2] = {base + 158 * N, base + 167 * N};
  ab.tb = (double *)(work + L.tb);
  double E0, mean;
  applied_field(p, E0, mean);
  const double inv_e0 = E0 > 0 ? 1.0 / E0 : 0.0;
  const bool walls = p.bc_y == LBM_BC_WALL;
  for (int k = 0; k < 2; ++k) {
    ab.dEext[k] = p.E_ext[k] * inv_e0;
    ab.dwall[k] = walls ? (p.wall_phi[k] - mean) * inv_e0 : 0.0;
  }
  HIPC(H, hipMemsetAsync(base, 0, (size_t)ADJ_AREA * N * sizeof(T), W->stream));
  HIPC(H, hipMemsetAsync(ab.tb, 0, (size_t)L.tb_slots * TB_SLOTS * sizeof(double), W->stream));
  int cur = 0, hs = 0;
  if (n_steps >= 1) {
    int sel[3] = {0, 0, 0}, count = 0;
    for (int b = 0; b < 3; ++b)
      if (mask & (1u << b)) sel[count++] = b;
    k_adj_seed<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, seed, make_int3(sel[0], sel[1], sel[2]), count,
                                                 ab.pb[0]);
    HIPC(H, hipGetLastError());
    for (int sg = L.nseg - 1; sg >= 0; --sg) {
      const int64_t s0 = (int64_t)sg * every, s1 = std::min<int64_t>(s0 + every, L.rev);
      int rc = lbm_ehd_restore(W, work + L.ckpt + (size_t)sg * L.ckpt_stride);
      if (rc) return H->fail(rc, "adjoint: restore: %s", W->err.c_str());
      for (int64_t t = s0; t < s1; ++t) step_record<T>(W, work + L.seg + (size_t)(t - s0) * L.slot_stride);
      for (int64_t t = s1 - 1; t >= s0; --t)
        step_adjoint<T>(W, work + L.seg + (size_t)(t - s0) * L.slot_stride, ab, cur, hs);
      HIPC(H, hipGetLastError());
    }
    // create: populations and field of the initial state
    int rc = lbm_ehd_restore(W, work + L.ckpt);
    if (rc) return H->fail(rc, "adjoint: restore: %s", W->err.c_str());
    k_adj_init_pops<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, ab, cur);
    Rec<T> rc0{};
    rc0.phi = (T *)I.phi[1];  // create's fields: buffer 1
    rc0.eps = (T *)I.eps;
    rc0.En = (T *)I.E;
    k_adj_mu<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, rc0, ab, cur, hs, 0);
    HIPC(H, hipGetLastError());
  }
  // initial potential guess
  {
    std::vector<T> buf(N);
    const std::vector<double> &ps = H->init_psi[0];
    const size_t nodes = (size_t)I.nn;  // dense host plane; the sweep's planes have stride N
    for (size_t k = 0; k < nodes; ++k) buf[k] = ps.empty() ? T(0) : (T)ps[k];
    HIPC(H, hipMemcpyAsync(psi0, buf.data(), nodes * sizeof(T), hipMemcpyHostToDevice, W->stream));
    HIPC(H, hipStreamSynchronize(W->stream));
  }
  const int K0 = p.init_sub_max;
  if (n_steps >= 1 && K0 > 0) {
    // cold start: chunk checkpoints, then each chunk recomputed with its
    // levels recorded and reversed
    const size_t lv = 9 * N;
    T *ck = (T *)(work + L.cold_ck);
    T *lev = (T *)(work + L.seg);
    k_h_equilibrium<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, psi0, cold[0]);
    int cp = 0;
    // checkpoints are needed up to the start of the last chunk
    const int kck = (L.cold_chunks - 1) * L.cold_len + 1;
    for (int k = 0; k < kck; ++k) {
      if (k % L.cold_len == 0)
        HIPC(H, hipMemcpyAsync(ck + (size_t)(k / L.cold_len) * lv, cold[cp], lv * sizeof(T), hipMemcpyDeviceToDevice,
                               W->stream));
      if (k + 1 < kck)
        k_poisson_buf<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, cold[cp], cold[cp ^ 1],
                                                        (const T *)I.eps, (const T *)I.q[1], nullptr);
      cp ^= 1;
    }
    for (int c = L.cold_chunks - 1; c >= 0; --c) {
      const int ka = c * L.cold_len, kb = std::min(K0, ka + L.cold_len);
      HIPC(H, hipMemcpyAsync(cold[0], ck + (size_t)c * lv, lv * sizeof(T), hipMemcpyDeviceToDevice, W->stream));
      cp = 0;
      for (int k = ka; k < kb; ++k) {
        k_poisson_buf<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, cold[cp], cold[cp ^ 1],
                                                        (const T *)I.eps, (const T *)I.q[1], lev + (size_t)(k - ka) * lv);
        cp ^= 1;
      }
      for (int k = kb - 1; k >= ka;) {
        if (k - 1 >= ka) {
          k_adj_poisson2<T><<<dim3(W->plan.total_tiles2), dim3(P2NT), 0, W->stream>>>(
              W->d_insts, W->table(0), lev + (size_t)(k - ka) * lv, lev + (size_t)(k - 1 - ka) * lv, (const T *)I.eps,
              ab, hs, ab.rb);
          k -= 2;
        } else {
          k_adj_poisson<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, lev + (size_t)(k - ka) * lv,
                                                          (const T *)I.eps, ab, hs, ab.rb);
          k -= 1;
        }
        hs ^= 1;
      }
      HIPC(H, hipGetLastError());
    }
  }
  if (n_steps >= 1)
    k_adj_create_tail<T><<<grid, block, 0, W->stream>>>(W->d_insts, W->d_b2i, ab, hs, (const T *)I.phi[1], psi0, mean,
                                                        inv_e0);
  double *out = (double *)(work + L.out);
  k_adj_reduce<<<1, block, 0, W->stream>>>(ab.tb, L.tb_slots, out);
  HIPC(H, hipGetLastError());
  double o[TB_SLOTS];
  HIPC(H, hipMemcpyAsync(o, out, sizeof o, hipMemcpyDeviceToHost, W->stream));
  HIPC(H, hipStreamSynchronize(W->stream));
  // theta = (eps2/eps1, eps3/eps1, sigma2/sigma1, sigma3/sigma1, E0)
  grad[0] = p.eps[0] * o[1];
  grad[1] = p.eps[0] * o[2];
  grad[2] = p.sigma[0] * o[4];
  grad[3] = p.sigma[0] * o[5];
  grad[4] = o[6];
  return LBM_EHD_OK;
}

}  // namespace

namespace {
constexpr int PERSIST_CHUNK = 256;  // steps per cooperative launch

// n steps as cooperative launches of PERSIST_CHUNK steps or fewer, each
// checked for a barrier wait that ran out.
template <typename S>
int do_step_persistent(lbm_ehd_s *H, int64_t n) {
  int per_cu = 0, ncu = 0;
  const void *kern = H->persist_timed ? (const void *)k_persistent<S, true> : (const void *)k_persistent<S, false>;
  HIPC(H, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, P2NT, 0));
  HIPC(H, hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, H->device));
  if (per_cu < 1 || ncu < 1) return H->fail(LBM_EHD_EUNSUPPORTED, "persistent step: the kernel does not fit a CU");
  const int grid = per_cu * ncu;
  unsigned *bar = (unsigned *)(H->ws + H->plan.bar_off);
  int *fail = (int *)(bar + PS_FAIL);
  PersistArgs *d_args = (PersistArgs *)(H->ws + H->plan.bar_off + align_up(PS_WORDS * sizeof(unsigned)));
  PersistArgs a;
  a.b2i4 = H->d_b2i4;
  a.tiles = H->table(2);
  a.b2i = H->d_b2i;
  a.bar = bar;
  a.n_ent4 = H->plan.total_blocks4;
  a.n_tiles = H->plan.total_tiles4;
  a.n_blk = H->plan.total_blocks;
  a.K = H->sub_max;
  a.spin_max = H->persist_polls;  // default 2^21 polls of ~1 us: a stage may take ~2 s
  const Inst *insts = H->d_insts;
  int khz = 0;
  HIPC(H, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, H->device));
  long long ticks[PS_STAGES] = {0, 0, 0, 0};
  for (double &v : H->persist_us) v = 0.0;
  H->persist_steps = 0;
  const int64_t n_all = n;
  while (n > 0) {
    const int chunk = (int)(n < PERSIST_CHUNK ? n : PERSIST_CHUNK);
    a.step0 = H->steps;
    a.n_steps = chunk;
    k_persist_begin<<<1, 64, 0, H->stream>>>(a, d_args);
    HIPC(H, hipGetLastError());
    const PersistArgs *pa = d_args;
    void *args[] = {(void *)&insts, (void *)&pa};
    HIPC(H, hipLaunchCooperativeKernel(kern, dim3(grid), dim3(P2NT), args, 0, H->stream));
    int f = 0;
    long long t[PS_STAGES];
    HIPC(H, hipMemcpyAsync(&f, fail, sizeof(int), hipMemcpyDeviceToHost, H->stream));
    HIPC(H, hipMemcpyAsync(t, bar + PS_CLOCK, sizeof t, hipMemcpyDeviceToHost, H->stream));
    HIPC(H, hipStreamSynchronize(H->stream));
    if (f) return H->fail(LBM_EHD_EHIP, "persistent step: a grid barrier wait ran out (state undefined)");
    for (int k = 0; k < PS_STAGES; ++k) ticks[k] += t[k];
    H->steps += chunk;
    n -= chunk;
  }
  if (khz > 0 && H->persist_timed) {
    for (int k = 0; k < PS_STAGES; ++k) H->persist_us[k] = (double)ticks[k] / (khz * 1e-3) / (double)n_all;
    H->persist_steps = n_all;
  }
  return LBM_EHD_OK;
}
}  // namespace

extern "C" {

int lbm_ehd_create(const lbm_ehd_params *params, int32_t n_inst, const lbm_ehd_init *init,
                   void *dev_workspace, void *hip_stream, lbm_ehd_t *out) {
  return create_impl(params, n_inst, init, dev_workspace, hip_stream, out, true);
}

int lbm_ehd_workspace_bytes(const lbm_ehd_params *params, int32_t n_inst, size_t *bytes) {
  if (!params || n_inst < 1 || !bytes) return LBM_EHD_EINVAL;
  for (int i = 0; i < n_inst; ++i)
    if (const char *m = validate(params[i], params[0])) {
      g_create_error = m;
      return LBM_EHD_EINVAL;
    }
  *bytes = make_plan(params, n_inst).total;
  return LBM_EHD_OK;
}

static int step_eager(lbm_ehd_t H, int64_t n) { return dispatch<StepF>(H, H, n); }

int lbm_ehd_step(lbm_ehd_t H, int64_t n) {
  if (!H || n < 0) return LBM_EHD_EINVAL;
  while (n > 0) {
    if (H->gexec && !H->prof && n >= H->glen && (H->steps & 1) == H->gpar) {
      HIPC(H, hipGraphLaunch(H->gexec, H->stream));
      H->steps += H->glen;
      n -= H->glen;
      continue;
    }
    // without a graph, or to restore the graph's step parity, or a tail
    const int64_t k = (H->gexec && !H->prof) ? (n >= H->glen ? 1 : n) : n;
    const int rc = step_eager(H, k);
    if (rc) return rc;
    n -= k;
  }
  return LBM_EHD_OK;
}

int lbm_ehd_step_persistent(lbm_ehd_t H, int64_t n) {
  if (!H || n < 0) return LBM_EHD_EINVAL;
  if (H->lattice != LBM_LATTICE_D2Q9 || (H->prec != LBM_PREC_FP32 && H->prec != LBM_PREC_FP16S))
    return H->fail(LBM_EHD_EUNSUPPORTED, "persistent step: D2Q9 with FP32 or FP16S storage only");
  if (H->adaptive || H->sub_max < 4 || H->sub_max % 4)
    return H->fail(LBM_EHD_EUNSUPPORTED, "persistent step: needs a fixed sub-iteration count, a multiple of 4");
  if (!H->vec_moments)
    return H->fail(LBM_EHD_EUNSUPPORTED, "persistent step: leaky-dielectric charge model only");
  if (H->prof) return H->fail(LBM_EHD_ESTATE, "persistent step: not while profiling");
  if (n == 0) return LBM_EHD_OK;
  return H->prec == LBM_PREC_FP16S ? do_step_persistent<__half>(H, n) : do_step_persistent<float>(H, n);
}

int lbm_ehd_graph(lbm_ehd_t H, int32_t steps_per_graph) {
  if (!H) return LBM_EHD_EINVAL;
  H->drop_graph();
  if (steps_per_graph == 0) return LBM_EHD_OK;
  if (steps_per_graph < 2 || (steps_per_graph & 1))
    return H->fail(LBM_EHD_EINVAL, "steps_per_graph must be an even number >= 2 (or 0 to release)");
  if (!H->stream) return H->fail(LBM_EHD_EINVAL, "graph capture needs a non-default stream");
  if (H->prof) return H->fail(LBM_EHD_ESTATE, "cannot capture while profiling");
  const long long saved = H->steps;
  HIPC(H, hipStreamBeginCapture(H->stream, hipStreamCaptureModeThreadLocal));
  const int rc = step_eager(H, steps_per_graph);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(H->stream, &g);
  H->steps = saved;  // captured work has not run
  if (rc || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return rc ? rc : H->fail(LBM_EHD_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  }
  H->graph = g;
  hipError_t ei = hipGraphInstantiate(&H->gexec, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    H->drop_graph();
    return H->fail(LBM_EHD_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
  }
  H->glen = steps_per_graph;
  H->gpar = (int)(saved & 1);
  return LBM_EHD_OK;
}

// Plane group of output field `bit`; fb: the field buffer of the last step
// (or of create), (steps + 1) & 1.
static void *field_src(const Inst &I, int bit, int fb) {
  switch (bit) {
    case 0: case 1: case 2: return I.phi[fb];  // offset applied by caller
    case 3: return I.rho;
    case 4: case 5: return I.u;
    case 6: return I.p;
    case 7: return I.psi;
    case 8: case 9: return I.E;
    case 10: return I.q[fb];
    case 11: case 12: case 13: return I.mu;
    case 14: return I.eps;
    case 15: return I.R;
    case 16: return I.u;
    case 17: return I.E;
    case 18: case 19: return I.ion;
    default: return nullptr;
  }
}
static int field_sub(int bit) {
  switch (bit) {
    case 1: case 5: case 9: case 12: case 19: return 1;
    case 2: case 13: case 16: case 17: return 2;
    default: return 0;
  }
}

int lbm_ehd_fields(lbm_ehd_t H, int32_t inst, uint32_t mask, void *dev_dst, int32_t dtype) {
  if (!H || inst < 0 || inst >= H->n_inst || !dev_dst || (mask >> 20) != 0)
    return H ? H->fail(LBM_EHD_EINVAL, "fields: bad argument") : LBM_EHD_EINVAL;
  if ((mask & (3u << 16)) != 0 && H->lattice != LBM_LATTICE_D3Q15)
    return H->fail(LBM_EHD_EINVAL, "fields: z components exist on D3Q15 only");
  if ((mask & (3u << 18)) != 0 && H->params[inst].charge_model != LBM_CHARGE_NERNST_PLANCK)
    return H->fail(LBM_EHD_EINVAL, "fields: ion concentrations exist under the Nernst-Planck model only");
  if (dtype != LBM_DTYPE_F32 && dtype != LBM_DTYPE_F64 && dtype != LBM_DTYPE_TANGENT_F64)
    return H->fail(LBM_EHD_EINVAL, "fields: bad dtype");
  const Inst &I = H->hinst[inst];
  // state planes have stride I.N; the output planes are dense (I.nn values)
  const size_t N = (size_t)I.N, M = (size_t)I.nn, te = elem_size(H->prec), de = dtype == LBM_DTYPE_F32 ? 4 : 8;
  char *dst = (char *)dev_dst;
  for (int bit = 0; bit < 20; ++bit) {
    if (!(mask & (1u << bit))) continue;
    const char *src = (const char *)field_src(I, bit, (int)((H->steps + 1) & 1)) + field_sub(bit) * N * te;
    int rc = convert_any(H, (int)te, src, dst, M, dtype);
    if (rc) return rc;
    dst += M * de;
  }
  return LBM_EHD_OK;
}

int lbm_ehd_populations(lbm_ehd_t H, int32_t inst, int32_t family, void *dev_dst, int32_t dtype) {
  if (!H || inst < 0 || inst >= H->n_inst || !dev_dst || family < 0 || family > 3)
    return H ? H->fail(LBM_EHD_EINVAL, "populations: bad argument") : LBM_EHD_EINVAL;
  if (dtype != LBM_DTYPE_F32 && dtype != LBM_DTYPE_F64) return H->fail(LBM_EHD_EINVAL, "populations: bad dtype");
  const Inst &I = H->hinst[inst];
  const dim3 grid((unsigned)((I.nn + NT - 1) / NT)), block(NT);
  const int pc = (int)(H->steps & 1);
  dispatch<ExportF>(H, H, grid, block, inst, family, pc, dev_dst, dtype);
  HIPC(H, hipGetLastError());
  return LBM_EHD_OK;
}

// Read and report the latched status of instance i (stream synchronised):
// EDIVERGED stays latched, ENOCONV is cleared once reported.
static int take_status(lbm_ehd_t H, int i, int &bits) {
  Ctl *dc = H->hinst[i].ctl;
  HIPC(H, hipMemcpy(&bits, &dc->status, sizeof(int), hipMemcpyDeviceToHost));
  if (bits & ST_NOCONV) {
    const int keep = bits & ~ST_NOCONV;
    HIPC(H, hipMemcpy(&dc->status, &keep, sizeof(int), hipMemcpyHostToDevice));
  }
  return LBM_EHD_OK;
}

// The diagnostics of instance inst after do_diag: synchronise, copy out,
// report the latched status.
static int finish_diag(lbm_ehd_t H, int32_t inst, double out[16]) {
  int rc;
  Ctl c;
  HIPC(H, hipStreamSynchronize(H->stream));
  HIPC(H, hipMemcpy(&c, H->hinst[inst].ctl, sizeof c, hipMemcpyDeviceToHost));
  for (int k = 0; k < 16; ++k) out[k] = c.diag[k];
  int bits = 0;
  if ((rc = take_status(H, inst, bits))) return rc;
  if (out[7] > 0 || (bits & ST_DIVERGED))
    return H->fail(LBM_EHD_EDIVERGED, "non-finite values in instance %d", inst);
  if (bits & ST_NOCONV)
    return H->fail(LBM_EHD_ENOCONV, "instance %d: a potential loop reached sub_max without meeting sub_tol", inst);
  return LBM_EHD_OK;
}

int lbm_ehd_diagnostics(lbm_ehd_t H, int32_t inst, double out[16]) {
  if (!H || inst < 0 || inst >= H->n_inst || !out) return LBM_EHD_EINVAL;
  int rc = dispatch<DiagF>(H, H, (double *)nullptr);
  if (rc) return rc;
  return finish_diag(H, inst, out);
}

int lbm_ehd_diagnostics_static(lbm_ehd_t H, int32_t inst, double out[16]) {
  if (!H || inst < 0 || inst >= H->n_inst || !out) return LBM_EHD_EINVAL;
  if (H->plan.total_blocks > DIAG_STATIC_MAX_BLOCKS)
    return H->fail(LBM_EHD_ENOMEM,
                   "diagnostics_static: the handle has %d node blocks of %d nodes; the static buffer holds %d",
                   H->plan.total_blocks, NT, DIAG_STATIC_MAX_BLOCKS);
  double *part = nullptr;
  int rc = static_scratch(H, &part);
  if (rc) return rc;
  // every slot the reduction reads is written by k_diag of this call first:
  // the buffer needs no clearing
  if ((rc = dispatch<DiagF>(H, H, part))) return rc;
  return finish_diag(H, inst, out);
}

int lbm_ehd_status(lbm_ehd_t H, int32_t *flags) {
  if (!H) return LBM_EHD_EINVAL;
  HIPC(H, hipStreamSynchronize(H->stream));
  int all = 0, rc;
  for (int i = 0; i < H->n_inst; ++i) {
    int bits = 0;
    if ((rc = take_status(H, i, bits))) return rc;
    all |= bits;
  }
  if (flags) *flags = all;
  if (all & ST_DIVERGED) return H->fail(LBM_EHD_EDIVERGED, "non-finite velocity or pressure formed");
  if (all & ST_NOCONV) return H->fail(LBM_EHD_ENOCONV, "a potential loop reached sub_max without meeting sub_tol");
  return LBM_EHD_OK;
}

int lbm_ehd_scalars(lbm_ehd_t H, double out[3]) {
  if (!H || !out) return LBM_EHD_EINVAL;
  HIPC(H, hipStreamSynchronize(H->stream));
  double ktot = 0;
  for (int i = 0; i < H->n_inst; ++i) {
    Ctl c;
    HIPC(H, hipMemcpy(&c, H->hinst[i].ctl, sizeof c, hipMemcpyDeviceToHost));
    ktot += (double)c.k_total;
  }
  out[0] = (double)H->steps;
  out[1] = ktot;
  out[2] = H->n_inst;
  return LBM_EHD_OK;
}

int lbm_ehd_get_tuning(lbm_ehd_t H, int32_t *config) {
  if (!H || !config) return LBM_EHD_EINVAL;
  *config = H->tuning;
  return LBM_EHD_OK;
}

int lbm_ehd_set_persistent_timing(lbm_ehd_t H, int32_t on) {
  if (!H || (on != 0 && on != 1)) return H ? H->fail(LBM_EHD_EINVAL, "set_persistent_timing: 0 or 1") : LBM_EHD_EINVAL;
  H->persist_timed = on;
  return LBM_EHD_OK;
}

int lbm_ehd_persistent_stage_times(lbm_ehd_t H, double us[4]) {
  if (!H || !us) return LBM_EHD_EINVAL;
  if (H->persist_steps <= 0)
    return H->fail(LBM_EHD_ESTATE, "persistent_stage_times: no timed persistent steps taken");
  for (int k = 0; k < 4; ++k) us[k] = H->persist_us[k];
  return LBM_EHD_OK;
}

int lbm_ehd_set_persistent_polls(lbm_ehd_t H, int32_t polls) {
  if (!H) return LBM_EHD_EINVAL;
  if (polls < 1) return H->fail(LBM_EHD_EINVAL, "set_persistent_polls: polls must be >= 1");
  H->persist_polls = polls;
  return LBM_EHD_OK;
}

int lbm_ehd_set_tuning(lbm_ehd_t H, int32_t config) {
  if (!H || (config & ~15) != 0) return H ? H->fail(LBM_EHD_EINVAL, "set_tuning: unknown bits") : LBM_EHD_EINVAL;
  if (H->prof) return H->fail(LBM_EHD_ESTATE, "set_tuning: not while profiling");
  const int glen = H->glen;
  H->drop_graph();  // a captured graph holds the previous tables
  H->tuning = config;
  H->apply_order();
  return glen ? lbm_ehd_graph(H, glen) : LBM_EHD_OK;
}

int lbm_ehd_tune(lbm_ehd_t H, int32_t steps, void *dev_scratch, double ms_per_step[16], int32_t *best) {
  if (!H || steps < 1 || !dev_scratch || !ms_per_step) return LBM_EHD_EINVAL;
  if (H->prof) return H->fail(LBM_EHD_ESTATE, "tune: not while profiling");
  // the LDS-tiled potential kernel exists for fixed-count D2Q9 FP32/FP16S/FP64 handles
  const bool pair_form = H->lattice == LBM_LATTICE_D2Q9 && !H->adaptive && H->prec != LBM_PREC_TANGENT;
  // the two collide load schedules differ for 4-byte arithmetic (FP32, FP16S)
  const bool sched_form = H->prec == LBM_PREC_FP32 || H->prec == LBM_PREC_FP16S;
  // the tall tile shapes exist for FP32, FP16S and FP64
  const bool tall_form = pair_form && (sched_form || H->prec == LBM_PREC_FP64);
  const int glen = H->glen;
  H->drop_graph();
  int rc = lbm_ehd_checkpoint(H, dev_scratch);
  if (rc) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPC(H, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return H->fail(LBM_EHD_EHIP, "tune: hipEventCreate failed");
  }
  int pick = -1;
  for (int c = 0; c < 16 && rc == LBM_EHD_OK; ++c) {
    ms_per_step[c] = -1.0;
    // bits that change nothing on this handle: same launches as without them
    if ((c & LBM_TUNE_SINGLE_POTENTIAL) && !pair_form) continue;
    if ((c & LBM_TUNE_COLLIDE_PER_FAMILY) && !sched_form) continue;
    if ((c & LBM_TUNE_TALL_TILES) && (!tall_form || (c & LBM_TUNE_SINGLE_POTENTIAL))) continue;
    H->tuning = c;
    H->apply_order();
    if ((rc = lbm_ehd_restore(H, dev_scratch)) || (rc = lbm_ehd_step(H, 2))) break;
    float ms = 0.f;
    hipError_t e = hipEventRecord(e0, H->stream);
    if (e == hipSuccess && (rc = lbm_ehd_step(H, steps)) == LBM_EHD_OK) {
      e = hipEventRecord(e1, H->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    }
    if (rc) break;
    if (e != hipSuccess) {
      rc = H->fail(LBM_EHD_EHIP, "tune: %s", hipGetErrorString(e));
      break;
    }
    ms_per_step[c] = (double)ms / steps;
    if (pick < 0 || ms_per_step[c] < ms_per_step[pick]) pick = c;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // the state as it was, the fastest configuration (or the previous one on failure)
  const int keep = rc == LBM_EHD_OK && pick >= 0 ? pick : 0;
  const int rr = lbm_ehd_restore(H, dev_scratch);
  if (rc) return rc;
  if (rr) return rr;
  if (best) *best = keep;
  H->tuning = keep;
  H->apply_order();
  return glen ? lbm_ehd_graph(H, glen) : LBM_EHD_OK;
}

int lbm_ehd_checkpoint_bytes(lbm_ehd_t H, size_t *bytes) {
  if (!H || !bytes) return LBM_EHD_EINVAL;
  *bytes = H->plan.total - H->plan.state_off;
  return LBM_EHD_OK;
}

int lbm_ehd_checkpoint(lbm_ehd_t H, void *dev_buf) {
  if (!H || !dev_buf) return LBM_EHD_EINVAL;
  HIPC(H, hipMemcpyAsync(dev_buf, H->ws + H->plan.state_off, H->plan.total - H->plan.state_off,
                         hipMemcpyDeviceToDevice, H->stream));
  H->err.clear();
  return LBM_EHD_OK;
}

int lbm_ehd_restore(lbm_ehd_t H, const void *dev_buf) {
  if (!H || !dev_buf) return LBM_EHD_EINVAL;
  HIPC(H, hipMemcpyAsync(H->ws + H->plan.state_off, dev_buf, H->plan.total - H->plan.state_off,
                         hipMemcpyDeviceToDevice, H->stream));
  // the population buffer parity follows the restored step count
  Ctl c;
  HIPC(H, hipStreamSynchronize(H->stream));
  HIPC(H, hipMemcpy(&c, H->hinst[0].ctl, sizeof c, hipMemcpyDeviceToHost));
  H->steps = c.steps;
  return LBM_EHD_OK;
}

static lbm_ehd_params tangent_params(const lbm_ehd_params &p, int dir) {
  lbm_ehd_params t = p;
  t.precision = LBM_PREC_TANGENT;
  for (int k = 0; k < 5; ++k) t.dtheta[k] = (k == dir) ? 1.0 : 0.0;
  return t;
}

int lbm_ehd_tangent_workspace_bytes(lbm_ehd_t H, size_t *bytes) {
  if (!H || !bytes) return LBM_EHD_EINVAL;
  if (H->n_inst != 1) return H->fail(LBM_EHD_EUNSUPPORTED, "gradients need a single-instance handle");
  const lbm_ehd_params t = tangent_params(H->params[0], 0);
  *bytes = make_plan(&t, 1).total;
  return LBM_EHD_OK;
}

int lbm_ehd_tangent_gradient(lbm_ehd_t H, int64_t n_steps, const void *dev_seed, uint32_t seed_mask,
                             void *dev_work, size_t work_bytes, double grad_theta[5]) {
  if (!H || !grad_theta || !dev_seed || n_steps < 0) return LBM_EHD_EINVAL;
  if (H->n_inst != 1) return H->fail(LBM_EHD_EUNSUPPORTED, "gradients need a single-instance handle");
  if (seed_mask == 0 || (seed_mask >> 20) != 0 ||
      ((seed_mask & (3u << 16)) != 0 && H->lattice != LBM_LATTICE_D3Q15) ||
      ((seed_mask & (3u << 18)) != 0 && H->params[0].charge_model != LBM_CHARGE_NERNST_PLANCK))
    return H->fail(LBM_EHD_EINVAL, "tangent gradient: bad seed mask");
  size_t need = 0;
  lbm_ehd_tangent_workspace_bytes(H, &need);
  if (!dev_work || work_bytes < need || ((uintptr_t)dev_work % ALIGN) != 0)
    return H->fail(LBM_EHD_ENOMEM, "tangent gradient: work buffer must be >= %zu bytes and 256-byte aligned", need);
  lbm_ehd_init ini;
  ini.phi0 = H->init_phi[0].data();
  ini.u0 = H->init_u[0].empty() ? nullptr : H->init_u[0].data();
  ini.q0 = H->init_q[0].empty() ? nullptr : H->init_q[0].data();
  ini.psi0 = H->init_psi[0].empty() ? nullptr : H->init_psi[0].data();
  ini.ions0 = H->init_ions[0].empty() ? nullptr : H->init_ions[0].data();
  for (int dir = 0; dir < 5; ++dir) {
    const lbm_ehd_params t = tangent_params(H->params[0], dir);
    lbm_ehd_t T = nullptr;
    int rc = lbm_ehd_create(&t, 1, &ini, dev_work, (void *)H->stream, &T);
    if (rc) return H->fail(rc, "tangent gradient: tangent run: %s", g_create_error.c_str());
    rc = lbm_ehd_step(T, n_steps);
    if (rc) {
      H->err = T->err;
      lbm_ehd_destroy(T);
      return rc;
    }
    // contract the tangent fields of the last step with the seed
    const Inst &I = T->hinst[0];
    SeedPlanes sp;
    sp.count = 0;
    for (int bit = 0; bit < 20; ++bit)
      if (seed_mask & (1u << bit))
        sp.plane[sp.count++] = (const DualD *)field_src(I, bit, (int)((T->steps + 1) & 1)) + (size_t)field_sub(bit) * I.N;
    k_seed_dot<<<dim3(I.nblk), dim3(NT), 0, T->stream>>>(T->d_insts, sp, (const double *)dev_seed);
    k_reduce_seed_dot<<<1, NT, 0, T->stream>>>(T->d_insts);
    Ctl c;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(T->stream);
    if (e == hipSuccess) e = hipMemcpy(&c, I.ctl, sizeof c, hipMemcpyDeviceToHost);
    lbm_ehd_destroy(T);
    if (e != hipSuccess) return H->fail(LBM_EHD_EHIP, "tangent gradient: %s", hipGetErrorString(e));
    grad_theta[dir] = c.diag[22];
  }
  return LBM_EHD_OK;
}

int lbm_ehd_adjoint_workspace_bytes(lbm_ehd_t H, int64_t n_steps, int32_t ckpt_every, size_t *bytes) {
  if (!H || !bytes || n_steps < 0 || ckpt_every < 1) return LBM_EHD_EINVAL;
  if (const char *m = adjoint_unsupported(H)) return H->fail(LBM_EHD_EUNSUPPORTED, "%s", m);
  *bytes = adj_layout(H, n_steps, ckpt_every).total;
  return LBM_EHD_OK;
}

int lbm_ehd_record(lbm_ehd_t H, int64_t n_steps, int32_t ckpt_every, void *dev_work, size_t work_bytes) {
  if (!H || n_steps < 0 || ckpt_every < 1) return LBM_EHD_EINVAL;
  if (const char *m = adjoint_unsupported(H)) return H->fail(LBM_EHD_EUNSUPPORTED, "%s", m);
  if (H->steps != 0) return H->fail(LBM_EHD_ESTATE, "record: the handle must be at its create state");
  const AdjLayout L = adj_layout(H, n_steps, ckpt_every);
  if (!dev_work || work_bytes < L.total || ((uintptr_t)dev_work % ALIGN) != 0)
    return H->fail(LBM_EHD_ENOMEM, "record: work buffer must be >= %zu bytes and 256-byte aligned", L.total);
  H->rec_work = nullptr;
  const int rc = record_run(H, (char *)dev_work, L, n_steps, ckpt_every);
  if (rc) return rc;
  H->rec_work = dev_work;
  H->rec_n = n_steps;
  H->rec_every = ckpt_every;
  return LBM_EHD_OK;
}

int lbm_ehd_adjoint(lbm_ehd_t H, int64_t n_steps, int32_t ckpt_every, const void *dev_seed, uint32_t seed_mask,
                    void *dev_work, size_t work_bytes, double grad_theta[5]) {
  if (!H || !grad_theta || !dev_seed || n_steps < 0 || ckpt_every < 1) return LBM_EHD_EINVAL;
  if (const char *m = adjoint_unsupported(H)) return H->fail(LBM_EHD_EUNSUPPORTED, "%s", m);
  if (seed_mask == 0 || (seed_mask & ~7u) != 0)
    return H->fail(LBM_EHD_EUNSUPPORTED, "adjoint: seeds on phi1..phi3 only (lbm_ehd_tangent_gradient takes any field)");
  const AdjLayout L = adj_layout(H, n_steps, ckpt_every);
  if (!dev_work || work_bytes < L.total || ((uintptr_t)dev_work % ALIGN) != 0)
    return H->fail(LBM_EHD_ENOMEM, "adjoint: work buffer must be >= %zu bytes and 256-byte aligned", L.total);
  char *work = (char *)dev_work;
  const bool recorded = H->rec_work == dev_work && H->rec_n == n_steps && H->rec_every == ckpt_every;
  lbm_ehd_t W = nullptr;
  int rc;
  // the sweep's handle runs in the caller's launch configuration: its
  // recomputed segments then repeat the recorded forward's kernels
  auto configure = [&]() {
    W->tuning = H->tuning;
    W->apply_order();
  };
  if (recorded) {
    rc = create_impl(&H->params[0], 1, nullptr, work + L.shell, (void *)H->stream, &W, false);
    if (!rc) configure();
  } else {
    lbm_ehd_init ini;
    ini.phi0 = H->init_phi[0].data();
    ini.u0 = H->init_u[0].empty() ? nullptr : H->init_u[0].data();
    ini.q0 = H->init_q[0].empty() ? nullptr : H->init_q[0].data();
    ini.psi0 = H->init_psi[0].empty() ? nullptr : H->init_psi[0].data();
    ini.ions0 = H->init_ions[0].empty() ? nullptr : H->init_ions[0].data();
    rc = create_impl(&H->params[0], 1, &ini, work + L.shell, (void *)H->stream, &W, true);
    if (!rc) {
      configure();
      rc = record_run(W, work, L, n_steps, ckpt_every);
      if (rc) H->err = W->err;
    }
  }
  if (rc) {
    if (W) lbm_ehd_destroy(W);
    else H->err = g_create_error;
    return rc;
  }
  if (H->prec == LBM_PREC_FP64)
    rc = reverse_sweep<double>(H, W, work, L, n_steps, ckpt_every, (const double *)dev_seed, seed_mask, grad_theta);
  else
    rc = reverse_sweep<float>(H, W, work, L, n_steps, ckpt_every, (const double *)dev_seed, seed_mask, grad_theta);
  lbm_ehd_destroy(W);
  return rc;
}

int lbm_ehd_profile_begin(lbm_ehd_t H) {
  if (!H) return LBM_EHD_EINVAL;
  H->prof = true;
  H->ev_used = 0;
  H->ev_kind.clear();
  return LBM_EHD_OK;
}

int lbm_ehd_profile_end(lbm_ehd_t H, double ms[8], int64_t launches[8]) {
  if (!H || !ms || !launches) return LBM_EHD_EINVAL;
  if (!H->prof) return H->fail(LBM_EHD_ESTATE, "profile_end without profile_begin");
  H->prof = false;
  for (int k = 0; k < 8; ++k) {
    ms[k] = 0;
    launches[k] = 0;
  }
  HIPC(H, hipStreamSynchronize(H->stream));
  for (size_t i = 0; i < H->ev_kind.size(); ++i) {
    float t = 0;
    HIPC(H, hipEventElapsedTime(&t, H->ev_pool[2 * i], H->ev_pool[2 * i + 1]));
    ms[H->ev_kind[i]] += t;
    launches[H->ev_kind[i]] += 1;
  }
  H->ev_used = 0;
  H->ev_kind.clear();
  return LBM_EHD_OK;
}

void lbm_ehd_destroy(lbm_ehd_t H) { delete H; }

const char *lbm_ehd_strerror(int code) {
  switch (code) {
    case LBM_EHD_OK: return "ok";
    case LBM_EHD_EINVAL: return "invalid argument";
    case LBM_EHD_ENOMEM: return "workspace too small or misaligned";
    case LBM_EHD_EHIP: return "HIP runtime error";
    case LBM_EHD_EDIVERGED: return "simulation diverged (non-finite populations)";
    case LBM_EHD_ENOCONV: return "potential iteration reached its cap";
    case LBM_EHD_ESTATE: return "call not valid in this state";
    case LBM_EHD_EUNSUPPORTED: return "not supported by this library";
    default: return "unknown error";
  }
}

const char *lbm_ehd_last_error(lbm_ehd_t H) { return H ? H->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
