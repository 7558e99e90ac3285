// Grid-resident batch step: n coupled time steps of every instance of a
// handle in one cooperative launch.  Each step runs the stages of the
// ordinary fixed-count D2Q9 step on tall potential tiles (a1 order-parameter
// moments; a2-a4 the charge step and the potential sub-iterations, four per
// tile pass; a5 field and chemical potentials; a6-a11 collide-and-stream)
// over the block and tile tables of all instances, with a grid-wide barrier
// between stages, in the same arithmetic as the separate launches (the
// state after n steps is bitwise that of lbm_ehd_step in a tall-tile launch
// configuration).
//
// Every block of the launch is resident (hipLaunchCooperativeKernel refuses
// a grid that does not fit), and every barrier wait is bounded: a block that
// waits too long, or sees that another block gave up, raises the failure
// word and leaves, so the launch always ends.
#ifndef LBM_EHD_PERSISTENT_H
#define LBM_EHD_PERSISTENT_H

#include "lbm_ehd_kernels.h"

namespace lbm {

struct PersistArgs {
  const int2 *b2i4;   // moments table (entries of 4 x 256 nodes), n_ent4 entries
  const int4 *tiles;  // tall four-sub-iteration tiles, n_tiles entries
  const int2 *b2i;    // node blocks, n_blk entries
  unsigned *bar;      // PS_WORDS barrier words (zero at launch; see grid_barrier)
  long long step0;    // steps taken before the launch (field buffer parity)
  int n_ent4, n_tiles, n_blk;
  int n_steps;        // steps of this launch
  int K;              // potential sub-iterations per step, a multiple of 4
  int spin_max;       // polls of a barrier wait before it gives up
};

constexpr int PS_SUB = P2NT / NT;  // node blocks one persistent block runs at once

// Barrier words: eight group counters (blocks take group blockIdx.x % 8,
// the order in which the dispatcher deals consecutive blocks to the XCDs),
// each on a 256-byte line of its own, then the counter of completed groups,
// then the failure word, then the stage clock sums (PS_STAGES 64-bit words:
// wall-clock ticks block 0 spent in each kind of stage, barrier included,
// summed over the launch's steps).
constexpr int PS_GROUPS = 8, PS_LINE = 64;  // groups; words per counter line
constexpr int PS_STAGES = 4;                // moments, charge + potential, field + mu, collide
constexpr int PS_TOP = PS_GROUPS * PS_LINE, PS_FAIL = PS_TOP + PS_LINE, PS_CLOCK = PS_FAIL + PS_LINE,
              PS_WORDS = PS_CLOCK + PS_LINE;

// Grid-wide barrier.  Every block arrives once per barrier, so a group's
// counter reaches (passed + 1) x (its blocks) when the group's last block
// arrives; that block then counts the group done, and all blocks wait for
// (passed + 1) x (groups) on the top counter.  Thread 0 publishes the
// block's writes (a device-scope release fence after the block barrier:
// this XCD's L2 written back), arrives and polls with relaxed atomics, and
// takes one device-scope acquire fence (this CU's and XCD's stale lines
// dropped) before the block goes on.  Returns false (uniformly over the block)
// once the wait ran out or another block gave up.
__device__ __forceinline__ bool grid_barrier(const cptr<PersistArgs> a, unsigned &passed) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int good = 1;
    unsigned *bar = a->bar;
    int *fail = (int *)(bar + PS_FAIL);
    const int spin_max = a->spin_max;
    const unsigned nb = gridDim.x, g = blockIdx.x % PS_GROUPS;
    const unsigned ng = nb < PS_GROUPS ? nb : PS_GROUPS;  // groups with blocks
    const unsigned in_g = (nb - g + PS_GROUPS - 1) / PS_GROUPS;  // blocks of group g
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned prev = __hip_atomic_fetch_add(bar + g * PS_LINE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (prev + 1 == (passed + 1) * in_g)
      __hip_atomic_fetch_add(bar + PS_TOP, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = (passed + 1) * ng;
    int polls = 0;
    while (__hip_atomic_load(bar + PS_TOP, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++polls > spin_max) {
        __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    ok = good;
  }
  __syncthreads();
  const bool r = ok != 0;
  ++passed;
  return r;
}

// The stages but the last, each a function of its own, called once per
// stage: the register allocator then sees one stage at a time, as in the
// separate launches (all inlined into one loop, the stages' values crowd
// the scalar registers and every stage spills).  A call's arguments are taken
// as wave-uniform (readfirstlane) and the launch arguments read with scalar
// loads from their device copy, so the instance descriptors are read with
// scalar loads as in the separate launches.  A persistent block of 1024
// threads runs the node stages as four node blocks of 256 at a time (one per
// 256-thread share, a wave-uniform index: a wave never straddles two).
__device__ __forceinline__ int ps_share() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x / NT); }
__device__ __forceinline__ int ps_u(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Entry of the node list a share runs in a round: share s of persistent
// block b takes entry (4 round + s) nb + b, so that, as with a launch of one
// block per entry, the entries an XCD runs are those equal to its index
// modulo 8 (the block order groups each XCD's rows; nb is a multiple of 8).
__device__ __forceinline__ int ps_entry(int round, int sub, int nb) {
  return (round * PS_SUB + sub) * nb + (int)blockIdx.x;
}

// a1: moments, two nodes per thread (the four-node form's 144 values of a
// thread do not fit beside the other stages' 128 VGPRs; same sums).
template <typename S>
__device__ __noinline__ void ps_moments(const Inst *insts0, const PersistArgs *pa, int pc0) {
  const Inst *insts = uniform_ptr(insts0);
  const cptr<PersistArgs> a = cst(uniform_ptr(pa));
  const int pc = ps_u(pc0), sub = ps_share(), tid = (int)threadIdx.x % NT, nb = (int)gridDim.x, n = 2 * a->n_ent4;
  const int2 *b2i4 = a->b2i4;
#pragma unroll 1
  for (int r = 0; r * PS_SUB * nb < n; ++r) {
    const int e = ps_entry(r, sub, nb);
    if (e < n) moments4_body<D2Q9, float, S, 2, true>(insts, b2i4, pc, Rec<float>{}, e, tid);
  }
}

// a2-a4: one pass of four potential sub-iterations over the tall tiles, the
// first pass of a step with the charge step (l: pass index).
__device__ __noinline__ void ps_potential(const Inst *insts0, const PersistArgs *pa, int pc0, int l0) {
  __shared__ float buf[(Q - 1) * P2EW * P2Shape<2, 4>::ER];
  const Inst *insts = uniform_ptr(insts0);
  const cptr<PersistArgs> a = cst(uniform_ptr(pa));
  const int pc = ps_u(pc0), l = ps_u(l0), L = a->K / 4, nb = (int)gridDim.x, n = a->n_tiles;
  const int4 *tiles = a->tiles;
#pragma unroll 1
  for (int ti = (int)blockIdx.x; ti < n; ti += nb) {
    if (l == 0)
      p2_body<float, 2, 4, true, true>(insts, tiles, ti, 0, L == 1 ? 1 : 0, pc, P2Rec<float, 4>{}, buf);
    else
      p2_body<float, 2, 4, false, true>(insts, tiles, ti, l & 1, l == L - 1 ? 1 : 0, pc, P2Rec<float, 4>{}, buf);
  }
}

// a5: field and chemical potentials; with part set, each node block's
// residual terms summed over its four waves in k_mu's order (the partials
// the diagnostics read: the last step of a launch is the one they see, and
// the other steps skip the block-wide sums).
__device__ __noinline__ void ps_mu(const Inst *insts0, const PersistArgs *pa, int pc0, int hflip0, int part0) {
  __shared__ double red[P2NT / 64][2];
  const Inst *insts = uniform_ptr(insts0);
  const cptr<PersistArgs> a = cst(uniform_ptr(pa));
  const int pc = ps_u(pc0), hflip = ps_u(hflip0), part = ps_u(part0), sub = ps_share(), tid = (int)threadIdx.x % NT,
            nb = (int)gridDim.x, n = a->n_blk;
  const int2 *b2i = a->b2i;
  // residual partials of one node block into its slot (when part)
  auto partials = [&](const MuIn<D2Q9, float> &in, int b, double (&r)[2]) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
      for (int o = 32; o > 0; o >>= 1) r[k] += __shfl_down(r[k], o, 64);
    if ((threadIdx.x & 63) == 0) {
      red[threadIdx.x >> 6][0] = r[0];
      red[threadIdx.x >> 6][1] = r[1];
    }
    __syncthreads();
    if (tid == 0 && b < n) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        double t = 0;
        for (int i = 0; i < NT / 64; ++i) t += red[sub * (NT / 64) + i][k];
        in.Ip->part_mu[(size_t)in.lblk * 2 + k] = t;
      }
    }
    __syncthreads();
  };
  // two node blocks per share and round: both blocks' loads are issued
  // before either waits (a wave waits for its oldest loads first, so the
  // control words of both are read before any plane)
#pragma unroll 1
  for (int rd = 0; rd * PS_SUB * nb < n; rd += 2) {
    const int b0 = ps_entry(rd, sub, nb), b1 = ps_entry(rd + 1, sub, nb);
    // (a block past the table's end fetches the last block's nodes and
    // finishes none)
    MuIn<D2Q9, float> in0, in1;
    mu_locate<D2Q9, float, true>(insts, b2i, b0 < n ? b0 : n - 1, tid, hflip, pc, in0);
    mu_locate<D2Q9, float, true>(insts, b2i, b1 < n ? b1 : n - 1, tid, hflip, pc, in1);
    if (b0 >= n) in0.nd.valid = false;
    if (b1 >= n) in1.nd.valid = false;
    // both blocks' plane addresses in registers before the first plane
    // load: no memory access moves across this point (left to itself, the
    // compiler puts the first block's plane loads before the second block's
    // lookups, whose wait then drains them)
    asm volatile("" ::"v"(in0.h), "v"(in0.phi), "v"(in1.h), "v"(in1.phi) : "memory");
    __builtin_amdgcn_sched_barrier(0);
    mu_fetch<D2Q9, float>(in0);
    mu_fetch<D2Q9, float>(in1);
    __builtin_amdgcn_sched_barrier(0);  // every load issued before any arithmetic on them
    double r0[2], r1[2];
    mu_finish<D2Q9, float>(in0, Rec<float>{}, r0);
    mu_finish<D2Q9, float>(in1, Rec<float>{}, r1);
    if (!part) continue;  // uniform over the launch
    partials(in0, b0, r0);
    partials(in1, b1, r1);
  }
}

// a6-a11: collide-and-stream (u, p and rho written when write_macro).
// Inlined into the step loop: as a call its spills cost more (156 against
// 141 us per 1024^2 step).
template <typename S>
__device__ __forceinline__ void ps_collide(const Inst *insts0, const PersistArgs *pa, int pc0, int hflip0, int wm0) {
  const Inst *insts = uniform_ptr(insts0);
  const cptr<PersistArgs> a = cst(uniform_ptr(pa));
  const int pc = ps_u(pc0), hflip = ps_u(hflip0), wm = ps_u(wm0), sub = ps_share(), tid = (int)threadIdx.x % NT,
            nb = (int)gridDim.x, n = a->n_blk, K = a->K;
  const int2 *b2i = a->b2i;
#pragma unroll 1
  for (int rd = 0; rd * PS_SUB * nb < n; ++rd) {
    const int b = ps_entry(rd, sub, nb);
    if (b < n) collide_body<D2Q9, float, S, false, true>(insts, b2i, pc, wm, K, hflip, Rec<float>{}, b, tid);
  }
}

// One block of 1024 threads per CU (the potential stage's tile needs all
// of them and 64 KB of LDS); the bound keeps every stage at 128 VGPRs, four
// waves per SIMD.
//   pa: the launch arguments in device memory (k_persist_begin copies them).
//   TIMED: block 0's thread 0 reads the wall clock after every barrier and
//   adds each stage's ticks to its sum (lbm_ehd_persistent_stage_times); a
//   separate instantiation, since the readings cost the stages registers.
template <typename S, bool TIMED = false>
__global__ __launch_bounds__(P2NT, 4) void k_persistent(const Inst *__restrict__ insts, const PersistArgs *pa) {
  const cptr<PersistArgs> a = cst(pa);
  const int L = a->K / 4, hflip = L & 1, n_steps = a->n_steps;
  const long long step0 = a->step0;
  // the sums and the last reading live in LDS, not in registers the
  // stages need
  __shared__ long long sum[PS_STAGES + 1];
  const bool timer = TIMED && blockIdx.x == 0 && threadIdx.x == 0;
  if (timer) {
#pragma unroll
    for (int k = 0; k < PS_STAGES; ++k) sum[k] = 0;
    sum[PS_STAGES] = wall_clock64();
  }
  auto lap = [&](int stage) {
    if (timer) {
      const long long t = wall_clock64();
      sum[stage] += t - sum[PS_STAGES];
      sum[PS_STAGES] = t;
    }
  };
  unsigned passed = 0;
  for (int s = 0; s < n_steps; ++s) {
    const int pc = (int)((step0 + s) & 1);
    ps_moments<S>(insts, pa, pc);
    if (!grid_barrier(a, passed)) return;
    lap(0);
    for (int l = 0; l < L; ++l) {
      ps_potential(insts, pa, pc, l);
      if (!grid_barrier(a, passed)) return;
    }
    lap(1);
    ps_mu(insts, pa, pc, hflip, s == n_steps - 1 ? 1 : 0);
    if (!grid_barrier(a, passed)) return;
    lap(2);
    ps_collide<S>(insts, pa, pc, hflip, s == n_steps - 1 ? 1 : 0);
    if (!grid_barrier(a, passed)) return;
    lap(3);
  }
  if (timer) {
    long long *out = (long long *)(a->bar + PS_CLOCK);
#pragma unroll
    for (int k = 0; k < PS_STAGES; ++k) out[k] = sum[k];
  }
}

// Before a launch: the launch arguments into device memory and the
// barrier words cleared (a kernel, not a copy and a memset).
__global__ void k_persist_begin(PersistArgs a, PersistArgs *dst) {
  for (int i = (int)threadIdx.x; i < PS_WORDS; i += (int)blockDim.x) a.bar[i] = 0u;
  if (threadIdx.x == 0) *dst = a;
}

}  // namespace lbm

#endif
