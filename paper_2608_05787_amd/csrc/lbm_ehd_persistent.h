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
  const int2 *b2i4;   // moments table (four nodes per thread), n_ent4 entries
  const int4 *tiles;  // tall four-sub-iteration tiles, n_tiles entries
  const int2 *b2i;    // node blocks, n_blk entries
  unsigned *bar;      // barrier arrivals since the launch (zero at launch)
  int *fail;          // raised when a barrier wait ran out (zero at launch)
  long long step0;    // steps taken before the launch (field buffer parity)
  int n_ent4, n_tiles, n_blk;
  int n_steps;        // steps of this launch
  int K;              // potential sub-iterations per step, a multiple of 4
  int spin_max;       // polls of a barrier wait before it gives up
};

constexpr int PS_SUB = P2NT / NT;  // node blocks one persistent block runs at once

// Grid-wide barrier: every block arrives once per barrier, so the
// arrivals counter reaches (passed + 1) x gridDim.x when the last block of
// this one arrives.  Thread 0 publishes the block's writes (device-scope
// release after the block barrier), arrives, polls, and takes the
// device-scope acquire that drops this CU's and XCD's stale cache lines
// before the block goes on.  Returns false (uniformly over the block) once
// the wait ran out or another block gave up.
__device__ __forceinline__ bool grid_barrier(const cptr<PersistArgs> a, unsigned &passed) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int good = 1;
    unsigned *bar = a->bar;
    int *fail = a->fail;
    const int spin_max = a->spin_max;
    __threadfence();
    const unsigned target = (passed + 1) * gridDim.x;
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int polls = 0;
    while (__hip_atomic_load(bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 || ++polls > spin_max) {
        __hip_atomic_store(fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        good = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(2);
    }
    __threadfence();
    ok = good;
  }
  __syncthreads();
  const bool r = ok != 0;
  ++passed;
  return r;
}

// The stages, each a function of its own, called once per stage: the
// register allocator then sees one stage at a time, as in the separate
// launches (inlined into one loop, the stages' values crowd the scalar
// registers and the collide stage spills).  A call's arguments are taken
// as wave-uniform (readfirstlane) and the launch arguments read with scalar
// loads from their device copy, so the instance descriptors are read with
// scalar loads as in the separate launches.  A persistent block of 1024
// threads runs the node stages as four node blocks of 256 at a time (one per
// 256-thread share, a wave-uniform index: a wave never straddles two).
__device__ __forceinline__ int ps_share() { return __builtin_amdgcn_readfirstlane((int)threadIdx.x / NT); }
__device__ __forceinline__ int ps_u(int v) { return __builtin_amdgcn_readfirstlane(v); }

// a1: moments (the block's four shares take four consecutive entries).
template <typename S>
__device__ __noinline__ void ps_moments(const Inst *insts0, const PersistArgs *pa, int pc0) {
  const Inst *insts = uniform_ptr(insts0);
  const cptr<PersistArgs> a = cst(uniform_ptr(pa));
  const int pc = ps_u(pc0), sub = ps_share(), tid = (int)threadIdx.x % NT, nb = (int)gridDim.x, n = a->n_ent4;
  const int2 *b2i4 = a->b2i4;
#pragma unroll 1
  for (int base = (int)blockIdx.x * PS_SUB; base < n; base += nb * PS_SUB)
    if (base + sub < n) moments4_body<D2Q9, float, S, 4>(insts, b2i4, pc, Rec<float>{}, base + sub, tid);
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

// a5: field and chemical potentials; each node block's residual terms
// summed over its four waves in k_mu's order.
__device__ __noinline__ void ps_mu(const Inst *insts0, const PersistArgs *pa, int pc0, int hflip0) {
  __shared__ double red[P2NT / 64][2];
  const Inst *insts = uniform_ptr(insts0);
  const cptr<PersistArgs> a = cst(uniform_ptr(pa));
  const int pc = ps_u(pc0), hflip = ps_u(hflip0), sub = ps_share(), tid = (int)threadIdx.x % NT,
            nb = (int)gridDim.x, n = a->n_blk;
  const int2 *b2i = a->b2i;
#pragma unroll 1
  for (int base = (int)blockIdx.x * PS_SUB; base < n; base += nb * PS_SUB) {
    const int b = base + sub;
    double r[2] = {0.0, 0.0};
    const Inst *Ip = nullptr;
    int lblk = 0;
    if (b < n) mu_body<D2Q9, float, true>(insts, b2i, hflip, pc, Rec<float>{}, b, tid, r, Ip, lblk);
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
        Ip->part_mu[(size_t)lblk * 2 + k] = t;
      }
    }
    __syncthreads();
  }
}

// a6-a11: collide-and-stream (u, p and rho written when write_macro).
template <typename S>
__device__ __noinline__ void ps_collide(const Inst *insts0, const PersistArgs *pa, int pc0, int hflip0, int wm0) {
  const Inst *insts = uniform_ptr(insts0);
  const cptr<PersistArgs> a = cst(uniform_ptr(pa));
  const int pc = ps_u(pc0), hflip = ps_u(hflip0), wm = ps_u(wm0), sub = ps_share(), tid = (int)threadIdx.x % NT,
            nb = (int)gridDim.x, n = a->n_blk, K = a->K;
  const int2 *b2i = a->b2i;
#pragma unroll 1
  for (int base = (int)blockIdx.x * PS_SUB; base < n; base += nb * PS_SUB)
    if (base + sub < n) collide_body<D2Q9, float, S, false>(insts, b2i, pc, wm, K, hflip, Rec<float>{}, base + sub, tid);
}

// One block of 1024 threads per CU (the potential stage's tile needs all
// of them and 64 KB of LDS); the bound keeps every stage at 128 VGPRs, four
// waves per SIMD.
//   pa: the launch arguments in device memory (k_persist_begin copies them).
template <typename S>
__global__ __launch_bounds__(P2NT, 4) void k_persistent(const Inst *__restrict__ insts, const PersistArgs *pa) {
  const cptr<PersistArgs> a = cst(pa);
  const int L = a->K / 4, hflip = L & 1, n_steps = a->n_steps;
  const long long step0 = a->step0;
  unsigned passed = 0;
  for (int s = 0; s < n_steps; ++s) {
    const int pc = (int)((step0 + s) & 1);
    ps_moments<S>(insts, pa, pc);
    if (!grid_barrier(a, passed)) return;
    for (int l = 0; l < L; ++l) {
      ps_potential(insts, pa, pc, l);
      if (!grid_barrier(a, passed)) return;
    }
    ps_mu(insts, pa, pc, hflip);
    if (!grid_barrier(a, passed)) return;
    ps_collide<S>(insts, pa, pc, hflip, s == n_steps - 1 ? 1 : 0);
    if (!grid_barrier(a, passed)) return;
  }
}

// Before a launch: the launch arguments into device memory and the
// barrier words cleared (a kernel, not a copy and a memset).
__global__ void k_persist_begin(PersistArgs a, PersistArgs *dst) {
  if (threadIdx.x == 0) {
    *dst = a;
    *a.bar = 0u;
    *a.fail = 0;
  }
}

}  // namespace lbm

#endif
