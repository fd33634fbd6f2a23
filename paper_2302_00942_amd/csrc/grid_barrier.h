// Grid-wide barrier for the cooperative kernels (device code only; included
// by the HIP sources that launch with hipLaunchCooperativeKernel).
#pragma once

#include <hip/hip_runtime.h>

#include "rfd_internal.h"

namespace rfd {

// A relaxed agent-scope store (global_store ... sc1 on gfx950): coherent at
// device scope once acknowledged, with no L2 write-back.
__device__ __forceinline__ void gst_agent(double* p, double v) {
  __hip_atomic_store((__attribute__((address_space(1))) double*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Two-level counter barrier over a cooperative grid. Workgroups arrive on the
// counter of their group of kBarGroup (128-byte apart lines); the last arrival
// of a group (seen from the returned count) bumps the top counter, which every
// workgroup polls; a grid of one group polls its group counter instead.
// Counters only grow: round r waits for r * groups top arrivals (r * nblocks
// group arrivals for one group).
//
// Visibility of the phase outputs: every one of them is written with a
// relaxed agent-scope store (`st`, global_store ... sc1), which is coherent at
// device scope once acknowledged, and every wave waits for its own stores
// before the workgroup arrives, so an arrival is counted only after its
// workgroup's outputs are visible to every XCD: no L2 write-back fence is
// needed (with plain stores, the agent-scope release fence's L2 write-back at
// every arrival cost about 31 us of a 180 us phi_1 call at m = 256). The poll
// is relaxed and followed by an agent-scope acquire fence (the L2 and L1
// invalidates that drop lines older than the phase), and every wave drops its
// L1 lines after the wait.
//
// The wait is bounded: on timeout the flag gets bit 2 and the workgroup
// proceeds, so every wave always exits. The counters start at zero (the plan
// zeroes them when it is created) and every launch leaves them at zero: after
// its last wait each workgroup arrives on an exit counter (word 1), and the
// last arrival, which knows that no workgroup of the launch reads a counter
// again, clears them all, so no clearing kernel runs between launches on a
// stream.
constexpr int kBarGroup = 32;
constexpr int kBarStride = 32;        // unsigned words between counters (128 bytes)
constexpr int kBarWords = kBarStride * (1 + 256 / kBarGroup);
static_assert(kBarWords <= kBarrierWords, "barrier counters exceed the plan's buffer");

struct GridBarrier {
  unsigned* ctr;
  unsigned nblocks;
  unsigned round;
  int* flag;
  __device__ __forceinline__ void sync() {
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's stores are acknowledged
    __syncthreads();
    if (threadIdx.x == 0) {
      ++round;
      const unsigned g = blockIdx.x / kBarGroup;
      const unsigned groups = (nblocks + kBarGroup - 1) / kBarGroup;
      const unsigned gsz = (g + 1 < groups) ? kBarGroup : nblocks - g * kBarGroup;
      const unsigned old =
          __hip_atomic_fetch_add(ctr + kBarStride * (1 + g), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      // one group: its counter is the top (no second arrival)
      unsigned* const top = groups == 1 ? ctr + kBarStride : ctr;
      if (groups > 1 && old + 1 == round * gsz) __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = groups == 1 ? round * nblocks : round * groups;
      unsigned spins = 0;
      while (__hip_atomic_load(top, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1u << 24)) {
          __hip_atomic_fetch_or(flag, 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    asm volatile("buffer_inv sc0" ::: "memory");  // drop this CU's L1 lines
  }
  // a phase output read by other workgroups after sync
  __device__ __forceinline__ void st(double* p, double v) const { gst_agent(p, v); }
  // Called once by every workgroup after its last sync.
  __device__ __forceinline__ void finish() {
    if (threadIdx.x != 0) return;
    const unsigned old = __hip_atomic_fetch_add(ctr + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 != nblocks) return;
    const unsigned groups = (nblocks + kBarGroup - 1) / kBarGroup;
    for (unsigned g = 0; g < groups; ++g)
      __hip_atomic_store(ctr + kBarStride * (1 + g), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(ctr + 1, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
};



}  // namespace rfd
