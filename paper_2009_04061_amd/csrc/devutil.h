// Device-side helpers shared by the kernel files: wave64 and workgroup scans
// and reductions, and small search routines.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gpa {

constexpr int kWave = 64;

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// inclusive scan over the 64 lanes of a wavefront
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const unsigned lane = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    T o = __shfl_up(v, d, kWave);
    if (lane >= (unsigned)d) v += o;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, d, kWave));
  return v;
}

// Workgroup barrier that orders LDS accesses only: global loads already
// issued stay in flight across it (__syncthreads waits for them as well).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <bool kLdsOnly>
__device__ __forceinline__ void wg_barrier() {
  if (kLdsOnly) lds_barrier();
  else __syncthreads();
}

// Exclusive scan across a workgroup of NT threads (NT a multiple of 64);
// `smem` holds NT/64 + 1 elements.  Returns the exclusive prefix of this
// thread and writes the workgroup total to *total.  kLdsOnly: its barriers
// order LDS only (see lds_barrier).
template <int NT, typename T, bool kLdsOnly = false>
__device__ __forceinline__ T block_excl_scan(T v, T *smem, T *total) {
  static_assert(NT % kWave == 0, "block must be whole waves");
  constexpr int NW = NT / kWave;
  const unsigned tid = threadIdx.x;
  const unsigned w = tid / kWave, lane = tid % kWave;
  T inc = wave_incl_scan(v);
  if (lane == kWave - 1) smem[w] = inc;
  wg_barrier<kLdsOnly>();
  if (tid == 0) {
    T run = 0;
    for (int k = 0; k < NW; ++k) {
      T t = smem[k];
      smem[k] = run;
      run += t;
    }
    smem[NW] = run;
  }
  wg_barrier<kLdsOnly>();
  T res = smem[w] + inc - v;
  *total = smem[NW];
  wg_barrier<kLdsOnly>();
  return res;
}

// first index in [lo, hi) with a[idx] >= key (a sorted ascending)
__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t *a, uint32_t lo, uint32_t hi,
                                                    uint32_t key) {
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// largest index in [lo, hi) with a[idx] <= key (a nondecreasing, a[lo] <= key)
__device__ __forceinline__ uint32_t upper_index_u32(const uint32_t *a, uint32_t lo, uint32_t hi,
                                                    uint32_t key) {
  while (hi - lo > 1) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (a[mid] <= key) lo = mid;
    else hi = mid;
  }
  return lo;
}

}  // namespace gpa
