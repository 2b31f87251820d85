// Device helpers shared by the iteration kernels (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "pcpm_internal.hpp"

namespace pcpm {

// Sum N FP64 values over the workgroup; results are valid in thread 0.
template <int BS, int N>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off);
  }
  __shared__ double sh[N * (BS / kWave)];
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) sh[N * w + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      v[i] = 0.0;
      for (int k = 0; k < BS / kWave; ++k) v[i] += sh[N * k + i];
    }
  }
}

// The same for G independent groups of BS threads in one workgroup of G*BS
// (group g = threadIdx.x / BS); valid in each group's first thread, summed in
// exactly the order of block_sum<BS>.  Every thread of the workgroup calls it.
template <int BS, int G, int N>
__device__ __forceinline__ void group_sum(double (&v)[N]) {
  if constexpr (G == 1) {
    block_sum<BS, N>(v);
  } else {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], off);
    }
    __shared__ double sh[G][N * (BS / kWave)];
    const int g = threadIdx.x / BS, t = threadIdx.x % BS, w = t / kWave;
    if ((t & (kWave - 1)) == 0) {
#pragma unroll
      for (int i = 0; i < N; ++i) sh[g][N * w + i] = v[i];
    }
    __syncthreads();
    if (t == 0) {
#pragma unroll
      for (int i = 0; i < N; ++i) {
        v[i] = 0.0;
        for (int k = 0; k < BS / kWave; ++k) v[i] += sh[g][N * k + i];
      }
    }
  }
}

// Largest of a non-negative value over the workgroup; valid in thread 0.
template <int BS>
__device__ __forceinline__ double block_max(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  __shared__ double sh[BS / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < BS / kWave; ++k) v = fmax(v, sh[k]);
  return v;
}

// The same for G groups of BS threads; valid in each group's first thread.
template <int BS, int G>
__device__ __forceinline__ double group_max(double v) {
  if constexpr (G == 1) {
    return block_max<BS>(v);
  } else {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
    __shared__ double sh[G][BS / kWave];
    const int g = threadIdx.x / BS, t = threadIdx.x % BS;
    if ((t & (kWave - 1)) == 0) sh[g][t / kWave] = v;
    __syncthreads();
    if (t == 0)
      for (int k = 0; k < BS / kWave; ++k) v = fmax(v, sh[g][k]);
    return v;
  }
}

// Fixed-point scale for sums of updates bounded by `bound` (the largest
// iterate value): 50 - ceil(log2(bound)), so every update times 2^sh stays
// at most 2^50, capped by `cap` (the sums' own bound).  Zero and negative
// shifts are valid (units of 2^-sh >= 1 for vectors of large values).
__device__ __forceinline__ int fx_shift_for(double bound, int cap) {
  int e = 0;
  if (bound > 0.0 && isfinite(bound)) e = static_cast<int>(ceil(log2(bound)));
  return min(cap, 50 - e);
}

// Conversion of an FP32 update to a signed integer in units of 2^-sh,
// rounded to nearest: v * 2^sh + 1.5*2^52 is formed by one FP64 FMA (exact
// product, one rounding) and the integer is read from the low mantissa bits.
// Valid for |v| * 2^sh < 2^51, which the choice of sh guarantees for every
// finite update; the result then carries the update to within 2^-(sh+1).
struct FixedConv {
  double scale;
  __device__ explicit FixedConv(int sh) : scale(ldexp(1.0, sh)) {}
  __device__ __forceinline__ int64_t operator()(float v) const {
    constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52
    const double y = fma(static_cast<double>(v), scale, kMagic);
    return __double_as_longlong(y) - __double_as_longlong(kMagic);
  }
  // the same for an FP64 value (an exact product of two FP32 values)
  __device__ __forceinline__ int64_t operator()(double v) const {
    constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52
    const double y = fma(v, scale, kMagic);
    return __double_as_longlong(y) - __double_as_longlong(kMagic);
  }
};

// Sum of the cnt fixed-point values base[c * stride], c = 0..cnt-1, with
// eight loads in flight (the partial slices of a split bin).  Integer
// addition modulo 2^64, so the result does not depend on the grouping.
__device__ __forceinline__ int64_t sum_slices(const int64_t* __restrict__ base, int cnt, int64_t stride) {
  uint64_t s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int c = 0;
  for (; c + 8 <= cnt; c += 8) {
#pragma unroll
    for (int j = 0; j < 8; ++j) s[j] += static_cast<uint64_t>(base[static_cast<int64_t>(c + j) * stride]);
  }
  for (; c < cnt; ++c) s[0] += static_cast<uint64_t>(base[static_cast<int64_t>(c) * stride]);
  return static_cast<int64_t>(((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7])));
}

// ---- persistent launches ---------------------------------------------------------
// A cooperative launch keeps every workgroup resident, so workgroups can wait
// for each other.  Every wait polls at most spin_limit times; a workgroup
// that runs out raises ps->err, and every wait returns at once when it sees
// err, so all workgroups leave their loops and the kernel ends.  Agent-scope
// fences around the barrier make the writes before it (which sit in the
// writer's XCD L2) visible to the readers after it, on any XCD.

__device__ __forceinline__ uint32_t ld_acquire(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ld_acquire(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier.  The last workgroup to arrive runs on_last() (thread 0,
// before releasing the others: counters reset there are seen by every
// workgroup after the barrier).  Returns false if a wait gave up.
// Every wave waits for its own memory operations to complete (its stores
// have reached its XCD's L2), so that thread 0's agent-scope release fence
// after the workgroup barrier writes them back with that L2's other lines.
__device__ __forceinline__ void wg_stores_done() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

template <class OnLast>
__device__ __forceinline__ bool grid_sync(PSync* ps, uint32_t spin_limit, OnLast on_last) {
  __shared__ int s_ok;
  wg_stores_done();
  if (threadIdx.x == 0) {
    int ok = 1;
    const uint32_t gen = ld_acquire(&ps->bar_gen);
    __threadfence();  // release this workgroup's writes
    const uint32_t arrived = __hip_atomic_fetch_add(&ps->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == gridDim.x - 1) {
      on_last();
      __hip_atomic_store(&ps->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ps->bar_gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      uint32_t spins = 0;
      while (ld_acquire(&ps->bar_gen) == gen) {
        if (ld_acquire(&ps->err) != 0 || ++spins > spin_limit) {
          __hip_atomic_store(&ps->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __threadfence();  // acquire the other workgroups' writes
    if (ld_acquire(&ps->err) != 0) ok = 0;
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Thread 0 waits until *ctr reaches target (other workgroups' release-ordered
// increments; counts compared modulo 2^32, so a counter may run over a whole
// solve); returns false (for the whole workgroup) if the wait gave up.
__device__ __forceinline__ bool wait_at_least(PSync* ps, const int32_t* ctr, int32_t target, uint32_t spin_limit) {
  __shared__ int s_ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    int ok = 1;
    uint32_t spins = 0;
    while (static_cast<int32_t>(static_cast<uint32_t>(ld_acquire(ctr)) - static_cast<uint32_t>(target)) < 0) {
      if (ld_acquire(&ps->err) != 0 || ++spins > spin_limit) {
        __hip_atomic_store(&ps->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __threadfence();
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Thread 0 takes the next unit of a shared counter; the whole workgroup gets
// it.  Two barriers: every thread has read the previous unit before the next
// one is published.
__device__ __forceinline__ int32_t grab(int32_t* ctr, int32_t count = 1) {
  __shared__ int32_t s_unit;
  __syncthreads();
  if (threadIdx.x == 0) s_unit = atomicAdd(ctr, count);
  __syncthreads();
  return s_unit;
}

// Thread 0 counts `count` finished units into *ctr with release order (after
// the workgroup's writes); returns the count before them to the whole
// workgroup.
__device__ __forceinline__ int32_t publish(int32_t* ctr, int32_t count = 1) {
  __shared__ int32_t s_old;
  wg_stores_done();
  if (threadIdx.x == 0) {
    __threadfence();
    s_old = __hip_atomic_fetch_add(ctr, count, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
  }
  __syncthreads();
  return s_old;
}

// Next scatter item of a workgroup: the items are dealt to the XCDs in
// contiguous ranges, as xcd_block does for one launch per phase (workgroup b
// runs on XCD b % 8), and the workgroups of an XCD take its range in order
// from a counter of their own.  Returns -1 when the range is used up.
__device__ __forceinline__ int32_t grab_scatter(PSync* ps, int32_t nitems) {
  const int x = static_cast<int>(blockIdx.x % kXcds);
  const int per = nitems / static_cast<int>(kXcds), rem = nitems % static_cast<int>(kXcds);
  const int len = per + (x < rem ? 1 : 0);
  const int j = grab(&ps->sc_next[x]);
  return j < len ? x * per + min(x, rem) + j : -1;
}

}  // namespace pcpm
