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

}  // namespace pcpm
