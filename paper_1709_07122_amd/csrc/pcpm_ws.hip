// Learned warm start: per-node graph features, a 3-layer MLP (width 64,
// ReLU) that predicts log(n * PR*(v)), its BF16/FP32 training kernels, and the
// normalisation of the prediction into a start vector.
//
// Features:
//   0 log1p(indeg)   1 log1p(outdeg)   2 dangling flag
//   3 log(n * PR_1(v)) = log((1-d) + d * (s1(v) + n_dangling/n)), the first
//     iterate of Eq. 1 from the uniform vector; s1(v) = sum_{u->v} 1/outdeg(u)
//     is the one-SpMV aggregate of the in-neighbours' degrees
//   4..7 zero padding (the MFMA K-block is 8 wide)
// In-degrees are counted once per handle from the destination-ID bins, and
// features 0 and 1 are kept per handle from then on; the first iterate is one
// PCPM iteration (scatter + gather + apply) from the uniform vector.
//
// Parameters (FP32 master copy, 4801 floats): W1[64][8], b1[64], W2[64][64],
// b2[64], w3[64], b3.  Compute is BF16 x BF16 -> FP32: weights, features and
// hidden activations are rounded to BF16 where they enter a product.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <mutex>
#include <vector>

#include "pcpm_device.hpp"
#include "pcpm_internal.hpp"

namespace pcpm {

constexpr int kF = PCPM_WS_FEATURES;
constexpr int kH = PCPM_WS_HIDDEN;
constexpr int kOW1 = 0, kOB1 = kH * kF, kOW2 = kOB1 + kH, kOB2 = kOW2 + kH * kH, kOW3 = kOB2 + kH, kOB3 = kOW3 + kH;
static_assert(kOB3 + 1 == PCPM_WS_PARAMS, "parameter layout");

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v16f __attribute__((ext_vector_type(16)));

// Round to the nearest BF16 (ties to even) with gfx950's conversion
// instruction (v_cvt_pk_bf16_f32), two values at a time where possible.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pack2(float a, float b) {
  const float2 f = make_float2(a, b);
  const bf16x2 h = __builtin_convertvector(*reinterpret_cast<const float __attribute__((ext_vector_type(2)))*>(&f), bf16x2);
  return __builtin_bit_cast(uint32_t, h);
}
__device__ __forceinline__ float bf16_round(float f) {
  return __uint_as_float(static_cast<uint32_t>(__builtin_bit_cast(uint16_t, static_cast<__bf16>(f))) << 16);
}
// four values as an MFMA operand (two packed registers)
__device__ __forceinline__ v4s bf16_op(float a, float b, float c, float d) {
  return __builtin_bit_cast(v4s, make_uint2(bf16_pack2(a, b), bf16_pack2(c, d)));
}

// ---- features -------------------------------------------------------------------
// In-degrees: one workgroup per gather item counts the destination IDs of its
// range of a bin in an LDS slice of 32-bit counters, reading 1024-ID tiles
// with eight 4-byte loads per lane as the gather does; a whole bin stores its
// counts, the items of a split bin add theirs to the (zeroed) global array.
constexpr int kCountBlock = 1024;

__global__ __launch_bounds__(kCountBlock) void k_ws_count(int64_t n, int s, const Item* __restrict__ items,
                                                         const uint16_t* __restrict__ did,
                                                         uint32_t* __restrict__ indeg) {
  extern __shared__ uint32_t cnt[];
  const Item it = items[blockIdx.x];
  const int64_t q = int64_t{1} << s;
  const int64_t v0 = static_cast<int64_t>(it.part) << s;
  const int qn = static_cast<int>(min(q, n - v0));
  const uint32_t qmask = static_cast<uint32_t>(q - 1);  // also drops the message and segment flags
  for (int i = threadIdx.x; i < qn; i += kCountBlock) cnt[i] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t lo = it.lo, hi = it.hi;
  const int64_t t_end = (hi + kTile - 1) / kTile;
  constexpr int kNW = kCountBlock / kWave;
  int64_t t = lo / kTile + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  uint32_t w[kPairs], wn[kPairs];
  if (t < t_end) load_tile_words(did + t * kTile, lane, w);
  for (; t < t_end; t += kNW) {
    const int64_t tb = t * kTile;
    // the next tile's IDs are in flight during this tile's adds
    if (t + kNW < t_end) load_tile_words(did + (t + kNW) * kTile, lane, wn);
    uint32_t x[kSub];
    unpack_tile(w, x);
    if (tb >= lo && tb + kTile <= hi) {
#pragma unroll
      for (int j = 0; j < kSub; ++j) atomicAdd(&cnt[x[j] & qmask], 1u);
    } else {
#pragma unroll
      for (int j = 0; j < kSub; ++j) {
        const int64_t e = tb + j * kWave + lane;
        if (e >= lo && e < hi) atomicAdd(&cnt[x[j] & qmask], 1u);
      }
    }
#pragma unroll
    for (int j = 0; j < kPairs; ++j) w[j] = wn[j];
  }
  __syncthreads();
  if (it.aux < 0) {
    for (int i = threadIdx.x; i < qn; i += kCountBlock) indeg[v0 + i] = cnt[i];
  } else {
    for (int i = threadIdx.x; i < qn; i += kCountBlock) {
      const uint32_t c = cnt[i];
      if (c) atomicAdd(&indeg[v0 + i], c);
    }
  }
}

__global__ __launch_bounds__(256) void k_ws_prep(uint32_t* __restrict__ indeg, float* __restrict__ x0, int64_t n,
                                                 float uni) {
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    if (indeg) indeg[v] = 0u;
    x0[v] = uni;
  }
}

// The graph's own features of every node, formed once per handle:
// (log1p(in-degree), log1p(out-degree)).  Most degrees are small: each
// workgroup first tabulates log1pf(k) for k < kLogTable in LDS (the same
// function, so the same values) and computes only larger ones directly.
constexpr int kLogTable = 1024;
constexpr int kStaticBlocks = 1024;

__device__ __forceinline__ float log1p_deg(const float* __restrict__ tab, uint32_t k) {
  return k < static_cast<uint32_t>(kLogTable) ? tab[k] : log1pf(static_cast<float>(k));
}

__global__ __launch_bounds__(256) void k_ws_static(const uint32_t* __restrict__ indeg,
                                                   const int32_t* __restrict__ outdeg, int64_t n,
                                                   float2* __restrict__ sfeat) {
  __shared__ float tab[kLogTable];
  for (int k = threadIdx.x; k < kLogTable; k += blockDim.x) tab[k] = log1pf(static_cast<float>(k));
  __syncthreads();
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += static_cast<int64_t>(gridDim.x) * blockDim.x)
    sfeat[v] = make_float2(log1p_deg(tab, indeg[v]), log1p_deg(tab, static_cast<uint32_t>(outdeg[v])));
}

// The four features of node v (the other four are zero).
struct FeatSrc {
  const float2* sfeat;  // log1p of in- and out-degree
  const uint32_t* dmask;
  const float* pr1;     // first iterate
  float fn;             // n
};

__device__ __forceinline__ float log_n_pr1(const FeatSrc& fs, float pr1) {
  return logf(pr1 * fs.fn);  // FP32 is ample: the network sees the value rounded to BF16
}

__device__ __forceinline__ float4 node_features(const FeatSrc& fs, int64_t v) {
  const float2 sf = fs.sfeat[v];
  return make_float4(sf.x, sf.y, static_cast<float>((fs.dmask[v >> 5] >> (v & 31)) & 1u), log_n_pr1(fs, fs.pr1[v]));
}

__global__ __launch_bounds__(256) void k_ws_features(float* __restrict__ feat, const FeatSrc fs, int64_t n) {
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    float4* out = reinterpret_cast<float4*>(feat + kF * v);
    out[0] = node_features(fs, v);
    out[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
}

// ---- inference on MFMA ------------------------------------------------------------
// One wavefront evaluates 32 nodes with transposed products, so the output of
// each layer is already the B operand of the next:
//   h1^T = W1 X^T + b1 (2 MFMA 32x32x8),  h2^T = W2 h1^T + b2 (8 MFMA
//   32x32x16),  y = w3 . h2 + b3 (BF16 dot products).
// Lane l owns node l%32.  In a 32x32 output block its value v is row
// 8(v/4) + 4(l/32) + v%4; values 8p .. 8p+7 of hidden block c are therefore
// rows 16t + 8(i/4) + 4(l/32) + i%4 (t = 2c + p, i = 0..7), which is what the
// lane supplies as B operand slot i of K-block t of the next product, and the
// A operand (W2) takes its columns in that same order.  The biases enter as
// the accumulator input, ReLU acts on the packed BF16 values (as 16-bit
// integers the negative ones, -0 included, are exactly those below zero,
// and rounding commutes with it), and the output layer is 16 two-wide BF16
// dot products per lane with FP32 sums.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v2s __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t relu_bf16x2(float a, float b) {
  const v2s z = {0, 0};
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(v2s, bf16_pack2(a, b)), z));
}

constexpr int kFwdBlock = 256;
constexpr int kFwdMaxBlocks = 2048;

// One node's inputs to the forward as loaded by this lane (fused: the low
// half loads the node's per-handle features, first iterate and dangling
// flag, the high half nothing; otherwise this lane's four features).
struct FwdRaw {
  float4 f;
  float pr1;
};

template <bool kFused>
__device__ __forceinline__ FwdRaw load_fwd_raw(const float* __restrict__ feat, const FeatSrc& fs, int64_t node,
                                               int64_t n, int half) {
  FwdRaw r = {make_float4(0.0f, 0.0f, 0.0f, 0.0f), 1.0f};
  if (node >= n) return r;
  if constexpr (kFused) {
    if (half == 0) {
      const float2 sf = fs.sfeat[node];
      r.f = make_float4(sf.x, sf.y, static_cast<float>((fs.dmask[node >> 5] >> (node & 31)) & 1u), 0.0f);
      r.pr1 = fs.pr1[node];
    }
  } else {
    r.f = *reinterpret_cast<const float4*>(feat + kF * node + 4 * half);
  }
  return r;
}

// kFused: the features are formed from their sources (in-degrees, out-degrees,
// dangling mask, first iterate) as k_ws_features forms them, instead of read
// from a feature matrix; the prediction is the same bit for bit.
template <bool kFused>
__global__ __launch_bounds__(kFwdBlock) void k_ws_forward(const float* __restrict__ P, const float* __restrict__ feat,
                                                          const FeatSrc fs, int64_t n, float* __restrict__ yhat) {
  const int l = threadIdx.x & (kWave - 1);
  const int col = l & 31, half = l >> 5;
  // A fragments: row 32*ob + col; W1 columns 4*half .. +3, W2 columns in the
  // B operand's slot order.  W2's fragments and w3 wait in LDS (written by
  // the first wavefront) and are read where they are used, which keeps the
  // kernel at three wavefronts per SIMD; W1 and the biases stay in registers.
  __shared__ uint4 s_a2[2][4][kWave];
  __shared__ uint4 s_w3[2][4];  // [half]: w3 of the half's 32 rows as packed pairs
  v4s a1[2];
  v16f c1[2], c2[2];
#pragma unroll
  for (int ob = 0; ob < 2; ++ob) {
    const int r = 32 * ob + col;
    const float* w1 = P + kOW1 + r * kF + 4 * half;
    a1[ob] = bf16_op(w1[0], w1[1], w1[2], w1[3]);
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int row = 32 * ob + 8 * (v / 4) + 4 * half + (v % 4);
      c1[ob][v] = P[kOB1 + row];
      c2[ob][v] = P[kOB2 + row];
    }
  }
  if (threadIdx.x < kWave) {
#pragma unroll
    for (int ob = 0; ob < 2; ++ob) {
      const int r = 32 * ob + col;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const float* w2 = P + kOW2 + r * kH + 16 * t + 4 * half;
        s_a2[ob][t][l] = make_uint4(bf16_pack2(w2[0], w2[1]), bf16_pack2(w2[2], w2[3]), bf16_pack2(w2[8], w2[9]),
                                    bf16_pack2(w2[10], w2[11]));
      }
    }
    if (col == 0) {
      uint32_t pk[16];
#pragma unroll
      for (int ob = 0; ob < 2; ++ob)
#pragma unroll
        for (int v = 0; v < 16; v += 2) {
          const int row = 32 * ob + 8 * (v / 4) + 4 * half + (v % 4);
          pk[8 * ob + v / 2] = bf16_pack2(P[kOW3 + row], P[kOW3 + row + 1]);
        }
#pragma unroll
      for (int i = 0; i < 4; ++i) s_w3[half][i] = make_uint4(pk[4 * i], pk[4 * i + 1], pk[4 * i + 2], pk[4 * i + 3]);
    }
  }
  __syncthreads();
  const float b3 = P[kOB3];
  // The inputs of the wavefront's next 32 nodes are loaded while the
  // current ones go through the network.
  const int64_t stride = static_cast<int64_t>(gridDim.x) * (kFwdBlock / kWave) * 32;
  int64_t base = (static_cast<int64_t>(blockIdx.x) * (kFwdBlock / kWave) + threadIdx.x / kWave) * 32;
  FwdRaw raw = load_fwd_raw<kFused>(feat, fs, base + col, n, half);
  for (; base < n; base += stride) {
    // LDS reads stay inside the loop (not hoisted into registers)
    __asm__ volatile("" ::: "memory");
    const int64_t node = base + col;
    const FwdRaw cur = raw;
    raw = load_fwd_raw<kFused>(feat, fs, base + stride + col, n, half);
    float4 fv = cur.f;
    if constexpr (kFused) {
      if (half == 0 && node < n) fv.w = log_n_pr1(fs, cur.pr1);
    }
    const v4s bx = bf16_op(fv.x, fv.y, fv.z, fv.w);
    uint32_t hp[2][8];  // relu(h1) as packed BF16 pairs (v, v+1)
#pragma unroll
    for (int ob = 0; ob < 2; ++ob) {
      const v16f h1 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1[ob], bx, c1[ob], 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 16; v += 2) hp[ob][v / 2] = relu_bf16x2(h1[v], h1[v + 1]);
    }
    v16f h2[2] = {c2[0], c2[1]};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const v8bf b = __builtin_bit_cast(
          v8bf, make_uint4(hp[t / 2][4 * (t % 2)], hp[t / 2][4 * (t % 2) + 1], hp[t / 2][4 * (t % 2) + 2],
                           hp[t / 2][4 * (t % 2) + 3]));
#pragma unroll
      for (int ob = 0; ob < 2; ++ob)
        h2[ob] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, s_a2[ob][t][l]), b, h2[ob], 0, 0, 0);
    }
    uint32_t w3p[16];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint4 q = s_w3[half][i];
      w3p[4 * i] = q.x;
      w3p[4 * i + 1] = q.y;
      w3p[4 * i + 2] = q.z;
      w3p[4 * i + 3] = q.w;
    }
    float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int ob = 0; ob < 2; ++ob) {
#pragma unroll
      for (int v = 0; v < 16; v += 2)
        part[v / 4] = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, relu_bf16x2(h2[ob][v], h2[ob][v + 1])),
                                                      __builtin_bit_cast(bf16x2, w3p[8 * ob + v / 2]), part[v / 4],
                                                      false);
    }
    float y = (part[0] + part[1]) + (part[2] + part[3]);
    y += __shfl_xor(y, 32);  // lanes l and l^32 hold the two halves of node col's rows
    if (half == 0 && node < n) yhat[node] = y + b3;
  }
}

// ---- start vector: softmax over nodes --------------------------------------------
// k_ws_soft_part: every thread keeps a running maximum m and the sum s of
// exp(y - m) over its nodes (FP64; s is rescaled when m grows), and the
// workgroup combines its threads' pairs into one (M, S, non-finite flag).
// k_ws_soft_final: one workgroup combines the kSoftBlocks partial pairs.
// k_ws_soft_norm writes exp(y - M) / S, or the uniform vector if a
// prediction was non-finite or S is not a positive finite number.
constexpr int kSoftBlocks = 1024;
constexpr int kSoftThreads = 256;

struct SoftPair {
  double m, s, bad;
};

__device__ __forceinline__ SoftPair soft_combine(SoftPair a, SoftPair b) {
  const double m = fmax(a.m, b.m);
  SoftPair r;
  r.m = m;
  r.s = (a.s > 0.0 ? a.s * exp(a.m - m) : 0.0) + (b.s > 0.0 ? b.s * exp(b.m - m) : 0.0);
  r.bad = fmax(a.bad, b.bad);
  return r;
}

// workgroup-wide combination of one pair per thread; the result in every thread
__device__ __forceinline__ SoftPair soft_block(SoftPair p) {
  __shared__ double sh[3][kSoftThreads / kWave];
  for (int off = kWave / 2; off > 0; off >>= 1) {
    SoftPair o;
    o.m = __shfl_xor(p.m, off);
    o.s = __shfl_xor(p.s, off);
    o.bad = __shfl_xor(p.bad, off);
    p = soft_combine(p, o);
  }
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sh[0][w] = p.m;
    sh[1][w] = p.s;
    sh[2][w] = p.bad;
  }
  __syncthreads();
  SoftPair r = {sh[0][0], sh[1][0], sh[2][0]};
  for (int i = 1; i < kSoftThreads / kWave; ++i) r = soft_combine(r, SoftPair{sh[0][i], sh[1][i], sh[2][i]});
  return r;
}

__global__ __launch_bounds__(kSoftThreads) void k_ws_soft_part(const float* __restrict__ y, int64_t n,
                                                               double* __restrict__ red) {
  SoftPair p = {-INFINITY, 0.0, 0.0};
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * kSoftThreads + threadIdx.x; v < n;
       v += static_cast<int64_t>(gridDim.x) * kSoftThreads) {
    const float yv = y[v];
    if (!isfinite(yv)) {
      p.bad = 1.0;
      continue;
    }
    const double yd = static_cast<double>(yv);
    if (yd > p.m) {
      p.s = p.s * exp(p.m - yd) + 1.0;
      p.m = yd;
    } else {
      p.s += exp(yd - p.m);
    }
  }
  const SoftPair r = soft_block(p);
  if (threadIdx.x == 0) {
    red[3 * blockIdx.x] = r.m;
    red[3 * blockIdx.x + 1] = r.s;
    red[3 * blockIdx.x + 2] = r.bad;
  }
}

__global__ __launch_bounds__(kSoftThreads) void k_ws_soft_final(double* __restrict__ red) {
  SoftPair p = {-INFINITY, 0.0, 0.0};
  for (int i = threadIdx.x; i < kSoftBlocks; i += kSoftThreads)
    p = soft_combine(p, SoftPair{red[3 * i], red[3 * i + 1], red[3 * i + 2]});
  const SoftPair r = soft_block(p);
  if (threadIdx.x == 0) {
    red[3 * kSoftBlocks] = r.m;
    red[3 * kSoftBlocks + 1] = r.s;
    red[3 * kSoftBlocks + 2] = r.bad;
  }
}

__global__ __launch_bounds__(kSoftThreads) void k_ws_soft_norm(const float* __restrict__ y, int64_t n,
                                                               const double* __restrict__ red,
                                                               float* __restrict__ pr0, int32_t* __restrict__ flag) {
  const SoftPair r = {red[3 * kSoftBlocks], red[3 * kSoftBlocks + 1], red[3 * kSoftBlocks + 2]};
  const bool fallback = r.bad > 0.0 || !(r.s > 0.0) || !isfinite(r.s);
  if (blockIdx.x == 0 && threadIdx.x == 0) *flag = fallback ? 1 : 0;
  const double inv = fallback ? 0.0 : 1.0 / r.s;
  const float uni = static_cast<float>(1.0 / static_cast<double>(n));
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * kSoftThreads + threadIdx.x; v < n;
       v += static_cast<int64_t>(gridDim.x) * kSoftThreads)
    pr0[v] = fallback ? uni : static_cast<float>(exp(static_cast<double>(y[v]) - r.m) * inv);
}

// ---- training: loss gradient over a minibatch -------------------------------------
// Loss = mean over the minibatch of (yhat - target)^2.  The forward pass
// rounds exactly as k_ws_forward does (BF16 weights, features and hidden
// activations; FP32 sums).  One workgroup takes chunks of 64 samples: four
// threads per sample for the activations, then every thread accumulates its
// own 16 + 2 (+3) parameter gradients over the chunk.  Partial gradients per
// workgroup are summed in a fixed order by k_ws_grad_reduce.
constexpr int kGradBlock = 256;
constexpr int kChunk = 64;

__global__ __launch_bounds__(kGradBlock) void k_ws_grad(const float* __restrict__ P, const float* __restrict__ feat,
                                                        const float* __restrict__ target, int64_t rows,
                                                        const int64_t* __restrict__ idx, int64_t b, float inv_b,
                                                        float* __restrict__ part, double* __restrict__ loss_part) {
  __shared__ float W1s[kH * kF], b1s[kH], W2s[kH * kH], b2s[kH], w3s[kH];
  __shared__ float xs[kChunk][kF + 1], h1s[kChunk][kH + 1], h2s[kChunk][kH + 1], dh2s[kChunk][kH + 1],
      dh1s[kChunk][kH + 1], dys[kChunk];
  const int tid = threadIdx.x;
  for (int i = tid; i < kH * kF; i += kGradBlock) W1s[i] = bf16_round(P[kOW1 + i]);
  for (int i = tid; i < kH * kH; i += kGradBlock) W2s[i] = bf16_round(P[kOW2 + i]);
  for (int i = tid; i < kH; i += kGradBlock) {
    b1s[i] = P[kOB1 + i];
    b2s[i] = P[kOB2 + i];
    w3s[i] = bf16_round(P[kOW3 + i]);
  }
  const float b3 = P[kOB3];
  const int s = tid / 4, qtr = tid % 4;  // sample of the chunk, quarter of the hidden units
  const int gi = tid / 4;                 // dW2 row owned by this thread
  float gW2[16] = {}, gW1[2] = {}, gb1 = 0.0f, gb2 = 0.0f, gw3 = 0.0f, gb3 = 0.0f;
  double loss = 0.0, bad = 0.0;
  __syncthreads();
  for (int64_t c0 = static_cast<int64_t>(blockIdx.x) * kChunk; c0 < b; c0 += static_cast<int64_t>(gridDim.x) * kChunk) {
    const int64_t ri = c0 + s < b ? idx[c0 + s] : -1;
    const bool in_range = ri >= 0 && ri < rows;
    if (c0 + s < b && !in_range && qtr == 0) bad += 1.0;
    const bool valid = c0 + s < b && in_range;
    const int64_t row = valid ? ri : 0;
    for (int k = qtr * 2; k < qtr * 2 + 2; ++k) xs[s][k] = valid ? bf16_round(feat[kF * row + k]) : 0.0f;
    const float tgt = valid ? target[row] : 0.0f;
    __syncthreads();
    for (int j = 16 * qtr; j < 16 * qtr + 16; ++j) {
      float a = b1s[j];
      for (int k = 0; k < kF; ++k) a += W1s[j * kF + k] * xs[s][k];
      h1s[s][j] = bf16_round(fmaxf(a, 0.0f));
    }
    __syncthreads();
    float yp = 0.0f;
    for (int i = 16 * qtr; i < 16 * qtr + 16; ++i) {
      float a = b2s[i];
      for (int k = 0; k < kH; ++k) a += W2s[i * kH + k] * h1s[s][k];
      const float h2 = bf16_round(fmaxf(a, 0.0f));
      h2s[s][i] = h2;
      yp += w3s[i] * h2;
    }
    yp += __shfl_xor(yp, 1);
    yp += __shfl_xor(yp, 2);
    const float y = yp + b3;
    const float dy = valid ? 2.0f * (y - tgt) * inv_b : 0.0f;
    if (qtr == 0) {
      dys[s] = dy;
      if (valid) loss += static_cast<double>(y - tgt) * static_cast<double>(y - tgt);
    }
    for (int i = 16 * qtr; i < 16 * qtr + 16; ++i) dh2s[s][i] = h2s[s][i] > 0.0f ? w3s[i] * dy : 0.0f;
    __syncthreads();
    for (int k = 16 * qtr; k < 16 * qtr + 16; ++k) {
      float a = 0.0f;
      for (int i = 0; i < kH; ++i) a += W2s[i * kH + k] * dh2s[s][i];
      dh1s[s][k] = h1s[s][k] > 0.0f ? a : 0.0f;
    }
    __syncthreads();
    // parameter gradients of this chunk
    for (int ss = 0; ss < kChunk; ++ss) {
      const float d2 = dh2s[ss][gi];
#pragma unroll
      for (int c = 0; c < 16; ++c) gW2[c] += d2 * h1s[ss][16 * qtr + c];
#pragma unroll
      for (int c = 0; c < 2; ++c) gW1[c] += dh1s[ss][(2 * tid + c) / kF] * xs[ss][(2 * tid + c) % kF];
    }
    if (tid < kH) {
      for (int ss = 0; ss < kChunk; ++ss) {
        gb1 += dh1s[ss][tid];
        gb2 += dh2s[ss][tid];
        gw3 += dys[ss] * h2s[ss][tid];
      }
    }
    if (tid == 0)
      for (int ss = 0; ss < kChunk; ++ss) gb3 += dys[ss];
    __syncthreads();
  }
  float* out = part + static_cast<int64_t>(blockIdx.x) * PCPM_WS_PARAMS;
#pragma unroll
  for (int c = 0; c < 16; ++c) out[kOW2 + gi * kH + 16 * qtr + c] = gW2[c];
  out[kOW1 + 2 * tid] = gW1[0];
  out[kOW1 + 2 * tid + 1] = gW1[1];
  if (tid < kH) {
    out[kOB1 + tid] = gb1;
    out[kOB2 + tid] = gb2;
    out[kOW3 + tid] = gw3;
  }
  if (tid == 0) out[kOB3] = gb3;
  double sums[2] = {loss, bad};
  block_sum<kGradBlock>(sums);
  if (tid == 0) {
    loss_part[2 * blockIdx.x] = sums[0];
    loss_part[2 * blockIdx.x + 1] = sums[1];
  }
}

__global__ __launch_bounds__(256) void k_ws_grad_reduce(const float* __restrict__ part, int nparts,
                                                        const double* __restrict__ loss_part, float* __restrict__ grad,
                                                        double* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p < PCPM_WS_PARAMS) {
    float s = 0.0f;
    for (int w = 0; w < nparts; ++w) s += part[static_cast<int64_t>(w) * PCPM_WS_PARAMS + p];
    grad[p] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double l = 0.0, bad = 0.0;
    for (int w = 0; w < nparts; ++w) {
      l += loss_part[2 * w];
      bad += loss_part[2 * w + 1];
    }
    loss[0] = l;
    loss[1] = bad;
  }
}

// Adam (Kingma & Ba 2015) on the FP32 master weights, bias-corrected.
// The constants 1 - beta and the bias corrections are rounded from FP64 on
// the host: 1 - 0.999f in FP32 would be off by 1e-5 relative.
__global__ __launch_bounds__(256) void k_ws_adam(float* __restrict__ P, const float* __restrict__ g,
                                                 float* __restrict__ m, float* __restrict__ v, float lr, float b1,
                                                 float omb1, float b2, float omb2, float eps, float c1, float c2) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= PCPM_WS_PARAMS) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + omb1 * gp;
  const float vp = b2 * v[p] + omb2 * gp * gp;
  m[p] = mp;
  v[p] = vp;
  P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

__global__ __launch_bounds__(256) void k_ws_targets(const float* __restrict__ pr, int64_t n, float* __restrict__ y) {
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; v < n;
       v += static_cast<int64_t>(gridDim.x) * 256)
    y[v] = static_cast<float>(log(static_cast<double>(pr[v]) * static_cast<double>(n)));
}

// 32 nodes per wavefront, 4 wavefronts per workgroup
static unsigned forward_blocks(int64_t n) {
  const int64_t groups = (n + 31) / 32;
  return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((groups + 3) / 4, kFwdMaxBlocks)));
}

static FeatSrc feat_src(const pcpm_png* g) {
  return FeatSrc{g->ws_sfeat, g->dmask, g->ws_x + g->n, static_cast<float>(g->n)};
}

static unsigned grid_for(int64_t n) { return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192))); }

// Per-handle state of the warm start, formed on first use: the uniform
// vector and a buffer for the first iterate (ws_x), the in-degrees counted
// from the bins and the per-node features that depend on the graph alone.
static pcpm_status_t ws_prepare(pcpm_png* g, hipStream_t st) {
  const int64_t n = g->n;
  if (g->ws_sfeat) return PCPM_OK;
  if (!g->ws_x) PCPM_TRY(dalloc(g, &g->ws_x, 2 * n));
  float2* sfeat = nullptr;
  PCPM_TRY(dalloc(g, &sfeat, n));
  uint32_t* indeg = nullptr;
  if (dalloc(g, &indeg, n) != PCPM_OK) {
    dfree(g, sfeat);
    return PCPM_ERR_OOM;
  }
  static bool lds_set = false;
  if (!lds_set) {
    PCPM_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_ws_count),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (1 << kMaxLog2) * 4));
    lds_set = true;
  }
  // the count's time (the array's allocation above is not part of it)
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  const auto t0 = std::chrono::steady_clock::now();
  const float uni = static_cast<float>(1.0 / static_cast<double>(n));
  PCPM_LAUNCH("pcpm_ws_features", k_ws_prep, dim3(grid_for(n)), dim3(256), 0, st, indeg, g->ws_x, n, uni);
  if (g->n_ga)
    PCPM_LAUNCH("pcpm_ws_features", k_ws_count, dim3(static_cast<unsigned>(g->n_ga)), dim3(kCountBlock),
                static_cast<size_t>(g->q) * 4, st, n, g->part_log2, g->ga_items, g->did, indeg);
  PCPM_LAUNCH("pcpm_ws_features", k_ws_static,
              dim3(static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, kStaticBlocks)))),
              dim3(256), 0, st, indeg, g->outdeg, n, sfeat);
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  g->ws_indeg_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  dfree(g, indeg);  // freeing is not part of the count's time (hipFree waits for the device)
  g->ws_sfeat = sfeat;
  return PCPM_OK;
}

static pcpm_status_t ws_check_device_ptr(const void* p, const char* what) {
  hipPointerAttribute_t a;
  if (!p || hipPointerGetAttributes(&a, p) != hipSuccess ||
      !(a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged)) {
    (void)hipGetLastError();
    return set_error(PCPM_ERR_INVALID_ARG, "%s must be a device pointer", what);
  }
  return PCPM_OK;
}

// Minibatch gradient (k_ws_grad + k_ws_grad_reduce) with the caller's or
// the fixed scratch as `work`: 2 (parts + 1) doubles (per-workgroup loss and
// bad-index count, then the totals), then parts * PARAMS floats of
// per-workgroup partial gradients.  Every entry the kernels read is written
// by them first in the same call, so nothing needs clearing between calls.
static pcpm_status_t ws_backward(const float* params, const float* feat, const float* target, int64_t rows,
                                 const int64_t* idx, int64_t b, float* grad, float* work, double* loss,
                                 hipStream_t st) {
  PCPM_TRY(ws_check_device_ptr(params, "params"));
  PCPM_TRY(ws_check_device_ptr(feat, "feat"));
  PCPM_TRY(ws_check_device_ptr(target, "target"));
  PCPM_TRY(ws_check_device_ptr(idx, "idx"));
  PCPM_TRY(ws_check_device_ptr(grad, "grad"));
  const int parts = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>((b + kChunk - 1) / kChunk, 1024)));
  double* lpart = reinterpret_cast<double*>(work);
  double* ldev = lpart + 2 * parts;
  float* part = work + 4 * (parts + 1);
  PCPM_LAUNCH("pcpm_ws_backward", k_ws_grad, dim3(parts), dim3(kGradBlock), 0, st, params, feat, target, rows, idx,
              b, 1.0f / static_cast<float>(b), part, lpart);
  PCPM_LAUNCH("pcpm_ws_backward", k_ws_grad_reduce, dim3((PCPM_WS_PARAMS + 255) / 256), dim3(256), 0, st, part,
              parts, lpart, grad, ldev);
  double tot[2] = {0.0, 0.0};
  PCPM_TRY_HIP(hipMemcpyAsync(tot, ldev, 16, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  if (tot[1] != 0.0)
    return set_error(PCPM_ERR_INVALID_ARG, "%.0f minibatch indices outside [0, %lld)", tot[1],
                     static_cast<long long>(rows));
  *loss = tot[0] / static_cast<double>(b);
  return PCPM_OK;
}

// Fixed scratch of pcpm_ws_backward_noalloc: the workspace of
// pcpm_ws_backward for up to kNoAllocParts workgroups, i.e. minibatches of
// up to kNoAllocParts * kChunk samples (4.9 MB).  Every GPU the library runs
// on holds its own copy until the process ends.  On the host, `scratch`
// names a host-side stand-in, not device memory: kernels get the device
// address that hipGetSymbolAddress returns, looked up once per device.
constexpr int kNoAllocParts = 256;
constexpr int64_t kNoAllocMaxBatch = int64_t{kNoAllocParts} * kChunk;
constexpr int64_t kNoAllocFloats = int64_t{kNoAllocParts} * PCPM_WS_PARAMS + 4 * (kNoAllocParts + 1);
static __device__ __align__(256) float scratch[kNoAllocFloats];

static pcpm_status_t noalloc_scratch(float** out) {
  static std::mutex mu;
  static std::vector<float*> per_device;
  int dev = -1;
  PCPM_TRY_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  if (static_cast<int>(per_device.size()) <= dev) per_device.resize(static_cast<size_t>(dev) + 1, nullptr);
  if (!per_device[dev]) {
    void* ptr = nullptr;
    PCPM_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return set_error(PCPM_ERR_DEVICE, "no device address for the fixed scratch on device %d", dev);
    per_device[dev] = static_cast<float*>(ptr);
  }
  *out = per_device[dev];
  return PCPM_OK;
}

}  // namespace pcpm

extern "C" {

pcpm_status_t pcpm_ws_features(pcpm_png_t g, double d, float* feat, double* first_call_ms, void* stream) {
  using namespace pcpm;
  if (!g || !feat) return set_error(PCPM_ERR_INVALID_ARG, "NULL handle or output");
  if (!(d >= 0.0 && d < 1.0)) return set_error(PCPM_ERR_INVALID_ARG, "d must lie in [0, 1)");
  if (g->ngroups != 1 || g->matrix)
    return set_error(PCPM_ERR_INVALID_ARG, "warm start needs a single-graph handle (not a matrix)");
  PCPM_TRY(ws_check_device_ptr(feat, "feat"));
  hipStream_t st = static_cast<hipStream_t>(stream);
  PCPM_TRY(ws_prepare(g, st));
  if (first_call_ms) *first_call_ms = g->ws_indeg_ms;
  const int64_t n = g->n;
  PCPM_TRY(pcpm_iterate(g, d, g->ws_x, g->ws_x + n, nullptr, stream));  // from the uniform vector
  PCPM_LAUNCH("pcpm_ws_features", k_ws_features, dim3(grid_for(n)), dim3(256), 0, st, feat, feat_src(g), n);
  return PCPM_OK;
}

pcpm_status_t pcpm_ws_predict(pcpm_png_t g, const float* params, double d, float* yhat, double* first_call_ms,
                              void* stream) {
  using namespace pcpm;
  if (!g || !yhat) return set_error(PCPM_ERR_INVALID_ARG, "NULL handle or output");
  if (!(d >= 0.0 && d < 1.0)) return set_error(PCPM_ERR_INVALID_ARG, "d must lie in [0, 1)");
  if (g->ngroups != 1 || g->matrix)
    return set_error(PCPM_ERR_INVALID_ARG, "warm start needs a single-graph handle (not a matrix)");
  PCPM_TRY(ws_check_device_ptr(params, "params"));
  PCPM_TRY(ws_check_device_ptr(yhat, "yhat"));
  hipStream_t st = static_cast<hipStream_t>(stream);
  PCPM_TRY(ws_prepare(g, st));
  if (first_call_ms) *first_call_ms = g->ws_indeg_ms;
  const int64_t n = g->n;
  PCPM_TRY(pcpm_iterate(g, d, g->ws_x, g->ws_x + n, nullptr, stream));  // from the uniform vector
  PCPM_LAUNCH("pcpm_ws_predict", k_ws_forward<true>, dim3(forward_blocks(n)), dim3(kFwdBlock), 0, st, params,
              nullptr, feat_src(g), n, yhat);
  return PCPM_OK;
}

pcpm_status_t pcpm_ws_forward(const float* params, const float* feat, int64_t n, float* yhat, void* stream) {
  using namespace pcpm;
  if (n < 1) return set_error(PCPM_ERR_INVALID_ARG, "n must be >= 1");
  PCPM_TRY(ws_check_device_ptr(params, "params"));
  PCPM_TRY(ws_check_device_ptr(feat, "feat"));
  PCPM_TRY(ws_check_device_ptr(yhat, "yhat"));
  hipStream_t st = static_cast<hipStream_t>(stream);
  PCPM_LAUNCH("pcpm_ws_forward", k_ws_forward<false>, dim3(forward_blocks(n)), dim3(kFwdBlock), 0, st, params, feat,
              FeatSrc{}, n, yhat);
  return PCPM_OK;
}

pcpm_status_t pcpm_ws_init(const float* yhat, int64_t n, float* pr0, float* work, int32_t* fallback, void* stream) {
  using namespace pcpm;
  if (n < 1 || !fallback) return set_error(PCPM_ERR_INVALID_ARG, "bad size or NULL flag");
  PCPM_TRY(ws_check_device_ptr(yhat, "yhat"));
  PCPM_TRY(ws_check_device_ptr(pr0, "pr0"));
  PCPM_TRY(ws_check_device_ptr(work, "work"));
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* red = reinterpret_cast<double*>(work);                   // 3 * (kSoftBlocks + 1) doubles
  int32_t* flag = reinterpret_cast<int32_t*>(work + 6 * (kSoftBlocks + 1));
  PCPM_LAUNCH("pcpm_ws_init", k_ws_soft_part, dim3(kSoftBlocks), dim3(kSoftThreads), 0, st, yhat, n, red);
  PCPM_LAUNCH("pcpm_ws_init", k_ws_soft_final, dim3(1), dim3(kSoftThreads), 0, st, red);
  PCPM_LAUNCH("pcpm_ws_init", k_ws_soft_norm, dim3(grid_for(n)), dim3(kSoftThreads), 0, st, yhat, n, red, pr0, flag);
  PCPM_TRY_HIP(hipMemcpyAsync(fallback, flag, 4, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  return PCPM_OK;
}

int64_t pcpm_ws_work_floats(int64_t b) {
  const int64_t parts = std::max<int64_t>(1, std::min<int64_t>((b + pcpm::kChunk - 1) / pcpm::kChunk, 1024));
  return std::max<int64_t>(parts * PCPM_WS_PARAMS + 4 * (parts + 1), 6 * (pcpm::kSoftBlocks + 1) + 4);
}

pcpm_status_t pcpm_ws_backward(const float* params, const float* feat, const float* target, int64_t rows,
                               const int64_t* idx, int64_t b, float* grad, float* work, double* loss, void* stream) {
  using namespace pcpm;
  if (b < 1 || rows < 1 || !loss) return set_error(PCPM_ERR_INVALID_ARG, "empty minibatch, no rows or NULL loss");
  PCPM_TRY(ws_check_device_ptr(work, "work"));
  return ws_backward(params, feat, target, rows, idx, b, grad, work, loss, static_cast<hipStream_t>(stream));
}

pcpm_status_t pcpm_ws_backward_noalloc(const float* params, const float* feat, const float* target, int64_t rows,
                                       const int64_t* idx, int64_t b, float* grad, double* loss, void* stream) {
  using namespace pcpm;
  if (b < 1 || rows < 1 || !loss) return set_error(PCPM_ERR_INVALID_ARG, "empty minibatch, no rows or NULL loss");
  if (b > kNoAllocMaxBatch)
    return set_error(PCPM_ERR_INVALID_ARG,
                     "minibatch of %lld samples exceeds the %lld that the fixed scratch of "
                     "pcpm_ws_backward_noalloc holds (use pcpm_ws_backward with a workspace)",
                     static_cast<long long>(b), static_cast<long long>(kNoAllocMaxBatch));
  float* work = nullptr;
  PCPM_TRY(noalloc_scratch(&work));
  return ws_backward(params, feat, target, rows, idx, b, grad, work, loss, static_cast<hipStream_t>(stream));
}

pcpm_status_t pcpm_ws_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr,
                           void* stream) {
  using namespace pcpm;
  if (step < 1 || !(lr > 0.0f)) return set_error(PCPM_ERR_INVALID_ARG, "step must be >= 1 and lr > 0");
  PCPM_TRY(ws_check_device_ptr(params, "params"));
  PCPM_TRY(ws_check_device_ptr(grad, "grad"));
  PCPM_TRY(ws_check_device_ptr(m, "m"));
  PCPM_TRY(ws_check_device_ptr(v, "v"));
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double c1 = 1.0 - std::pow(b1, step), c2 = 1.0 - std::pow(b2, step);
  PCPM_LAUNCH("pcpm_ws_adam", k_ws_adam, dim3((PCPM_WS_PARAMS + 255) / 256), dim3(256), 0,
              static_cast<hipStream_t>(stream), params, grad, m, v, lr, static_cast<float>(b1),
              static_cast<float>(1.0 - b1), static_cast<float>(b2), static_cast<float>(1.0 - b2),
              static_cast<float>(eps), static_cast<float>(c1), static_cast<float>(c2));
  return PCPM_OK;
}

pcpm_status_t pcpm_ws_targets(const float* pr, int64_t n, float* y, void* stream) {
  using namespace pcpm;
  if (n < 1) return set_error(PCPM_ERR_INVALID_ARG, "n must be >= 1");
  PCPM_TRY(ws_check_device_ptr(pr, "pr"));
  PCPM_TRY(ws_check_device_ptr(y, "y"));
  PCPM_LAUNCH("pcpm_ws_targets", k_ws_targets, dim3(grid_for(n)), dim3(256), 0, static_cast<hipStream_t>(stream), pr,
              n, y);
  return PCPM_OK;
}

}  // extern "C"
