// Batched personalised PageRank over one PNG: kt vectors share every PNG
// edge and every destination ID.
//
// Vector j teleports to its seed set S_j: x'(v) = (1-d) t_j(v) + d (sum_{u->v}
// x(u)/outdeg(u) + D_j t_j(v)) with t_j uniform on S_j and D_j the vector's
// dangling mass, i.e. the recurrence of Eq. 1 with the uniform jump replaced
// by t_j.  An update slot holds kt values (one per vector of the tile), so the
// scatter of Alg. 3 writes kt floats per PNG edge and the gather of Alg. 5
// decodes each destination ID once for kt accumulations.  The kt slots of
// the tile take the batch's vectors from a queue: a vector whose residual
// falls below tol (or that reaches the iteration limit) is stored and its
// slot starts the next vector at once, so slots never idle while vectors
// wait.  A slot with no vector left keeps its last iterate.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "pcpm_device.hpp"
#include "pcpm_internal.hpp"

namespace pcpm {

constexpr int kPprBlock = 512;          // merge workgroups
constexpr int kPprScatterBlock = 1024;  // scatter workgroups (a pair's slice takes up to 128 KB of LDS)
constexpr int kPprGatherBlock = 1024;  // gather workgroups (a 128 KB slice leaves room for one per CU)

// Copy of a slot's KT values; kNt: non-temporal stores (the PNG-ordered
// update stream, one contiguous run per tile: the batch ran ~5% faster on
// RMAT-22 with them).
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int KT, bool kNt = false>
__device__ __forceinline__ void copy_kt(float* __restrict__ dst, const float* __restrict__ src) {
  if constexpr (KT % 4 == 0) {
#pragma unroll
    for (int c = 0; c < KT; c += 4) {
      const f32x4 v = *reinterpret_cast<const f32x4*>(src + c);
      if constexpr (kNt) __builtin_nontemporal_store(v, reinterpret_cast<f32x4*>(dst + c));
      else *reinterpret_cast<f32x4*>(dst + c) = v;
    }
  } else {
#pragma unroll
    for (int c = 0; c < KT; ++c) {
      if constexpr (kNt) __builtin_nontemporal_store(src[c], dst + c);
      else dst[c] = src[c];
    }
  }
}

// Scatter (Alg. 3) for a tile of KT vectors: the source pair's scaled values
// x(u, j)/outdeg(u) are staged in LDS ([2q][KT]); every PNG edge copies its
// node's KT values to its update slot: slot e in PNG order (kPng; a tile of
// 1024 PNG edges writes one contiguous run), else the slot its pair segment's
// delta gives, with a ballot per 64 entries decoding the segments.  The next
// tile's source IDs are loaded while this one is written.
template <int KT, bool kPng>
__device__ __forceinline__ void ppr_scatter_item(const Item it, float* __restrict__ spr, int64_t n, int s,
                                                 const float* __restrict__ x, const int32_t* __restrict__ outdeg,
                                                 const uint16_t* __restrict__ png_src,
                                                 const int32_t* __restrict__ png_blk,
                                                 const int32_t* __restrict__ seg_delta, float* __restrict__ upd,
                                                 int64_t spare) {
  // spr: 2q * KT scaled values of the source partition pair
  const int64_t v0 = static_cast<int64_t>(it.part) << (s + 1);  // a partition pair
  const int qn = static_cast<int>(min(int64_t{2} << s, n - v0));
  for (int i = threadIdx.x; i < qn * KT; i += kPprScatterBlock) {
    const int od = outdeg[v0 + i / KT];
    spr[i] = od > 0 ? x[v0 * KT + i] / static_cast<float>(od) : 0.0f;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t qmask = (2u << s) - 1u;
  const int64_t lo = it.lo, hi = it.hi;
  const int64_t t_end = (hi + kTile - 1) / kTile;
  constexpr int kNW = kPprScatterBlock / kWave;
  uint32_t w[kPairs], wn[kPairs];
  int64_t t = lo / kTile + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  // bin order: the tile's pair-segment counts and deltas come in with its
  // IDs, the counts of the next tile one step earlier (as in the gather)
  int32_t cv = 0, cvn = 0, dl = 0;
  if (t < t_end) {
    load_tile_words(png_src + t * kTile, lane, w);
    if constexpr (!kPng) {
      cv = load_counts(png_blk, nullptr, t, lane);
      if (t + kNW < t_end) cvn = load_counts(png_blk, nullptr, t + kNW, lane);
      dl = tile_deltas(seg_delta, __builtin_amdgcn_readlane(cv, 0), lane);
    }
  }
  for (; t < t_end; t += kNW) {
    const int64_t tb = t * kTile;
    int32_t dln = 0, cvnn = 0;
    if (t + kNW < t_end) {
      load_tile_words(png_src + (t + kNW) * kTile, lane, wn);
      if constexpr (!kPng) {
        dln = tile_deltas(seg_delta, __builtin_amdgcn_readlane(cvn, 0), lane);
        if (t + 2 * kNW < t_end) cvnn = load_counts(png_blk, nullptr, t + 2 * kNW, lane);
      }
    }
    uint32_t xs[kSub];
    unpack_tile(w, xs);
    if constexpr (kPng) {
      if (tb >= lo && tb + kTile <= hi) {
        float* ut = upd + tb * KT;
#pragma unroll
        for (int j = 0; j < kSub; ++j)
          copy_kt<KT, true>(ut + static_cast<int64_t>(j * kWave + lane) * KT, spr + (xs[j] & qmask) * KT);
      } else {
#pragma unroll
        for (int j = 0; j < kSub; ++j) {
          const int64_t e = tb + j * kWave + lane;
          if (e >= lo && e < hi) copy_kt<KT, true>(upd + e * KT, spr + (xs[j] & qmask) * KT);
        }
      }
    } else {
      // every entry of a tile has a valid segment (entry 0 is flagged and
      // padding follows the last segment); its delta comes from the 64 that
      // came in with the tile (dl) or from seg_delta
      const int32_t sb = __builtin_amdgcn_readlane(cv, 0);
      int32_t run = sb - 1;
      int32_t seg[kSub];
#pragma unroll
      for (int j = 0; j < kSub; ++j) {
        const bool f = (xs[j] & kDidFlag) != 0u;
        const uint64_t bal = wave_ballot(f);
        seg[j] = run + lanes_below(bal) + (f ? 1 : 0);
        run += __popcll(bal);
      }
      const int32_t sbase = max(sb - 1, 0);
      int32_t d[kSub];
      if (run - sbase < kWave) {
#pragma unroll
        for (int j = 0; j < kSub; ++j) d[j] = __builtin_amdgcn_ds_bpermute((seg[j] - sbase) << 2, dl);
      } else {
#pragma unroll
        for (int j = 0; j < kSub; ++j) d[j] = seg_delta[seg[j]];
      }
      if (tb >= lo && tb + kTile <= hi) {
        float* ut = upd + tb * KT;
#pragma unroll
        for (int j = 0; j < kSub; ++j)
          copy_kt<KT>(ut + static_cast<int64_t>(j * kWave + lane + d[j]) * KT, spr + (xs[j] & qmask) * KT);
      } else {
#pragma unroll
        for (int j = 0; j < kSub; ++j) {
          const int64_t e = tb + j * kWave + lane;
          const bool in = e >= lo && e < hi;
          copy_kt<KT>(upd + (in ? e + d[j] : spare) * KT, spr + (xs[j] & qmask) * KT);
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kPairs; ++j) w[j] = wn[j];
    cv = cvn;
    cvn = cvnn;
    dl = dln;
  }
}

template <int KT, bool kPng>
__global__ __launch_bounds__(kPprScatterBlock) void k_ppr_scatter(const Ctl* __restrict__ ctl, int64_t n, int s,
                                                           const Item* __restrict__ items, const float* __restrict__ x,
                                                           const int32_t* __restrict__ outdeg,
                                                           const uint16_t* __restrict__ png_src,
                                                           const int32_t* __restrict__ png_blk,
                                                           const int32_t* __restrict__ seg_delta,
                                                           float* __restrict__ upd, int64_t spare) {
  if (ctl->done) return;
  extern __shared__ float spr[];
  ppr_scatter_item<KT, kPng>(items[xcd_block(blockIdx.x, gridDim.x)], spr, n, s, x, outdeg, png_src, png_blk,
                             seg_delta, upd, spare);  // as in the plain scatter
}

// Apply for nodes n0..n1-1 of a destination partition and all KT vectors:
//   x'(v, j) = d * acc(v, j) + [v in S_j] * ((1-d) + d*D_j)/|S_j|
// and each vector's share of the residual and of the next dangling mass.
// Thread i serves vector i % KT; kU nodes per step, loads first.  G > 1: G
// groups of BS threads in the workgroup, each applying its own range (an
// empty one with red_slot NULL for a group without work) exactly as a
// workgroup of BS threads does; every thread calls it.
template <int KT, int BS, class AccFn, int G = 1>
__device__ __forceinline__ void apply_ppr(const Ctl* __restrict__ ctl, const VCtl* __restrict__ vctl, int64_t v0,
                                          int n0, int n1, AccFn acc, const float* __restrict__ x_in,
                                          float* __restrict__ x_out, const uint32_t* __restrict__ dmask,
                                          const uint32_t* __restrict__ seedmask, double* __restrict__ red_slot) {
  static_assert(BS % KT == 0 && kWave % KT == 0, "vectors per tile must divide the wavefront");
  const int tid = static_cast<int>(threadIdx.x % BS), grp = static_cast<int>(threadIdx.x / BS);
  const int kk = tid % KT;
  const bool frozen = vctl[kk].done != 0;
  const double coef = vctl[kk].coef;
  const double d = ctl->d;
  const double unit = ldexp(1.0, -ctl->fx_shift);
  double r = 0.0, dm = 0.0;
  float mx = 0.0f;  // largest new value: the next fixed-point scale
  constexpr int kU = 4;
  constexpr int kStep = BS / KT;
  for (int node = n0 + tid / KT; node < n1; node += kU * kStep) {
    float xo[kU];
    uint32_t sm[kU], dw[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t v = v0 + min(node + u * kStep, n1 - 1);
      xo[u] = x_in[v * KT + kk];
      sm[u] = seedmask[v];
      dw[u] = dmask[v >> 5];
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int nd = node + u * kStep;
      if (nd < n1) {
        const int64_t v = v0 + nd;
        const bool seed = (sm[u] >> kk) & 1u;
        const double a = static_cast<double>(acc(nd, kk)) * unit;
        const float xn = frozen ? xo[u] : static_cast<float>(fma(d, a, seed ? coef : 0.0));
        r += fabs(static_cast<double>(xn) - static_cast<double>(xo[u]));
        if ((dw[u] >> (v & 31)) & 1u) dm += static_cast<double>(xn);
        mx = fmaxf(mx, fabsf(xn));
        x_out[v * KT + kk] = xn;
      }
    }
  }
  // lanes of one vector are those congruent to kk modulo KT
#pragma unroll
  for (int off = kWave / 2; off >= KT; off >>= 1) {
    r += __shfl_xor(r, off);
    dm += __shfl_xor(dm, off);
    mx = fmaxf(mx, __shfl_xor(mx, off));
  }
  __shared__ double shg[G][(BS / kWave) * KT * 3];
  double* sh = shg[grp];
  const int w = tid / kWave, lane = tid & (kWave - 1);
  if (lane < KT) {
    sh[(w * KT + lane) * 3] = r;
    sh[(w * KT + lane) * 3 + 1] = dm;
    sh[(w * KT + lane) * 3 + 2] = static_cast<double>(mx);
  }
  __syncthreads();
  if (tid < KT && red_slot) {
    double rs = 0.0, ds = 0.0, ms = 0.0;
    for (int ww = 0; ww < BS / kWave; ++ww) {
      rs += sh[(ww * KT + tid) * 3];
      ds += sh[(ww * KT + tid) * 3 + 1];
      ms = fmax(ms, sh[(ww * KT + tid) * 3 + 2]);
    }
    red_slot[tid * 3] = rs;
    red_slot[tid * 3 + 1] = ds;
    red_slot[tid * 3 + 2] = ms;
  }
}

// Gather (Alg. 5) for a tile of KT vectors: each destination ID is decoded
// once (its update is the one of the message it belongs to: flags so far,
// inclusive, minus one) and adds KT fixed-point values to the LDS slice
// ([KT][q] 64-bit sums: vector-major, so the 64 lanes of one add spread over
// the banks as in the single-vector gather; node-major rows of KT sums put
// them on 32/KT bank pairs).  The next tile's IDs are loaded while this one is
// accumulated; the update values of kG sub-blocks are in flight together.
template <int KT, bool kPng>
__device__ __forceinline__ void ppr_gather_item(const Item it, unsigned long long* __restrict__ acc,
                                                const Ctl* __restrict__ ctl, int64_t n, int s,
                                                const uint16_t* __restrict__ did, const int32_t* __restrict__ did_blk,
                                                const int32_t* __restrict__ did_sblk,
                                                const int32_t* __restrict__ seg_delta, const float* __restrict__ upd,
                                                const float* __restrict__ x_in, float* __restrict__ x_out,
                                                const uint32_t* __restrict__ dmask,
                                                const uint32_t* __restrict__ seedmask, int64_t* __restrict__ partial,
                                                double* __restrict__ red, const VCtl* __restrict__ vctl) {
  constexpr int BS = kPprGatherBlock;  // acc: q * KT fixed-point sums
  const int64_t q = int64_t{1} << s;
  const int64_t v0 = static_cast<int64_t>(it.part) << s;
  const int qn = static_cast<int>(min(q, n - v0));
  const FixedConv to_fixed(ctl->fx_shift);
  const int lane = threadIdx.x & (kWave - 1);
  const uint32_t qmask = static_cast<uint32_t>(q - 1);
  const uint32_t qs = static_cast<uint32_t>(q);
  const int64_t lo = it.lo, hi = it.hi;
  const int64_t t_end = (hi + kTile - 1) / kTile;
  constexpr int kNW = BS / kWave;
  constexpr int kG = KT >= 16 ? 2 : (KT >= 8 ? 4 : (KT >= 4 ? 8 : 16));
  // Loads go out as in the single-vector gather: the first value group of
  // this tile, then the next tile's IDs and segment deltas and the flag
  // counts of the tile after that, so the prefetches stay in flight through
  // this tile's adds.
  uint32_t w[kPairs], wn[kPairs];
  const int64_t t0 = lo / kTile + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int32_t* sblk_arr = kPng ? did_sblk : nullptr;
  int32_t cv = 0, cvn = 0, dl = 0;
  // the first tiles' loads stay in flight through the clear of the slice
  if (t0 < t_end) {
    load_tile_words(did + t0 * kTile, lane, w);
    cv = load_counts(did_blk, sblk_arr, t0, lane);
    if (t0 + kNW < t_end) cvn = load_counts(did_blk, sblk_arr, t0 + kNW, lane);
  }
  for (int i = threadIdx.x; i < q * KT; i += BS) acc[i] = 0ull;
  if constexpr (kPng) {
    if (t0 < t_end) dl = tile_deltas(seg_delta, __builtin_amdgcn_readlane(cv, 1), lane);
  }
  __syncthreads();
  for (int64_t t = t0; t < t_end; t += kNW) {
    const int64_t tb = t * kTile;
    uint32_t xs[kSub];
    unpack_tile(w, xs);
    // every entry has a valid update slot
    int32_t slot[kSub];
    tile_slots<kPng>(xs, __builtin_amdgcn_readlane(cv, 0), __builtin_amdgcn_readlane(cv, 1), dl, seg_delta, slot);
    int32_t dln = 0, cvnn = 0;
    const bool full = tb >= lo && tb + kTile <= hi;
#pragma unroll
    for (int g0 = 0; g0 < kSub; g0 += kG) {
      float val[kG][KT];
#pragma unroll
      for (int jj = 0; jj < kG; ++jj) copy_kt<KT>(val[jj], upd + static_cast<int64_t>(slot[g0 + jj]) * KT);
      if (g0 == 0 && t + kNW < t_end) {  // prefetch (g0 is a constant after unrolling)
        load_tile_words(did + (t + kNW) * kTile, lane, wn);
        if constexpr (kPng) dln = tile_deltas(seg_delta, __builtin_amdgcn_readlane(cvn, 1), lane);
        if (t + 2 * kNW < t_end) cvnn = load_counts(did_blk, sblk_arr, t + 2 * kNW, lane);
      }
      if (full) {
#pragma unroll
        for (int jj = 0; jj < kG; ++jj) {
          const uint32_t li = xs[g0 + jj] & qmask;
#pragma unroll
          for (int c = 0; c < KT; ++c)
            atomicAdd(&acc[c * qs + li], static_cast<unsigned long long>(to_fixed(val[jj][c])));
        }
      } else {  // edge tile: entries outside [lo, hi) add nothing
#pragma unroll
        for (int jj = 0; jj < kG; ++jj) {
          const int64_t e = tb + (g0 + jj) * kWave + lane;
          const bool in = e >= lo && e < hi;
          const uint32_t li = in ? (xs[g0 + jj] & qmask) : 0u;
#pragma unroll
          for (int c = 0; c < KT; ++c)
            atomicAdd(&acc[c * qs + li], static_cast<unsigned long long>(in ? to_fixed(val[jj][c]) : 0));
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kPairs; ++j) w[j] = wn[j];
    cv = cvn;
    cvn = cvnn;
    dl = dln;
  }
  __syncthreads();
  if (it.aux >= 0) {
    int64_t* dst = partial + static_cast<int64_t>(it.aux) * q * KT;  // the same [KT][q] layout
    for (int i = threadIdx.x; i < q * KT; i += BS) dst[i] = static_cast<int64_t>(acc[i]);
    return;
  }
  apply_ppr<KT, BS>(ctl, vctl, v0, 0, qn, [&](int nd, int c) { return static_cast<int64_t>(acc[c * q + nd]); }, x_in,
                    x_out, dmask, seedmask, red + static_cast<int64_t>(it.part) * KT * 3);
}

template <int KT, bool kPng>
__global__ __launch_bounds__(kPprGatherBlock) void k_ppr_gather(const Ctl* __restrict__ ctl, int64_t n, int s,
                                                                const Item* __restrict__ items,
                                                                const uint16_t* __restrict__ did,
                                                                const int32_t* __restrict__ did_blk,
                                                                const int32_t* __restrict__ did_sblk,
                                                                const int32_t* __restrict__ seg_delta,
                                                                const float* __restrict__ upd,
                                                                const float* __restrict__ x_in,
                                                                float* __restrict__ x_out,
                                                                const uint32_t* __restrict__ dmask,
                                                                const uint32_t* __restrict__ seedmask,
                                                                int64_t* __restrict__ partial,
                                                                double* __restrict__ red,
                                                                const VCtl* __restrict__ vctl) {
  if (ctl->done) return;
  extern __shared__ unsigned long long acc[];
  ppr_gather_item<KT, kPng>(items[xcd_block(blockIdx.x, gridDim.x)], acc, ctl, n, s, did, did_blk, did_sblk, seg_delta, upd, x_in, x_out,
                            dmask, seedmask, partial, red, vctl);
}

// Merge unit u (u < 0: none, for a group without work; G groups of
// kPprBlock threads as in apply_ppr).
template <int KT, int G = 1>
__device__ __forceinline__ void ppr_merge_unit(const Merge mu, int64_t u, const Ctl* __restrict__ ctl, int64_t n,
                                               int s, const int64_t* __restrict__ partial,
                                               const float* __restrict__ x_in, float* __restrict__ x_out,
                                               const uint32_t* __restrict__ dmask,
                                               const uint32_t* __restrict__ seedmask, double* __restrict__ red,
                                               int64_t red_base, const VCtl* __restrict__ vctl) {
  const int64_t q = int64_t{1} << s;
  const int64_t v0 = static_cast<int64_t>(mu.part) << s;
  const int qn = static_cast<int>(min(q, n - v0));
  const int64_t* base = partial + static_cast<int64_t>(mu.first) * q * KT;
  const int cnt = mu.count;
  auto acc = [&](int nd, int vec) {  // partial slices are [KT][q]
    return sum_slices(base + static_cast<int64_t>(vec) * q + nd, cnt, q * KT);
  };
  const bool has = u >= 0;
  apply_ppr<KT, kPprBlock, decltype(acc), G>(ctl, vctl, v0, has ? mu.node_lo : 0, has ? min(qn, mu.node_lo + 256) : 0,
                                             acc, x_in, x_out, dmask, seedmask,
                                             has ? red + (red_base + u) * KT * 3 : nullptr);
}

template <int KT>
__global__ __launch_bounds__(kPprBlock) void k_ppr_merge(const Ctl* __restrict__ ctl, int64_t n, int s,
                                                         const Merge* __restrict__ mg,
                                                         const int64_t* __restrict__ partial,
                                                         const float* __restrict__ x_in, float* __restrict__ x_out,
                                                         const uint32_t* __restrict__ dmask,
                                                         const uint32_t* __restrict__ seedmask,
                                                         double* __restrict__ red, int64_t red_base,
                                                         const VCtl* __restrict__ vctl) {
  if (ctl->done) return;
  ppr_merge_unit<KT>(mg[blockIdx.x], blockIdx.x, ctl, n, s, partial, x_in, x_out, dmask, seedmask, red, red_base,
                     vctl);
}

// Per-vector residual, dangling mass and jump coefficient; one wavefront per
// slot, apply units in order.  Then the refill plan: every slot whose vector
// finished (below tol, or at the iteration limit) records the vector's
// iteration count, residual and convergence, and takes the next vector of the
// queue; the batch is done when every slot is idle.
// Per-vector sums by one wavefront per slot go through LDS; every field of the
// control structs is then read and written by thread 0 alone (stores of
// different wavefronts to one struct are not ordered by a workgroup barrier).
__device__ __forceinline__ void ppr_finalize_body(Ctl* __restrict__ ctl, VCtl* __restrict__ vctl, int kt,
                                                  const double* __restrict__ red, int64_t nslots,
                                                  double* __restrict__ hist, PprQueue* __restrict__ queue,
                                                  int32_t* __restrict__ out_it, double* __restrict__ out_res,
                                                  int32_t* __restrict__ out_conv) {
  double vmax = 0.0;  // largest value of the new iterates (all vectors of the tile)
  for (int64_t j = threadIdx.x; j < nslots * kt; j += 1024) vmax = fmax(vmax, red[3 * j + 2]);
  vmax = block_max<1024>(vmax);
  __shared__ double s_r[16], s_dm[16];
  const int lane = threadIdx.x & (kWave - 1);
  for (int kk = threadIdx.x / kWave; kk < kt; kk += 1024 / kWave) {
    double r = 0.0, dm = 0.0;
    for (int64_t sl = lane; sl < nslots; sl += kWave) {
      r += red[(sl * kt + kk) * 3];
      dm += red[(sl * kt + kk) * 3 + 1];
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
      r += __shfl_xor(r, off);
      dm += __shfl_xor(dm, off);
    }
    if (lane == 0) {
      s_r[kk] = r;
      s_dm[kk] = dm;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const double d = ctl->d, tol = ctl->tol;
    int bad = 0;
    for (int kk = 0; kk < kt; ++kk) {
      VCtl& vc = vctl[kk];
      if (!vc.done) {
        const double r = s_r[kk], dm = s_dm[kk];
        vc.res = r;
        vc.iter += 1;
        vc.dmass = dm;
        vc.coef = ((1.0 - d) + d * dm) * vc.inv_s;
        if (!isfinite(r) || !isfinite(dm)) bad = 1;
        else if (tol > 0.0 && r < tol) vc.done = 1;
      }
    }
    double rmax = 0.0;  // largest residual of the vectors still running
    for (int kk = 0; kk < kt; ++kk)
      if (vctl[kk].vec >= 0 && !vctl[kk].done) rmax = fmax(rmax, vctl[kk].res);
    int pending = 0, any_new = 0, all_idle = 1;
    for (int kk = 0; kk < kt; ++kk) {
      VCtl& vc = vctl[kk];
      queue->old_vec[kk] = -1;
      queue->new_vec[kk] = -1;
      if (vc.vec >= 0 && (vc.done || vc.iter >= queue->max_iters)) {
        out_it[vc.vec] = vc.iter;
        out_res[vc.vec] = vc.res;
        out_conv[vc.vec] = vc.done;
        const int nv = queue->head < queue->k ? queue->head++ : -1;
        queue->old_vec[kk] = vc.vec;
        queue->new_vec[kk] = nv;
        vc.vec = nv;
        vc.done = 1;  // keeps its column until the refill starts the next vector
        pending = 1;
        any_new |= nv >= 0;
      }
      all_idle &= vc.vec < 0;
    }
    queue->pending = pending;
    if (bad) rmax = NAN;
    const int32_t it = ctl->iter;
    ctl->res_prev = ctl->res;
    ctl->res = rmax;
    if (it < kMaxHist) hist[it] = rmax;
    ctl->iter = it + 1;
    if (bad) ctl->nonfinite = 1;
    if (bad || all_idle) ctl->done = 1;
    // a new vector starts with values up to 1 (a single seed)
    ctl->fx_shift = fx_shift_for(any_new ? fmax(vmax, 1.0) : vmax, ctl->fx_cap);
  }
}

__global__ __launch_bounds__(1024) void k_ppr_finalize(Ctl* __restrict__ ctl, VCtl* __restrict__ vctl, int kt,
                                                       const double* __restrict__ red, int64_t nslots,
                                                       double* __restrict__ hist, PprQueue* __restrict__ queue,
                                                       int32_t* __restrict__ out_it, double* __restrict__ out_res,
                                                       int32_t* __restrict__ out_conv) {
  if (ctl->done) return;
  ppr_finalize_body(ctl, vctl, kt, red, nslots, hist, queue, out_it, out_res, out_conv);
}

// Refill, first part (whole grid): the finished vectors' columns go to
// pr_out[v][vec], and the columns of slots that start a new vector are
// cleared.  Nothing to do unless the last iteration planned a refill.
// Nodes t0, t0 + stride, ... of the refill's first part.
template <int KT>
__device__ __forceinline__ void ppr_refill_cols_nodes(const PprQueue* __restrict__ queue, float* __restrict__ x,
                                                      float* __restrict__ out, int64_t n, int k, int64_t t0,
                                                      int64_t stride) {
  int ov[KT], nv[KT];
#pragma unroll
  for (int c = 0; c < KT; ++c) {
    ov[c] = queue->old_vec[c];
    nv[c] = queue->new_vec[c];
  }
  for (int64_t v = t0; v < n; v += stride) {
    float row[KT];
    copy_kt<KT>(row, x + v * KT);
    bool clear = false;
#pragma unroll
    for (int c = 0; c < KT; ++c) {
      if (ov[c] >= 0) out[v * k + ov[c]] = row[c];
      if (nv[c] >= 0) {
        row[c] = 0.0f;
        clear = true;
      }
    }
    if (clear) copy_kt<KT>(x + v * KT, row);
  }
}

template <int KT>
__global__ __launch_bounds__(256) void k_ppr_refill_cols(const PprQueue* __restrict__ queue, float* __restrict__ x,
                                                         float* __restrict__ out, int64_t n, int k) {
  if (!queue->pending) return;
  ppr_refill_cols_nodes<KT>(queue, x, out, n, k, static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x,
                            static_cast<int64_t>(gridDim.x) * blockDim.x);
}

// Refill, second part (one workgroup): seed bits of the finished vectors are
// cleared, then each new vector gets x_0 = t_j on its seeds, its seed bits,
// dangling mass and jump coefficient; one wavefront per slot.
__device__ __forceinline__ void ppr_refill_seeds_body(PprQueue* __restrict__ queue, float* __restrict__ x,
                                                      uint32_t* __restrict__ mask, const int32_t* __restrict__ seeds,
                                                      const int32_t* __restrict__ seed_off, int kt,
                                                      VCtl* __restrict__ vctl, const uint32_t* __restrict__ dmask,
                                                      double d) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int kk = threadIdx.x / kWave; kk < kt; kk += 1024 / kWave) {
    const int ov = queue->old_vec[kk];
    if (ov >= 0)
      for (int i = seed_off[ov] + lane; i < seed_off[ov + 1]; i += kWave) atomicAnd(&mask[seeds[i]], ~(1u << kk));
  }
  __threadfence();
  __syncthreads();
  for (int kk = threadIdx.x / kWave; kk < kt; kk += 1024 / kWave) {
    const int nv = queue->new_vec[kk];
    double dm = 0.0, inv = 0.0;
    if (nv >= 0) {
      const int a = seed_off[nv], b = seed_off[nv + 1];
      inv = 1.0 / static_cast<double>(b - a);
      for (int i = a + lane; i < b; i += kWave) {
        const int v = seeds[i];
        x[static_cast<int64_t>(v) * kt + kk] = static_cast<float>(inv);
        atomicOr(&mask[v], 1u << kk);
        if ((dmask[v >> 5] >> (v & 31)) & 1u) dm += inv;
      }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) dm += __shfl_xor(dm, off);
    if (lane == 0 && nv >= 0) {
      VCtl& vc = vctl[kk];
      vc.inv_s = inv;
      vc.dmass = dm;
      vc.coef = ((1.0 - d) + d * dm) * inv;
      vc.res = 0.0;
      vc.iter = 0;
      vc.done = 0;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) queue->pending = 0;
}

__global__ __launch_bounds__(1024) void k_ppr_refill_seeds(PprQueue* __restrict__ queue, float* __restrict__ x,
                                                           uint32_t* __restrict__ mask,
                                                           const int32_t* __restrict__ seeds,
                                                           const int32_t* __restrict__ seed_off, int kt,
                                                           VCtl* __restrict__ vctl,
                                                           const uint32_t* __restrict__ dmask, double d) {
  if (!queue->pending) return;
  ppr_refill_seeds_body(queue, x, mask, seeds, seed_off, kt, vctl, dmask, d);
}

// pr_out[v][j] = x[v][j] for the first kv slots (batches that fit one tile:
// every vector keeps its slot, and its last iterate, to the end).
__global__ __launch_bounds__(256) void k_ppr_store(float* __restrict__ out, const float* __restrict__ x, int64_t n,
                                                   int k, int kv, int kt) {
  const int64_t total = n * kv;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t v = i / kv;
    const int j = static_cast<int>(i - v * kv);
    out[v * k + j] = x[v * kt + j];
  }
}

__global__ __launch_bounds__(256) void k_ppr_persist_init(PSync* __restrict__ ps, int32_t* __restrict__ bin_done,
                                                          int64_t k) {
  for (int64_t p = threadIdx.x; p < k; p += 256) bin_done[p] = 0;
  if (threadIdx.x == 0) {
    ps->bar_count = 0;
    ps->bar_gen = 0;
    ps->err = 0;
    ps->applied = 0;
    ps->ga_next = 0;
    ps->mg_next = 0;
    for (unsigned x = 0; x < kXcds; ++x) ps->sc_next[x] = 0;
  }
}

__global__ void k_ppr_queue_init(PprQueue* queue, int head, int k, int max_iters) {
  if (threadIdx.x == 0) {
    queue->head = head;
    queue->k = k;
    queue->max_iters = max_iters;
    queue->pending = 0;
  }
}

// Start of a tile: x_0 = t_j (1/|S_j| on the seeds), the seed bitmask, and
// each vector's dangling mass and jump coefficient.  One wavefront per vector;
// slots past the tile's last vector are marked converged (they stay zero).
__global__ __launch_bounds__(1024) void k_ppr_seed(float* __restrict__ x, uint32_t* __restrict__ mask,
                                                   const int32_t* __restrict__ seeds,
                                                   const int32_t* __restrict__ seed_off, int first, int kv, int kt,
                                                   VCtl* __restrict__ vctl, const uint32_t* __restrict__ dmask,
                                                   double d) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int kk = threadIdx.x / kWave; kk < kt; kk += 1024 / kWave) {
    double dm = 0.0, inv = 0.0;
    if (kk < kv) {
      const int a = seed_off[first + kk], b = seed_off[first + kk + 1];
      inv = 1.0 / static_cast<double>(b - a);
      for (int i = a + lane; i < b; i += kWave) {
        const int v = seeds[i];
        x[static_cast<int64_t>(v) * kt + kk] = static_cast<float>(inv);
        atomicOr(&mask[v], 1u << kk);
        if ((dmask[v >> 5] >> (v & 31)) & 1u) dm += inv;
      }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) dm += __shfl_xor(dm, off);
    if (lane == 0) {
      VCtl& vc = vctl[kk];
      vc.inv_s = inv;
      vc.dmass = dm;
      vc.coef = ((1.0 - d) + d * dm) * inv;
      vc.res = 0.0;
      vc.iter = 0;
      vc.done = kk < kv ? 0 : 1;
      vc.vec = kk < kv ? first + kk : -1;
    }
  }
}

__global__ void k_ppr_ctl(Ctl* ctl, double tol, double d) {
  if (threadIdx.x == 0) {
    ctl->res = 0.0;
    ctl->res_prev = 0.0;
    ctl->tol = tol;
    ctl->d = d;
    ctl->iter = 0;
    ctl->done = 0;
    ctl->nonfinite = 0;
    ctl->fx_shift = 50;  // every vector has unit mass
    ctl->fx_cap = 61;
    ctl->ngroups = 1;
  }
}

// ---- persistent batch ---------------------------------------------------------
// Every iteration of the batch in one cooperative launch, phase by phase as
// the plain persistent solve (scatter items; grid barrier; gather items and
// merge units, the last apply unit running the finalize and the refill plan;
// grid barrier), then, when the finalize planned a refill, the finished
// columns stored and cleared by the whole grid, a barrier, the new vectors'
// seeds by workgroup 0 and a barrier.  The launch ends when every slot is
// idle (or a bounded wait gives up).

template <int KT, bool kPng>
__global__ __launch_bounds__(1024) void k_ppr_persist(const PprPersistArgs a) {
  constexpr int BS = 1024;
  constexpr int kMG = BS / kPprBlock;  // merge units per workgroup, one per group of kPprBlock threads
  extern __shared__ unsigned long long lds[];
  PSync* ps = a.ps;
  auto reset = [&]() {  // by the last arrival at the iteration's second barrier
    for (unsigned x = 0; x < kXcds; ++x) __hip_atomic_store(&ps->sc_next[x], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ps->ga_next, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ps->mg_next, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ps->applied, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  const int64_t nslots = a.k + a.n_mg;
  for (int64_t it = 0; it < a.max_loops; ++it) {
    const float* in = (it & 1) ? a.x1 : a.x0;
    float* out = (it & 1) ? a.x0 : a.x1;
    for (;;) {
      const int32_t j = grab_scatter(ps, a.n_sc);
      if (j < 0) break;
      ppr_scatter_item<KT, kPng>(a.sc_items[j], reinterpret_cast<float*>(lds), a.n, a.s, in, a.outdeg, a.png_src,
                                 a.png_blk, a.seg_delta, a.upd, a.spare);
    }
    if (!grid_sync(ps, a.spin_limit, [] {})) return;
    for (;;) {
      const int32_t j = grab(&ps->ga_next);
      if (j >= a.n_ga) break;
      const Item itm = a.ga_items[xcd_block(static_cast<unsigned>(j), static_cast<unsigned>(a.n_ga))];
      ppr_gather_item<KT, kPng>(itm, lds, a.ctl, a.n, a.s, a.did, a.did_blk, a.did_sblk, a.seg_delta, a.upd, in, out,
                                a.dmask, a.seedmask, a.partial, a.red, a.vctl);
      if (itm.aux >= 0) {
        publish(&a.bin_done[itm.part]);
      } else if (publish(&ps->applied) == a.n_apply - 1) {
        ppr_finalize_body(a.ctl, a.vctl, KT, a.red, nslots, a.hist, a.queue, a.out_it, a.out_res, a.out_conv);
      }
    }
    for (;;) {
      const int32_t u0 = grab(&ps->mg_next, kMG);
      if (u0 >= a.n_mg) break;
      const int32_t cnt = min(kMG, a.n_mg - u0);
      for (int32_t c = 0; c < cnt; ++c) {
        const Merge mc = a.mg_items[u0 + c];
        if (c > 0 && mc.part == a.mg_items[u0 + c - 1].part) continue;
        const int32_t target = static_cast<int32_t>(static_cast<uint32_t>(mc.count) * static_cast<uint32_t>(it + 1));
        if (!wait_at_least(ps, &a.bin_done[mc.part], target, a.spin_limit)) return;
      }
      const int g = static_cast<int>(threadIdx.x) / kPprBlock;
      ppr_merge_unit<KT, kMG>(a.mg_items[u0 + (g < cnt ? g : 0)], g < cnt ? u0 + g : -1, a.ctl, a.n, a.s, a.partial,
                              in, out, a.dmask, a.seedmask, a.red, a.k, a.vctl);
      if (publish(&ps->applied, cnt) + cnt == a.n_apply)
        ppr_finalize_body(a.ctl, a.vctl, KT, a.red, nslots, a.hist, a.queue, a.out_it, a.out_res, a.out_conv);
    }
    if (!grid_sync(ps, a.spin_limit, reset)) return;
    if (a.refill && ld_acquire(&a.queue->pending)) {
      // the finished columns stored and cleared by the whole grid, then the
      // new vectors' seeds by workgroup 0
      ppr_refill_cols_nodes<KT>(a.queue, out, a.pr_out, a.n, a.kvec,
                                static_cast<int64_t>(blockIdx.x) * BS + threadIdx.x,
                                static_cast<int64_t>(gridDim.x) * BS);
      if (!grid_sync(ps, a.spin_limit, [] {})) return;
      if (blockIdx.x == 0)
        ppr_refill_seeds_body(a.queue, out, a.seedmask, a.seeds, a.seed_off, KT, a.vctl, a.dmask, a.d);
      if (!grid_sync(ps, a.spin_limit, [] {})) return;
    }
    if (ld_acquire(&a.ctl->done)) return;
  }
}

// ---- host ------------------------------------------------------------------

template <int KT>
static pcpm_status_t ppr_set_lds(int s) {
  for (const void* f : {reinterpret_cast<const void*>(k_ppr_scatter<KT, false>),
                        reinterpret_cast<const void*>(k_ppr_scatter<KT, true>)})
    PCPM_TRY_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (2 << s) * KT * 4));
  for (const void* f : {reinterpret_cast<const void*>(k_ppr_gather<KT, false>),
                        reinterpret_cast<const void*>(k_ppr_gather<KT, true>),
                        reinterpret_cast<const void*>(k_ppr_persist<KT, false>),
                        reinterpret_cast<const void*>(k_ppr_persist<KT, true>)})
    PCPM_TRY_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (1 << s) * KT * 8));
  return PCPM_OK;
}

// Workgroups of the persistent batch (all resident), 0 if it cannot run here
// or the handle asks for one launch per phase.
template <int KT>
static pcpm_status_t ppr_persist_grid(pcpm_png* g, int* grid) {
  *grid = 0;
  if (g->launch_mode != 2) return PCPM_OK;
  int cus = 0, coop = 0, per = 0;
  PCPM_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
  PCPM_TRY_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, g->device));
  const void* f = g->png_order ? reinterpret_cast<const void*>(k_ppr_persist<KT, true>)
                               : reinterpret_cast<const void*>(k_ppr_persist<KT, false>);
  PCPM_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, 1024, static_cast<size_t>(g->q) * KT * 8));
  if (coop && per * cus >= static_cast<int>(kXcds)) *grid = per * cus;
  return PCPM_OK;
}

template <int KT>
static pcpm_status_t ppr_run_persistent(pcpm_png* g, int grid, double d, int k, int64_t cap, float* pr_out, float* a,
                                        float* b, hipStream_t st) {
  PCPM_LAUNCH("pcpm_ppr_init", k_ppr_persist_init, dim3(1), dim3(256), 0, st, g->psync, g->bin_done, g->k);
  PprPersistArgs pa;
  pa.ctl = g->ctl;
  pa.vctl = g->ppr_vctl;
  pa.ps = g->psync;
  pa.bin_done = g->bin_done;
  pa.queue = g->ppr_queue;
  pa.n = g->n;
  pa.k = g->k;
  pa.max_loops = cap;
  pa.spare = g->eprime;
  pa.s = g->part_log2;
  pa.n_sc = g->n_sc;
  pa.n_ga = g->n_ga;
  pa.n_mg = g->n_mg;
  pa.n_apply = static_cast<int32_t>(g->k - g->n_split_bins) + g->n_mg;
  pa.kvec = k;
  pa.refill = k > KT ? 1 : 0;
  pa.spin_limit = g->spin_limit;
  pa.d = d;
  pa.sc_items = g->sc_items;
  pa.ga_items = g->ga_items;
  pa.mg_items = g->mg_items;
  pa.outdeg = g->outdeg;
  pa.png_src = g->png_src;
  pa.png_blk = g->png_blk;
  pa.seg_delta = g->seg_delta;
  pa.upd = g->ppr_upd;
  pa.did = g->did;
  pa.did_blk = g->did_blk;
  pa.did_sblk = g->did_sblk;
  pa.dmask = g->dmask;
  pa.seedmask = g->ppr_mask;
  pa.partial = g->ppr_partial;
  pa.red = g->ppr_red;
  pa.hist = g->hist;
  pa.out_it = g->ppr_out_it;
  pa.out_res = g->ppr_out_res;
  pa.out_conv = g->ppr_out_conv;
  pa.pr_out = pr_out;
  pa.seeds = g->ppr_seeds;
  pa.seed_off = g->ppr_seed_off;
  pa.x0 = a;
  pa.x1 = b;
  void* args[] = {&pa};
  const void* f = g->png_order ? reinterpret_cast<const void*>(k_ppr_persist<KT, true>)
                               : reinterpret_cast<const void*>(k_ppr_persist<KT, false>);
  {
    TimerScope ts("pcpm_ppr_persist", st);
    PCPM_TRY_HIP(hipLaunchCooperativeKernel(f, dim3(static_cast<unsigned>(grid)), dim3(1024), args,
                                            static_cast<unsigned>(g->q * KT * 8), st));
  }
  PCPM_TRY_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipMemcpyAsync(g->psync_host, g->psync, sizeof(PSync), hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  if (g->psync_host->err)
    return set_error(PCPM_ERR_DEVICE, "a device-side wait of the persistent batch ran past its limit of %u polls",
                     g->spin_limit);
  return PCPM_OK;
}

// Scatter and gather of one iteration in the handle's update order.
template <int KT, bool kPng>
static pcpm_status_t ppr_scatter_gather(pcpm_png* g, const float* in, float* out, hipStream_t st) {
  const int s = g->part_log2;
  if (g->n_sc)
    PCPM_LAUNCH("pcpm_ppr_scatter", (k_ppr_scatter<KT, kPng>), dim3(static_cast<unsigned>(g->n_sc)),
                dim3(kPprScatterBlock), static_cast<size_t>(g->q) * KT * 8, st, g->ctl, g->n, s, g->sc_items, in,
                g->outdeg, g->png_src, g->png_blk, g->seg_delta, g->ppr_upd, g->eprime);
  PCPM_LAUNCH("pcpm_ppr_gather", (k_ppr_gather<KT, kPng>), dim3(static_cast<unsigned>(g->n_ga)),
              dim3(kPprGatherBlock), static_cast<size_t>(g->q) * KT * 8, st, g->ctl, g->n, s, g->ga_items, g->did,
              g->did_blk, g->did_sblk, g->seg_delta, g->ppr_upd, in, out, g->dmask, g->ppr_mask, g->ppr_partial,
              g->ppr_red, g->ppr_vctl);
  return PCPM_OK;
}

template <int KT>
static pcpm_status_t ppr_iteration(pcpm_png* g, const float* in, float* out, float* pr_out, int k, double d,
                                   hipStream_t st) {
  const int s = g->part_log2;
  PCPM_TRY(g->png_order ? (ppr_scatter_gather<KT, true>(g, in, out, st)) : (ppr_scatter_gather<KT, false>(g, in, out, st)));
  if (g->n_mg)
    PCPM_LAUNCH("pcpm_ppr_merge", k_ppr_merge<KT>, dim3(static_cast<unsigned>(g->n_mg)), dim3(kPprBlock), 0, st,
                g->ctl, g->n, s, g->mg_items, g->ppr_partial, in, out, g->dmask, g->ppr_mask, g->ppr_red, g->k,
                g->ppr_vctl);
  PCPM_LAUNCH("pcpm_ppr_finalize", k_ppr_finalize, dim3(1), dim3(1024), 0, st, g->ctl, g->ppr_vctl, KT, g->ppr_red,
              g->k + g->n_mg, g->hist, g->ppr_queue, g->ppr_out_it, g->ppr_out_res, g->ppr_out_conv);
  if (k <= KT) return PCPM_OK;  // one tile: no refill, the columns are stored at the end
  const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((g->n + 255) / 256, 4096));
  PCPM_LAUNCH("pcpm_ppr_refill", k_ppr_refill_cols<KT>, dim3(blocks), dim3(256), 0, st, g->ppr_queue, out, pr_out,
              g->n, k);
  PCPM_LAUNCH("pcpm_ppr_refill", k_ppr_refill_seeds, dim3(1), dim3(1024), 0, st, g->ppr_queue, out, g->ppr_mask,
              g->ppr_seeds, g->ppr_seed_off, KT, g->ppr_vctl, g->dmask, d);
  return PCPM_OK;
}

// Working set for tiles of kt vectors (kept in the handle, grown on demand).
static pcpm_status_t ppr_alloc(pcpm_png* g, int kt, int64_t nseeds, int k) {
  if (g->ppr_kt < kt) {
    for (void* p : {static_cast<void*>(g->ppr_x[0]), static_cast<void*>(g->ppr_x[1]),
                    static_cast<void*>(g->ppr_upd), static_cast<void*>(g->ppr_partial),
                    static_cast<void*>(g->ppr_red), static_cast<void*>(g->ppr_vctl), static_cast<void*>(g->ppr_mask)})
      if (p) dfree(g, p);
    g->ppr_kt = 0;
    PCPM_TRY(dalloc(g, &g->ppr_x[0], g->n * kt));
    PCPM_TRY(dalloc(g, &g->ppr_x[1], g->n * kt));
    PCPM_TRY(dalloc(g, &g->ppr_upd, (g->eprime + 1) * kt));
    PCPM_TRY(dalloc(g, &g->ppr_partial, static_cast<int64_t>(g->n_split_slots) * g->q * kt));
    PCPM_TRY(dalloc(g, &g->ppr_red, (g->k + g->n_mg) * kt * 3));
    PCPM_TRY(dalloc(g, &g->ppr_vctl, kt));
    PCPM_TRY(dalloc(g, &g->ppr_mask, g->n));
    g->ppr_kt = kt;
  }
  if (g->ppr_seed_cap < nseeds) {
    if (g->ppr_seeds) dfree(g, g->ppr_seeds);
    g->ppr_seeds = nullptr;
    PCPM_TRY(dalloc(g, &g->ppr_seeds, nseeds));
    g->ppr_seed_cap = nseeds;
  }
  if (g->ppr_off_cap < k + 1) {
    if (g->ppr_seed_off) dfree(g, g->ppr_seed_off);
    g->ppr_seed_off = nullptr;
    PCPM_TRY(dalloc(g, &g->ppr_seed_off, k + 1));
    g->ppr_off_cap = k + 1;
  }
  if (g->ppr_vec_cap < k) {
    for (void* p : {static_cast<void*>(g->ppr_out_it), static_cast<void*>(g->ppr_out_res),
                    static_cast<void*>(g->ppr_out_conv)})
      if (p) dfree(g, p);
    g->ppr_out_it = g->ppr_out_conv = nullptr;
    g->ppr_out_res = nullptr;
    g->ppr_vec_cap = 0;
    PCPM_TRY(dalloc(g, &g->ppr_out_it, k));
    PCPM_TRY(dalloc(g, &g->ppr_out_res, k));
    PCPM_TRY(dalloc(g, &g->ppr_out_conv, k));
    g->ppr_vec_cap = k;
  }
  if (!g->ppr_queue) PCPM_TRY(dalloc(g, &g->ppr_queue, 1));
  if (!g->ppr_vctl_host)
    PCPM_TRY_HIP(hipHostMalloc(reinterpret_cast<void**>(&g->ppr_vctl_host), sizeof(VCtl) * 64, hipHostMallocDefault));
  return PCPM_OK;
}

template <int KT>
static pcpm_status_t ppr_run(pcpm_png* g, double d, int k, double tol, int max_iters, float* pr_out, int32_t* iters,
                             double* resid, hipStream_t st, bool* all_converged, bool* nonfinite) {
  PCPM_TRY(ppr_set_lds<KT>(g->part_log2));
  const int64_t n = g->n;
  *all_converged = true;
  *nonfinite = false;
  // slots of split bins are never written by the gather: keep them zero
  PCPM_TRY_HIP(hipMemsetAsync(g->ppr_red, 0, static_cast<size_t>((g->k + g->n_mg) * KT * 3) * 8, st));
  const int kv = std::min(KT, k);
  float* a = g->ppr_x[0];
  float* b = g->ppr_x[1];
  PCPM_TRY_HIP(hipMemsetAsync(a, 0, static_cast<size_t>(n) * KT * 4, st));
  PCPM_TRY_HIP(hipMemsetAsync(g->ppr_mask, 0, static_cast<size_t>(n) * 4, st));
  PCPM_LAUNCH("pcpm_ppr_init", k_ppr_ctl, dim3(1), dim3(64), 0, st, g->ctl, tol, d);
  PCPM_LAUNCH("pcpm_ppr_init", k_ppr_seed, dim3(1), dim3(1024), 0, st, a, g->ppr_mask, g->ppr_seeds,
              g->ppr_seed_off, 0, kv, KT, g->ppr_vctl, g->dmask, d);
  PCPM_LAUNCH("pcpm_ppr_init", k_ppr_queue_init, dim3(1), dim3(64), 0, st, g->ppr_queue, kv, k, max_iters);
  // Every slot is busy while vectors wait, so the queue is empty after at
  // most ceil(k/KT) * max_iters iterations, and the last vectors finish
  // within max_iters more.
  const int64_t cap = (static_cast<int64_t>(k + KT - 1) / KT + 1) * max_iters;
  int grid = 0;
  PCPM_TRY(ppr_persist_grid<KT>(g, &grid));
  Ctl c{};
  if (grid > 0) {
    PCPM_TRY(ppr_run_persistent<KT>(g, grid, d, k, cap, pr_out, a, b, st));  // every iteration it needed
    c = g->ctl_host[0];
  } else {
    PCPM_TRY(pipelined_iterations(
        g, tol, cap, st,
        [&](int64_t it) {
          return (it % 2) == 0 ? ppr_iteration<KT>(g, a, b, pr_out, k, d, st)
                               : ppr_iteration<KT>(g, b, a, pr_out, k, d, st);
        },
        &c));
  }
  if (!c.done)
    return set_error(PCPM_ERR_DEVICE, "personalised PageRank did not drain its queue in %d iterations (cap %lld)",
                     c.iter, static_cast<long long>(cap));
  if (k <= KT) {
    const int it_done = c.iter;
    const float* xr = (it_done > 0 && ((it_done - 1) % 2) == 0) ? b : a;
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((n * k + 255) / 256, 8192));
    PCPM_LAUNCH("pcpm_ppr_store", k_ppr_store, dim3(blocks), dim3(256), 0, st, pr_out, xr, n, k, k, KT);
  }
  std::vector<int32_t> it(k), conv(k);
  PCPM_TRY_HIP(hipMemcpyAsync(it.data(), g->ppr_out_it, static_cast<size_t>(k) * 4, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipMemcpyAsync(resid, g->ppr_out_res, static_cast<size_t>(k) * 8, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipMemcpyAsync(conv.data(), g->ppr_out_conv, static_cast<size_t>(k) * 4, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  for (int j = 0; j < k; ++j) {
    iters[j] = it[j];
    if (!conv[j]) *all_converged = false;
  }
  if (c.nonfinite) *nonfinite = true;
  return PCPM_OK;
}

static pcpm_status_t check_device_ppr(pcpm_png* g) {
  int dev = -1;
  PCPM_TRY_HIP(hipGetDevice(&dev));
  if (dev != g->device)
    return set_error(PCPM_ERR_INVALID_ARG, "handle lives on device %d but device %d is current", g->device, dev);
  return PCPM_OK;
}

}  // namespace pcpm

extern "C" {

pcpm_status_t pcpm_ppr_batch(pcpm_png_t g, double d, int32_t k, const int32_t* seed_off, const int32_t* seeds,
                             double tol, int32_t max_iters, float* pr_out, int32_t* iters, double* resid,
                             void* stream) {
  using namespace pcpm;
  if (!g || !seed_off || !seeds || !pr_out || !iters || !resid)
    return set_error(PCPM_ERR_INVALID_ARG, "NULL handle, seed list or output");
  if (g->ngroups != 1 || g->matrix)
    return set_error(PCPM_ERR_INVALID_ARG, "personalised PageRank needs a single-graph handle (not a matrix)");
  if (k < 1) return set_error(PCPM_ERR_INVALID_ARG, "k must be >= 1");
  if (!(d >= 0.0 && d < 1.0)) return set_error(PCPM_ERR_INVALID_ARG, "d must lie in [0, 1)");
  if (max_iters < 1 || max_iters > kMaxHist)
    return set_error(PCPM_ERR_INVALID_ARG, "max_iters must lie in [1, %d]", kMaxHist);
  if (!(tol == tol)) return set_error(PCPM_ERR_INVALID_ARG, "tol is NaN");
  PCPM_TRY(check_device_ppr(g));
  // validate the seed sets on the host: non-empty, in range, distinct
  if (seed_off[0] != 0) return set_error(PCPM_ERR_INVALID_ARG, "seed_off[0] must be 0");
  std::vector<int32_t> scratch;
  for (int j = 0; j < k; ++j) {
    const int32_t a = seed_off[j], b = seed_off[j + 1];
    if (b <= a) return set_error(PCPM_ERR_INVALID_ARG, "seed set %d is empty", j);
    scratch.assign(seeds + a, seeds + b);
    std::sort(scratch.begin(), scratch.end());
    if (scratch.front() < 0 || scratch.back() >= g->n)
      return set_error(PCPM_ERR_INVALID_ARG, "seed set %d has a node outside [0, n)", j);
    if (std::adjacent_find(scratch.begin(), scratch.end()) != scratch.end())
      return set_error(PCPM_ERR_INVALID_ARG, "seed set %d repeats a node", j);
  }
  // kt vectors per tile: q * kt fixed-point sums must fit the LDS slice
  int kt_max = std::max(1, std::min(16, (1 << kMaxLog2) >> g->part_log2));
  int kt = 1;
  while (kt < k && kt < kt_max) kt <<= 1;
  hipStream_t st = static_cast<hipStream_t>(stream);
  PCPM_TRY(ppr_alloc(g, kt, seed_off[k], k));
  PCPM_TRY_HIP(hipMemcpyAsync(g->ppr_seeds, seeds, static_cast<size_t>(seed_off[k]) * 4, hipMemcpyHostToDevice, st));
  PCPM_TRY_HIP(hipMemcpyAsync(g->ppr_seed_off, seed_off, static_cast<size_t>(k + 1) * 4, hipMemcpyHostToDevice, st));
  bool conv = true, bad = false;
  pcpm_status_t rc;
  switch (kt) {
    case 1: rc = ppr_run<1>(g, d, k, tol, max_iters, pr_out, iters, resid, st, &conv, &bad); break;
    case 2: rc = ppr_run<2>(g, d, k, tol, max_iters, pr_out, iters, resid, st, &conv, &bad); break;
    case 4: rc = ppr_run<4>(g, d, k, tol, max_iters, pr_out, iters, resid, st, &conv, &bad); break;
    case 8: rc = ppr_run<8>(g, d, k, tol, max_iters, pr_out, iters, resid, st, &conv, &bad); break;
    default: rc = ppr_run<16>(g, d, k, tol, max_iters, pr_out, iters, resid, st, &conv, &bad); break;
  }
  if (rc != PCPM_OK) return rc;
  if (bad) return set_error(PCPM_ERR_NUMERIC, "non-finite residual or dangling mass");
  if (tol > 0.0 && !conv) return set_error(PCPM_ERR_NOT_CONVERGED, "some vectors are above tol after max_iters");
  return PCPM_OK;
}

int32_t pcpm_ppr_tile_width(pcpm_png_t g) {
  if (!g) return 0;
  return std::max(1, std::min(16, (1 << pcpm::kMaxLog2) >> g->part_log2));
}

}  // extern "C"
