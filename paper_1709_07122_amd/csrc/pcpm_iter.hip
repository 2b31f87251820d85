// One PCPM PageRank iteration on the GPU: scatter (Alg. 3 over the PNG),
// gather (Alg. 5, branch-free) with the apply of Alg. 2 fused into its
// epilogue, and an FP64 reduction of the L1 residual and the dangling mass.
//
// Per iteration, on the caller's stream:
//   k_scatter   one workgroup per scatter item (a range of one source
//               partition pair's PNG edges): the pair's scaled ranks
//               PR(u)/outdeg(u) are staged in LDS and PNG edges are streamed.
//               Each XCD runs one contiguous range of the item array.
//   k_gather    one workgroup per gather item (a range of one destination
//               bin): destination IDs are streamed, the update of an ID is
//               found from the running count of message flags, and sums
//               build up in an LDS slice of the destination partition.
//               A whole bin is applied in place; a split bin stores its
//               partial slice for k_merge.
//   k_merge     applies split bins, adding their partial slices in order;
//               one workgroup per slice of a split bin's nodes.
//   k_finalize  one workgroup: residual and next dangling mass in FP64, in a
//               fixed order; sets the convergence flag that makes the kernels
//               of later iterations return at once.
//
// Updates are stored in one of two orders, chosen per handle at build time:
//   bin order   (Sec. 3.1) the updates of bin p' are contiguous, in message
//               order; the scatter writes one run per (pair, bin) segment at
//               the segment's write offset, and the gather reads its bin's
//               updates in sequence.
//   PNG order   update e belongs to PNG edge e: the scatter's stores are one
//               contiguous stream, and the gather reads one run per (bin,
//               pair) segment, locating an ID's update as its message index
//               plus its segment's delta (segment flags on the IDs).
// Short segments make the scatter's runs of writes costly on HBM (partial
// lines, scattered rows), while runs of reads cost less; the build takes PNG
// order when the average segment is short.
//
// Sums in the gather are kept in 64-bit fixed point: every FP32 update is
// rounded to a multiple of 2^-fx_shift and added with LDS integer atomics.
// Integer addition is associative, so the ranks do not depend on the order
// in which wavefronts add, and split bins merge exactly.  The scale follows
// the iterate: an update is at most the largest value of the vector it comes
// from, so fx_shift = 50 - ceil(log2(max x)) keeps every converted update
// below 2^50, and the sums (at most the vector's mass) below 2^63 when
// fx_shift <= 61 - ceil(log2(mass)).  The first iteration takes the start
// vector's mass as the bound; each later one the largest value of the
// previous iterate, which the apply reports.  With ranks of a large graph
// near 1/n, this keeps the rounding of an update far below FP32 resolution.
#include <algorithm>
#include <cmath>

#include "pcpm_device.hpp"
#include "pcpm_internal.hpp"

namespace pcpm {

constexpr int kMergeNodes = 256;  // nodes per merge workgroup (one per thread)

// Apply (Alg. 2) for nodes v0+i0 .. v0+i1-1 of partition `part`:
//   x_new(v) = d * acc(v) + base_g,  base_g = (1-d)/n_g + d*D_g/n_g
// for the partition's group g, plus their share of sum |x_new - x_old| and of
// the next dangling mass.  Padding nodes (past the group's last node) stay 0;
// a converged group keeps its iterate.  G > 1: the workgroup holds G groups
// of BS threads, each applying its own range (an empty one, with red_slot
// NULL, for a group without work); every thread calls it, and each group
// computes exactly what a workgroup of BS threads computes.
//
// The apply's node loads: kU nodes per thread per step, all issued before
// any is used, so their latencies overlap; a 1024-thread gather covers a
// whole 16K-node slice in one step.
template <int BS>
struct NodeLoads {
  static constexpr int kU = BS >= 1024 ? 16 : 4;
  float xo[kU];     // previous iterate
  uint32_t dw[kU];  // dangling-mask word of each node
  // thread-relative node i of the range [.., i1) and the kU-1 nodes BS apart
  __device__ __forceinline__ void load(const float* __restrict__ pr_in, const uint32_t* __restrict__ dmask,
                                       int64_t v0, int i, int i1) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t v = v0 + min(i + u * BS, i1 - 1);
      xo[u] = pr_in[v];
      dw[u] = dmask[v >> 5];
    }
  }
};

// kPre: the caller has loaded this thread's nodes into *pre, and the range
// fits in one step (i1 - i0 <= kU * BS).
template <int BS, class AccFn, int G = 1, bool kPre = false>
__device__ __forceinline__ void apply_nodes(const Ctl* __restrict__ ctl, const GCtl* __restrict__ gctl,
                                            const int32_t* __restrict__ part_group,
                                            const int32_t* __restrict__ part_valid, int part, int64_t v0, int i0,
                                            int i1, AccFn acc, const float* __restrict__ pr_in,
                                            float* __restrict__ pr_out, const uint32_t* __restrict__ dmask,
                                            double* __restrict__ red_slot, const NodeLoads<BS>* pre = nullptr) {
  const int tid = static_cast<int>(threadIdx.x % BS);
  const GCtl& gc = gctl[part_group[part]];
  const double base = gc.base;
  const bool frozen = gc.done != 0;
  const int valid = part_valid[part];
  const double d = ctl->d;
  const double unit = ldexp(1.0, -ctl->fx_shift);
  double sums[2] = {0.0, 0.0};  // residual, dangling mass
  float mx = 0.0f;               // largest new value: the next fixed-point scale
  constexpr int kU = NodeLoads<BS>::kU;
  auto step = [&](int i, const NodeLoads<BS>& nl) {
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int ii = i + u * BS;
      if (ii < i1) {
        const int64_t v = v0 + ii;
        float xn = 0.0f;
        if (ii < valid) {
          const double sv = static_cast<double>(acc(ii)) * unit;
          xn = frozen ? nl.xo[u] : static_cast<float>(fma(d, sv, base));
        }
        mx = fmaxf(mx, fabsf(xn));
        sums[0] += fabs(static_cast<double>(xn) - static_cast<double>(nl.xo[u]));
        if ((nl.dw[u] >> (v & 31)) & 1u) sums[1] += static_cast<double>(xn);
        __builtin_nontemporal_store(xn, pr_out + v);  // read by the next scatter, not this kernel
      }
    }
  };
  if constexpr (kPre) {
    if (i0 + tid < i1) step(i0 + tid, *pre);
  } else {
    for (int i = i0 + tid; i < i1; i += kU * BS) {
      NodeLoads<BS> nl;
      nl.load(pr_in, dmask, v0, i, i1);
      step(i, nl);
    }
  }
  group_sum<BS, G>(sums);
  const double vmax = group_max<BS, G>(static_cast<double>(mx));
  if (tid == 0 && red_slot) {
    red_slot[0] = sums[0];
    red_slot[1] = sums[1];
    red_slot[2] = vmax;
  }
}

// One scatter item (a range of one source pair's PNG edges) by the whole
// workgroup; spr is its LDS staging area (2q floats).
// kScale: stage PR(u)/outdeg(u) (PageRank); otherwise x(u) itself (SpMV).
// kPng: updates in PNG order, else in bin order.
template <int BS, bool kScale, bool kPng>
__device__ __forceinline__ void scatter_item(const Item it, float* __restrict__ spr, int64_t n, int s,
                                             const float* __restrict__ pr, const int32_t* __restrict__ outdeg,
                                             const uint16_t* __restrict__ png_src,
                                             const int32_t* __restrict__ png_blk,
                                             const int32_t* __restrict__ seg_delta, float* __restrict__ upd,
                                             int64_t spare) {
  // a scatter item covers PNG edges of one partition pair: stage both slices
  const int64_t v0 = static_cast<int64_t>(it.part) << (s + 1);
  const int qn = static_cast<int>(min(int64_t{2} << s, n - v0));
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t lo = it.lo, hi = it.hi;
  const int64_t t_end = (hi + kTile - 1) / kTile;
  constexpr int kNW = BS / kWave;
  uint32_t w[kPairs], wn[kPairs];
  int64_t t = lo / kTile + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  // the first tile's source IDs (bin order: also its pair-segment counts and
  // deltas, and the counts of the next tile) are in flight during the staging
  int32_t cv = 0, cvn = 0, dl = 0;
  if (t < t_end) {
    load_tile_words(png_src + t * kTile, lane, w);
    if constexpr (!kPng) {
      cv = load_counts(png_blk, nullptr, t, lane);
      if (t + kNW < t_end) cvn = load_counts(png_blk, nullptr, t + kNW, lane);
    }
  }
  // kSU nodes per thread per step, loads first, so their latencies overlap
  constexpr int kSU = 8;
  for (int i0 = threadIdx.x; i0 < qn; i0 += kSU * BS) {
    float xv[kSU];
    int od[kSU];
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      const int64_t v = v0 + min(i0 + u * BS, qn - 1);
      xv[u] = pr[v];
      if constexpr (kScale) od[u] = outdeg[v];
    }
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      const int i = i0 + u * BS;
      if (i < qn) {
        if constexpr (kScale) spr[i] = od[u] > 0 ? xv[u] / static_cast<float>(od[u]) : 0.0f;
        else spr[i] = xv[u];
      }
    }
  }
  if constexpr (!kPng) {
    if (t < t_end) dl = tile_deltas(seg_delta, __builtin_amdgcn_readlane(cv, 0), lane);
  }
  __syncthreads();
  const uint32_t qmask = (2u << s) - 1u;  // source IDs are local to the pair
  for (; t < t_end; t += kNW) {
    const int64_t tb = t * kTile;
    // the next tile's loads overlap this tile's work
    int32_t dln = 0, cvnn = 0;
    if (t + kNW < t_end) {
      load_tile_words(png_src + (t + kNW) * kTile, lane, wn);
      if constexpr (!kPng) {
        dln = tile_deltas(seg_delta, __builtin_amdgcn_readlane(cvn, 0), lane);
        if (t + 2 * kNW < t_end) cvnn = load_counts(png_blk, nullptr, t + 2 * kNW, lane);
      }
    }
    uint32_t x[kSub];
    unpack_tile(w, x);
    if constexpr (kPng) {
      // PNG edge e writes upd[e]: a tile's stores are one contiguous run of
      // whole lines, written non-temporally (measured: the gather that reads
      // them is ~2% faster at RMAT-26 EF24).  A source ID masked with 2q-1 is
      // its slot in the pair's rank slice.
      if (tb >= lo && tb + kTile <= hi) {
        float* ut = upd + tb;
#pragma unroll
        for (int j = 0; j < kSub; ++j) __builtin_nontemporal_store(spr[x[j] & qmask], ut + j * kWave + lane);
      } else {
#pragma unroll
        for (int j = 0; j < kSub; ++j) {
          const int64_t e = tb + j * kWave + lane;
          if (e >= lo && e < hi) __builtin_nontemporal_store(spr[x[j] & qmask], upd + e);
        }
      }
    } else {
      // Every entry of a tile has a valid segment index (entry 0 of the array
      // is flagged and padding follows the last segment), so the loads below
      // need no predicate.  A source ID masked with 2q-1 is its slot in the
      // pair's rank slice (entries of other pairs, in edge tiles, only read a
      // stale slot and store to the spare update slot E').
      // The segment index counts pair-segment flags as the gather counts
      // messages (flags before the tile: lane 0 of cv); the deltas of the
      // tile's first 64 segments came in with the tile (dl), others are read.
      const int32_t sb = __builtin_amdgcn_readlane(cv, 0);
      int32_t run = sb - 1;
      int32_t seg[kSub];
#pragma unroll
      for (int j = 0; j < kSub; ++j) {
        const bool f = (x[j] & kDidFlag) != 0u;
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
        float* ut = upd + tb;
#pragma unroll
        for (int j = 0; j < kSub; ++j) ut[static_cast<int64_t>(j * kWave + lane + d[j])] = spr[x[j] & qmask];
      } else {
#pragma unroll
        for (int j = 0; j < kSub; ++j) {
          const int64_t e = tb + j * kWave + lane;
          const bool in = e >= lo && e < hi;
          upd[in ? e + d[j] : spare] = spr[x[j] & qmask];
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

template <int BS, bool kScale, bool kPng>
__global__ __launch_bounds__(BS) void k_scatter(const Ctl* __restrict__ ctl, int64_t n, int s,
                                                const Item* __restrict__ items, const float* __restrict__ pr,
                                                const int32_t* __restrict__ outdeg,
                                                const uint16_t* __restrict__ png_src,
                                                const int32_t* __restrict__ png_blk,
                                                const int32_t* __restrict__ seg_delta, float* __restrict__ upd,
                                                int64_t spare) {
  if (ctl->done) return;
  extern __shared__ float spr[];
  // XCD-contiguous renumbering (the build arranges the item array for it)
  scatter_item<BS, kScale, kPng>(items[xcd_block(blockIdx.x, gridDim.x)], spr, n, s, pr, outdeg, png_src, png_blk,
                                 seg_delta, upd, spare);
}

// kMode 0: PageRank (apply, residual, dangling mass); 1: SpMV, y(v) = sum of
// the updates; 2: SpMV with the edge weight stored beside each destination ID
// applied to its update (Sec. 3.5).  In SpMV modes pr_out receives y.
// kPng: updates in PNG order (an ID's update is at its message index plus
// its segment's delta), else in bin order (at its message index).
// One gather item (a range of one bin's destination IDs) by the whole
// workgroup; acc is its LDS slice (q 64-bit sums).
// kEarlyApply: the apply's node loads go out before the final barrier (the
// persistent kernel, short of registers already, leaves them where they are).
template <int BS, int kMode, bool kPng, bool kEarlyApply = true>
__device__ __forceinline__ void gather_item(const Item it, unsigned long long* __restrict__ acc,
                                            const Ctl* __restrict__ ctl, int64_t n, int s,
                                            const uint16_t* __restrict__ did, const int32_t* __restrict__ did_blk,
                                            const int32_t* __restrict__ did_sblk,
                                            const int32_t* __restrict__ seg_delta, const float* __restrict__ upd,
                                            const float* __restrict__ pr_in, float* __restrict__ pr_out,
                                            const uint32_t* __restrict__ dmask, int64_t* __restrict__ partial,
                                            double* __restrict__ red, const GCtl* __restrict__ gctl,
                                            const int32_t* __restrict__ part_group,
                                            const int32_t* __restrict__ part_valid,
                                            const float* __restrict__ wbin) {
  const int64_t q = int64_t{1} << s;
  const int64_t v0 = static_cast<int64_t>(it.part) << s;
  const int qn = static_cast<int>(min(q, n - v0));
  const FixedConv to_fixed(ctl->fx_shift);
  const uint32_t qmask = static_cast<uint32_t>(q - 1);
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t lo = it.lo, hi = it.hi;
  const int64_t t_end = (hi + kTile - 1) / kTile;
  constexpr int kNW = BS / kWave;
  // Each wavefront walks every kNW-th tile.  Its loads go out in this order:
  // this tile's updates, then the next tile's IDs and segment deltas and the
  // flag counts of the tile after that.  Loads return in order, so the wait
  // for the updates does not wait for the prefetches, which stay in flight
  // through this tile's adds.
  uint32_t w[kPairs], wn[kPairs];
  const int64_t t0 = lo / kTile + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int32_t* sblk_arr = kPng ? did_sblk : nullptr;
  int32_t cv = 0, cvn = 0, dl = 0;
  // The first tiles' loads go out before the slice is cleared and stay in
  // flight through the clear and the barrier.  Not in the weighted gather:
  // there the registers they hold through the clear make the loop spill.
  constexpr bool kEarly = kMode != 2;
  if constexpr (!kEarly) {
    for (int i = threadIdx.x; i < qn; i += BS) acc[i] = 0ull;
    __syncthreads();
  }
  if (t0 < t_end) {
    load_tile_words(did + t0 * kTile, lane, w);
    cv = load_counts(did_blk, sblk_arr, t0, lane);
    if (t0 + kNW < t_end) cvn = load_counts(did_blk, sblk_arr, t0 + kNW, lane);
  }
  if constexpr (kEarly) {
    for (int i = threadIdx.x; i < qn; i += BS) acc[i] = 0ull;
  }
  if constexpr (kPng) {
    if (t0 < t_end) dl = tile_deltas(seg_delta, __builtin_amdgcn_readlane(cv, 1), lane);
  }
  if constexpr (kEarly) __syncthreads();
  for (int64_t t = t0; t < t_end; t += kNW) {
    const int64_t tb = t * kTile;
    const int32_t blk = __builtin_amdgcn_readlane(cv, 0);
    uint32_t x[kSub];
    unpack_tile(w, x);
    // Every entry has a valid update slot (entry 0 of the array carries
    // every flag and padding follows the last message), so the update loads
    // need no predicate.
    float val[kSub];
    if constexpr (kPng) {
      int32_t msg[kSub];
      tile_slots<true>(x, blk, __builtin_amdgcn_readlane(cv, 1), dl, seg_delta, msg);
#pragma unroll
      for (int j = 0; j < kSub; ++j) val[j] = upd[msg[j]];
    } else {
      // a tile's updates lie in [blk-1, blk_next-1]: a per-tile base and
      // 32-bit lane offsets
      const char* ub = reinterpret_cast<const char*>(upd) + (static_cast<int64_t>(blk) - 1) * 4;
      int32_t run = 0;  // flags in the earlier sub-blocks of this tile
      uint32_t off[kSub];
#pragma unroll
      for (int j = 0; j < kSub; ++j) {
        const bool f = (x[j] & kDidFlag) != 0u;
        const uint64_t bal = wave_ballot(f);
        off[j] = static_cast<uint32_t>(run + lanes_below(bal) + (f ? 1 : 0)) * 4u;
        run += __popcll(bal);
      }
#pragma unroll
      for (int j = 0; j < kSub; ++j) val[j] = *reinterpret_cast<const float*>(ub + off[j]);
    }
    // weights are stored in bin order, padded to whole tiles
    float wv[kMode == 2 ? kSub : 1];
    if constexpr (kMode == 2) {
#pragma unroll
      for (int j = 0; j < kSub; ++j) wv[j] = wbin[tb + j * kWave + lane];
    }
    // prefetch: the next tile's IDs and deltas, the counts of the one after
    int32_t dln = 0, cvnn = 0;
    if (t + kNW < t_end) {
      load_tile_words(did + (t + kNW) * kTile, lane, wn);
      if constexpr (kPng) dln = tile_deltas(seg_delta, __builtin_amdgcn_readlane(cvn, 1), lane);
      if (t + 2 * kNW < t_end) cvnn = load_counts(did_blk, sblk_arr, t + 2 * kNW, lane);
    }
    // the update (times its weight, formed exactly in FP64) as a fixed-point integer
    auto fixed = [&](int j) -> int64_t {
      if constexpr (kMode == 2) return to_fixed(static_cast<double>(wv[j]) * static_cast<double>(val[j]));
      else return to_fixed(val[j]);
    };
    if (tb >= lo && tb + kTile <= hi) {
#pragma unroll
      for (int j = 0; j < kSub; ++j) atomicAdd(&acc[x[j] & qmask], static_cast<unsigned long long>(fixed(j)));
    } else {  // edge tile: entries outside [lo, hi) add nothing
#pragma unroll
      for (int j = 0; j < kSub; ++j) {
        const int64_t e = tb + j * kWave + lane;
        const bool in = e >= lo && e < hi;
        atomicAdd(&acc[in ? (x[j] & qmask) : 0u], static_cast<unsigned long long>(in ? fixed(j) : 0));
      }
    }
#pragma unroll
    for (int j = 0; j < kPairs; ++j) w[j] = wn[j];
    cv = cvn;
    cvn = cvnn;
    dl = dln;
  }
  // A whole bin's apply is one step of node loads at 1024 threads: they go
  // out before the barrier, while the other wavefronts finish their adds.
  constexpr bool kPre = kEarlyApply && kMode == 0 && NodeLoads<BS>::kU * BS >= (1 << kMaxLog2);
  NodeLoads<BS> pre;
  if constexpr (kPre) {
    if (it.aux < 0 && static_cast<int>(threadIdx.x) < qn) pre.load(pr_in, dmask, v0, threadIdx.x, qn);
  }
  __syncthreads();
  if (it.aux >= 0) {
    int64_t* dst = partial + static_cast<int64_t>(it.aux) * q;
    for (int i = threadIdx.x; i < qn; i += BS) dst[i] = static_cast<int64_t>(acc[i]);
    return;
  }
  if constexpr (kMode != 0) {
    const double unit = ldexp(1.0, -ctl->fx_shift);
    const bool bad = ctl->nonfinite != 0;
    for (int i = threadIdx.x; i < qn; i += BS)
      __builtin_nontemporal_store(
          bad ? __builtin_nanf("") : static_cast<float>(static_cast<double>(static_cast<int64_t>(acc[i])) * unit),
          pr_out + v0 + i);
    return;
  }
  auto slice = [&](int i) { return static_cast<int64_t>(acc[i]); };
  apply_nodes<BS, decltype(slice), 1, kPre>(ctl, gctl, part_group, part_valid, it.part, v0, 0, qn, slice, pr_in,
                                           pr_out, dmask, red + 3 * it.part, &pre);
}

template <int BS, int kMode, bool kPng>
__global__ __launch_bounds__(BS) void k_gather(const Ctl* __restrict__ ctl, int64_t n, int s,
                                               const Item* __restrict__ items, const uint16_t* __restrict__ did,
                                               const int32_t* __restrict__ did_blk,
                                               const int32_t* __restrict__ did_sblk,
                                               const int32_t* __restrict__ seg_delta, const float* __restrict__ upd,
                                               const float* __restrict__ pr_in, float* __restrict__ pr_out,
                                               const uint32_t* __restrict__ dmask, int64_t* __restrict__ partial,
                                               double* __restrict__ red, const GCtl* __restrict__ gctl,
                                               const int32_t* __restrict__ part_group,
                                               const int32_t* __restrict__ part_valid,
                                               const float* __restrict__ wbin) {
  if (ctl->done) return;
  extern __shared__ unsigned long long acc[];
  // the build arranges the item array for the XCD-contiguous renumbering
  gather_item<BS, kMode, kPng>(items[xcd_block(blockIdx.x, gridDim.x)], acc, ctl, n, s, did, did_blk, did_sblk, seg_delta, upd, pr_in,
                               pr_out, dmask, partial, red, gctl, part_group, part_valid, wbin);
}

// Merge unit u of split bins: its nodes' partial slices summed in order, then
// applied; its residual / dangling / largest-value triple goes to slot
// red_base + u.
// G > 1: G groups of BS threads, group g takes unit u (u < 0: no unit);
// every thread of the workgroup calls it.
template <int BS, int G = 1>
__device__ __forceinline__ void merge_unit(const Merge mu, int64_t u, const Ctl* __restrict__ ctl, int64_t n, int s,
                                           const int64_t* __restrict__ partial, const float* __restrict__ pr_in,
                                           float* __restrict__ pr_out, const uint32_t* __restrict__ dmask,
                                           double* __restrict__ red, int64_t red_base,
                                           const GCtl* __restrict__ gctl, const int32_t* __restrict__ part_group,
                                           const int32_t* __restrict__ part_valid) {
  const int64_t q = int64_t{1} << s;
  const int64_t v0 = static_cast<int64_t>(mu.part) << s;
  const int qn = static_cast<int>(min(q, n - v0));
  const int64_t* base = partial + static_cast<int64_t>(mu.first) * q;
  const int cnt = mu.count;
  auto acc = [&](int i) { return sum_slices(base + i, cnt, q); };
  const bool has = u >= 0;
  apply_nodes<BS, decltype(acc), G>(ctl, gctl, part_group, part_valid, mu.part, v0, has ? mu.node_lo : 0,
                                    has ? min(qn, mu.node_lo + kMergeNodes) : 0, acc, pr_in, pr_out, dmask,
                                    has ? red + 3 * (red_base + u) : nullptr);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_merge(const Ctl* __restrict__ ctl, int64_t n, int s,
                                              const Merge* __restrict__ mg, const int64_t* __restrict__ partial,
                                              const float* __restrict__ pr_in, float* __restrict__ pr_out,
                                              const uint32_t* __restrict__ dmask, double* __restrict__ red,
                                              int64_t red_base, const GCtl* __restrict__ gctl,
                                              const int32_t* __restrict__ part_group,
                                              const int32_t* __restrict__ part_valid) {
  if (ctl->done) return;
  merge_unit<BS>(mg[blockIdx.x], blockIdx.x, ctl, n, s, partial, pr_in, pr_out, dmask, red, red_base, gctl,
                 part_group, part_valid);
}

// Per-group totals of the apply units' (residual, dangling, mass) partial
// sums: one wavefront per group, partitions then merge units, in order.
__device__ __forceinline__ void group_sums(const int32_t* __restrict__ group_slots, const double* __restrict__ red,
                                           int64_t k, int grp, bool with_merge, double (&s)[3]) {
  const int lane = threadIdx.x & (kWave - 1);
  s[0] = s[1] = s[2] = 0.0;
  const int p0 = group_slots[2 * grp], p1 = group_slots[2 * grp + 2];
  for (int j = p0 + lane; j < p1; j += kWave)
    for (int c = 0; c < 3; ++c) s[c] += red[3 * j + c];
  if (with_merge) {
    const int u0 = group_slots[2 * grp + 1], u1 = group_slots[2 * grp + 3];
    for (int j = u0 + lane; j < u1; j += kWave)
      for (int c = 0; c < 3; ++c) s[c] += red[3 * (k + j) + c];
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1)
    for (int c = 0; c < 3; ++c) s[c] += __shfl_xor(s[c], off);
}

// A group's apply slots at the end of an iteration: the sums of the residual
// and dangling parts and the largest value of the new iterate.  By one
// wavefront (valid in lane 0, summed in the order of group_sums) or, kBlock,
// by the whole workgroup for few groups (valid in thread 0; a fixed strided
// assignment and reduction order, one barrier), so results are reproducible.
template <bool kBlock>
__device__ __forceinline__ void group_stats(const int32_t* __restrict__ group_slots, const double* __restrict__ red,
                                            int64_t k, int grp, double (&s)[3]) {
  const int t = kBlock ? static_cast<int>(threadIdx.x) : static_cast<int>(threadIdx.x & (kWave - 1));
  constexpr int kStride = kBlock ? 1024 : kWave;
  s[0] = s[1] = s[2] = 0.0;
  const int p0 = group_slots[2 * grp], p1 = group_slots[2 * grp + 2];
  const int u0 = group_slots[2 * grp + 1], u1 = group_slots[2 * grp + 3];
  for (int j = p0 + t; j < p1; j += kStride) {
    s[0] += red[3 * j];
    s[1] += red[3 * j + 1];
    s[2] = fmax(s[2], red[3 * j + 2]);
  }
  for (int j = u0 + t; j < u1; j += kStride) {
    s[0] += red[3 * (k + j)];
    s[1] += red[3 * (k + j) + 1];
    s[2] = fmax(s[2], red[3 * (k + j) + 2]);
  }
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    s[0] += __shfl_xor(s[0], off);
    s[1] += __shfl_xor(s[1], off);
    s[2] = fmax(s[2], __shfl_xor(s[2], off));
  }
  if constexpr (kBlock) {
    constexpr int kW = 1024 / kWave;
    __shared__ double sh[3 * kW];
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0) {
      sh[3 * w] = s[0];
      sh[3 * w + 1] = s[1];
      sh[3 * w + 2] = s[2];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s[0] = s[1] = s[2] = 0.0;
      for (int ww = 0; ww < kW; ++ww) {
        s[0] += sh[3 * ww];
        s[1] += sh[3 * ww + 1];
        s[2] = fmax(s[2], sh[3 * ww + 2]);
      }
    }
  }
}

// End of an iteration: per-group residual, next dangling mass and base, group
// convergence; then the largest residual, the iteration count and the flag
// that makes the kernels of later iterations return at once.  One workgroup
// of 1024 threads.
// Each group's control struct is read and written by one thread only, and
// the workgroup-wide results (largest residual, all converged) go through
// LDS: stores of different wavefronts to global memory are not ordered by a
// workgroup barrier.
__device__ __forceinline__ void finalize_body(Ctl* __restrict__ ctl, GCtl* __restrict__ gctl,
                                              const int32_t* __restrict__ group_slots,
                                              const double* __restrict__ red, int64_t k, int64_t /*nslots*/,
                                              double* __restrict__ hist) {
  constexpr int kW = 1024 / kWave;
  __shared__ int s_bad[kW], s_done[kW];
  __shared__ double s_rmax[kW], s_vmax[kW];
  const int G = ctl->ngroups;
  const double d = ctl->d, tol = ctl->tol;
  // the group's update; returns its residual and convergence after it
  auto update = [&](int grp, const double (&sm)[3], int& bad) -> GCtl {
    GCtl& gc = gctl[grp];
    if (!gc.done) {
      gc.res = sm[0];
      gc.iter += 1;
      gc.dmass = sm[1];
      gc.base = (1.0 - d) * gc.inv_n + d * sm[1] * gc.inv_n;
      if (!isfinite(sm[0]) || !isfinite(sm[1])) bad = 1;
      else if (tol > 0.0 && sm[0] < tol) gc.done = 1;
    }
    return gc;
  };
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  int bad = 0, all_done = 1;
  double rmax = 0.0;
  double vmax = 0.0;  // largest value of the new iterate over all apply units (the groups cover them all)
  if (G < kW) {  // few groups: the whole workgroup sums each one, thread 0 updates it
    for (int grp = 0; grp < G; ++grp) {
      double sm[3];
      group_stats<true>(group_slots, red, k, grp, sm);
      if (threadIdx.x == 0) {
        const GCtl gc = update(grp, sm, bad);
        rmax = fmax(rmax, gc.res);
        all_done &= gc.done;
        vmax = fmax(vmax, sm[2]);
      }
      __syncthreads();
    }
  } else {  // one wavefront per group, lane 0 updates it
    for (int grp = w; grp < G; grp += kW) {
      double sm[3];
      group_stats<false>(group_slots, red, k, grp, sm);
      if (lane == 0) {
        const GCtl gc = update(grp, sm, bad);
        rmax = fmax(rmax, gc.res);
        all_done &= gc.done;
        vmax = fmax(vmax, sm[2]);
      }
    }
  }
  if (lane == 0) {
    s_bad[w] = bad;
    s_done[w] = all_done;
    s_rmax[w] = rmax;
    s_vmax[w] = vmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int ww = 1; ww < kW; ++ww) {
      bad |= s_bad[ww];
      all_done &= s_done[ww];
      rmax = fmax(rmax, s_rmax[ww]);
      vmax = fmax(vmax, s_vmax[ww]);
    }
    if (bad) rmax = NAN;
    const int32_t it = ctl->iter;
    ctl->res_prev = ctl->res;
    ctl->res = rmax;
    hist[it] = rmax;
    ctl->iter = it + 1;
    if (bad) ctl->nonfinite = 1;
    if (bad || all_done) ctl->done = 1;
    ctl->fx_shift = fx_shift_for(vmax, ctl->fx_cap);
  }
}

__global__ __launch_bounds__(1024) void k_finalize(Ctl* __restrict__ ctl, GCtl* __restrict__ gctl,
                                                   const int32_t* __restrict__ group_slots,
                                                   const double* __restrict__ red, int64_t k, int64_t nslots,
                                                   double* __restrict__ hist) {
  if (ctl->done) return;
  finalize_body(ctl, gctl, group_slots, red, k, nslots, hist);
}

// ---- persistent solve ------------------------------------------------------------------
// Every iteration of a solve in one cooperative launch (every workgroup
// resident, one per CU at a 128 KB slice).  Per iteration:
//   1. scatter items, each XCD's workgroups taking its contiguous range;
//   2. grid barrier;
//   3. gather items (largest first), then merge units, from one counter; a
//      split bin's items count themselves finished in bin_done, and its
//      merge units wait for that count; every apply unit (a whole-bin item
//      or a merge unit) counts itself finished, and the workgroup that
//      finishes the last one runs the finalize (FP64 sums, convergence);
//   4. grid barrier (its last arrival resets the work counters); every
//      workgroup reads the convergence flag and leaves when it is set.
// Waits are bounded (PSync::err), so the kernel ends in every case.

__global__ __launch_bounds__(256) void k_persist_init(PSync* __restrict__ ps, int32_t* __restrict__ bin_done,
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

template <bool kPng>
__global__ __launch_bounds__(1024) void k_persist(const PersistArgs a) {
  constexpr int BS = 1024;
  constexpr int kMG = BS / kMergeNodes;  // merge units per workgroup, one per group of 256 threads
  extern __shared__ unsigned long long lds[];
  PSync* ps = a.ps;
  auto reset = [&]() {  // by the last arrival at the iteration's second barrier
    for (unsigned x = 0; x < kXcds; ++x) __hip_atomic_store(&ps->sc_next[x], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ps->ga_next, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ps->mg_next, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&ps->applied, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  for (int32_t it = 0; it < a.max_iters; ++it) {
    const float* in = (it & 1) ? a.x1 : a.x0;
    float* out = (it & 1) ? a.x0 : a.x1;
    for (;;) {
      const int32_t j = grab_scatter(ps, a.n_sc);
      if (j < 0) break;
      scatter_item<BS, true, kPng>(a.sc_items[j], reinterpret_cast<float*>(lds), a.n, a.s, in, a.outdeg, a.png_src,
                                   a.png_blk, a.seg_delta, a.upd, a.spare);
    }
    if (!grid_sync(ps, a.spin_limit, [] {})) return;
    for (;;) {  // gather items in the order of a launch per phase
      const int32_t j = grab(&ps->ga_next);
      if (j >= a.n_ga) break;
      const Item itm = a.ga_items[xcd_block(static_cast<unsigned>(j), static_cast<unsigned>(a.n_ga))];
      gather_item<BS, 0, kPng, false>(itm, lds, a.ctl, a.n, a.s, a.did, a.did_blk, a.did_sblk, a.seg_delta, a.upd, in, out,
                               a.dmask, a.partial, a.red, a.gctl, a.part_group, a.part_valid, nullptr);
      if (itm.aux >= 0) {  // a split bin's slice: applied by its merge units
        publish(&a.bin_done[itm.part]);
      } else if (publish(&ps->applied) == a.n_apply - 1) {  // the iteration's last apply unit
        finalize_body(a.ctl, a.gctl, a.group_slots, a.red, a.k, a.k + a.n_mg, a.hist);
      }
    }
    for (;;) {  // merge units of split bins, kMG at a time
      const int32_t u0 = grab(&ps->mg_next, kMG);
      if (u0 >= a.n_mg) break;
      const int32_t cnt = min(kMG, a.n_mg - u0);
      for (int32_t c = 0; c < cnt; ++c) {  // every bin of these units has all its slices
        const Merge mc = a.mg_items[u0 + c];
        if (c > 0 && mc.part == a.mg_items[u0 + c - 1].part) continue;
        const int32_t target = static_cast<int32_t>(static_cast<uint32_t>(mc.count) * static_cast<uint32_t>(it + 1));
        if (!wait_at_least(ps, &a.bin_done[mc.part], target, a.spin_limit)) return;
      }
      const int g = static_cast<int>(threadIdx.x) / kMergeNodes;
      merge_unit<kMergeNodes, kMG>(a.mg_items[u0 + (g < cnt ? g : 0)], g < cnt ? u0 + g : -1, a.ctl, a.n, a.s,
                                   a.partial, in, out, a.dmask, a.red, a.k, a.gctl, a.part_group, a.part_valid);
      if (publish(&ps->applied, cnt) + cnt == a.n_apply)
        finalize_body(a.ctl, a.gctl, a.group_slots, a.red, a.k, a.k + a.n_mg, a.hist);
    }
    if (!grid_sync(ps, a.spin_limit, reset)) return;
    if (ld_acquire(&a.ctl->done)) return;
  }
}

// ---- SpMV (Sec. 3.5) -----------------------------------------------------------------
// Split bins of an SpMV: y = the sum of the item slices, in slot order.
__global__ __launch_bounds__(kMergeNodes) void k_spmv_merge(const Ctl* __restrict__ ctl, int64_t n, int s,
                                                           const Merge* __restrict__ mg,
                                                           const int64_t* __restrict__ partial, float* __restrict__ y) {
  const Merge mu = mg[blockIdx.x];
  const int64_t q = int64_t{1} << s;
  const int64_t v0 = static_cast<int64_t>(mu.part) << s;
  const int qn = static_cast<int>(min(q, n - v0));
  const int i = mu.node_lo + static_cast<int>(threadIdx.x);
  if (i >= qn) return;
  const int64_t* base = partial + static_cast<int64_t>(mu.first) * q;
  const int64_t sum = sum_slices(base + i, mu.count, q);
  __builtin_nontemporal_store(
      ctl->nonfinite ? __builtin_nanf("") : static_cast<float>(static_cast<double>(sum) * ldexp(1.0, -ctl->fx_shift)),
      y + v0 + i);
}

// Largest |x| per workgroup (+inf if x holds a non-finite value).
__global__ __launch_bounds__(256) void k_spmv_absmax(const float* __restrict__ x, int64_t n,
                                                      float* __restrict__ blockmax) {
  float m = 0.0f;
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; v < n;
       v += static_cast<int64_t>(gridDim.x) * 256) {
    const float a = fabsf(x[v]);
    m = fmaxf(m, isfinite(a) ? a : __builtin_inff());
  }
  const double bm = block_max<256>(static_cast<double>(m));
  if (threadIdx.x == 0) blockmax[blockIdx.x] = static_cast<float>(bm);
}

// Fixed-point scale of one SpMV: every product w*x(u) is at most
// wabs * max|x| (kept below 2^50 units) and every sum, partial or whole, at
// most wcol * max|x| (kept below 2^62 units).
__global__ __launch_bounds__(1024) void k_spmv_scale(Ctl* __restrict__ ctl, const float* __restrict__ blockmax,
                                                      int nb, const unsigned long long* __restrict__ wstats) {
  const double wcol = __longlong_as_double(static_cast<long long>(wstats[0]));
  const double wabs = __longlong_as_double(static_cast<long long>(wstats[1]));
  double m = 0.0;
  for (int b = threadIdx.x; b < nb; b += 1024) m = fmax(m, static_cast<double>(blockmax[b]));
  m = block_max<1024>(m);
  if (threadIdx.x == 0) {
    int sh = 0;
    const bool bad = !isfinite(m);
    if (!bad && m > 0.0 && wabs > 0.0 && wcol > 0.0) {
      const int e1 = static_cast<int>(ceil(log2(wabs * m)));
      const int e2 = static_cast<int>(ceil(log2(wcol * m)));
      sh = min(50 - e1, 62 - e2);
    }
    ctl->done = 0;
    ctl->nonfinite = bad ? 1 : 0;
    ctl->fx_shift = sh;
  }
}

// ---- start of a solve ----------------------------------------------------------------

// Start vector statistics per partition: non-finite count, dangling mass and
// L1 mass, into the partition's start slot, and its largest |value| (after
// the 3k slots).  Padding entries are cleared.  fill: the start vector is
// written here, 1/n_g on every real node of group g, instead of read.
// One workgroup per partition.
__global__ __launch_bounds__(256) void k_start_parts(float* __restrict__ x, const uint32_t* __restrict__ dmask,
                                                     int64_t n, int s, const int32_t* __restrict__ part_valid,
                                                     double* __restrict__ red, bool fill,
                                                     const GCtl* __restrict__ gctl,
                                                     const int32_t* __restrict__ part_group) {
  const int64_t v0 = static_cast<int64_t>(blockIdx.x) << s;
  const int qn = static_cast<int>(min(int64_t{1} << s, n - v0));
  const int valid = part_valid[blockIdx.x];
  const float u = fill ? static_cast<float>(gctl[part_group[blockIdx.x]].inv_n) : 0.0f;
  double sums[3] = {0.0, 0.0, 0.0};
  float mx = 0.0f;
  for (int i = threadIdx.x; i < qn; i += 256) {
    const int64_t v = v0 + i;
    if (i >= valid) {
      x[v] = 0.0f;
      continue;
    }
    float xv;
    if (fill) {
      xv = u;
      x[v] = u;
    } else {
      xv = x[v];
    }
    if (!isfinite(xv)) sums[0] += 1.0;
    if ((dmask[v >> 5] >> (v & 31)) & 1u) sums[1] += static_cast<double>(xv);
    sums[2] += fabs(static_cast<double>(xv));
    mx = fmaxf(mx, fabsf(xv));
  }
  block_sum<256>(sums);
  const double vmax = block_max<256>(static_cast<double>(mx));
  if (threadIdx.x == 0) {
    red[3 * blockIdx.x] = sums[0];
    red[3 * blockIdx.x + 1] = sums[1];
    red[3 * blockIdx.x + 2] = sums[2];
    red[3 * gridDim.x + blockIdx.x] = vmax;
  }
}

// Per-group dangling mass and base of the start vector, and the fixed-point
// scale of the first gather: every gather sum is bounded by max(1, L1 mass of
// the start vector), which later iterates never exceed (teleport vectors are
// non-negative and sum to one per group), which caps the scale at
// 61 - ceil(log2(that bound)); within the cap, the start vector's largest
// value sets it.
__global__ __launch_bounds__(1024) void k_start_finalize(Ctl* __restrict__ ctl, GCtl* __restrict__ gctl,
                                                         const int32_t* __restrict__ group_slots,
                                                         const double* __restrict__ red, int64_t k, int G,
                                                         double tol, double d) {
  double vmax = 0.0;  // largest |value| of the start vector
  for (int64_t j = threadIdx.x; j < k; j += 1024) vmax = fmax(vmax, red[3 * k + j]);
  vmax = block_max<1024>(vmax);
  __shared__ int bad;
  __shared__ double mass_w[1024 / kWave];
  if (threadIdx.x == 0) bad = 0;
  if (threadIdx.x < 1024 / kWave) mass_w[threadIdx.x] = 0.0;
  __syncthreads();
  double wmass = 0.0;
  // each group's control struct is set by one thread: the one that sums it
  for (int grp = threadIdx.x / kWave; grp < G; grp += 1024 / kWave) {
    double sm[3];
    group_sums(group_slots, red, k, grp, false, sm);
    if ((threadIdx.x & (kWave - 1)) == 0) {
      GCtl& gc = gctl[grp];
      gc.res = 0.0;
      gc.iter = 0;
      gc.done = 0;
      gc.dmass = sm[1];
      gc.base = (1.0 - d) * gc.inv_n + d * sm[1] * gc.inv_n;
      if (sm[0] > 0.0 || !isfinite(sm[1]) || !isfinite(sm[2])) atomicOr(&bad, 1);
      wmass += sm[2];
    }
  }
  if ((threadIdx.x & (kWave - 1)) == 0) mass_w[threadIdx.x / kWave] = wmass;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mass = 0.0;
    for (int w = 0; w < 1024 / kWave; ++w) mass += mass_w[w];
    int e = 0;
    if (isfinite(mass) && mass > 1.0) e = static_cast<int>(ceil(log2(mass)));
    ctl->res = 0.0;
    ctl->res_prev = 0.0;
    ctl->tol = tol;
    ctl->d = d;
    ctl->iter = 0;
    ctl->ngroups = G;
    ctl->fx_cap = 61 - min(e, 1000);
    ctl->fx_shift = fx_shift_for(vmax, ctl->fx_cap);
    ctl->nonfinite = bad ? 1 : 0;
    ctl->done = bad ? 1 : 0;
  }
}

// NaN everywhere in x when the solve met a non-finite value (the kernels of
// an iteration return at once then, leaving x unwritten).
__global__ __launch_bounds__(256) void k_nan_if_nonfinite(const Ctl* __restrict__ ctl, float* __restrict__ x,
                                                          int64_t n) {
  if (!ctl->nonfinite) return;
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; v < n;
       v += static_cast<int64_t>(gridDim.x) * 256)
    x[v] = __builtin_nanf("");
}

template <bool kPng>
static pcpm_status_t iter_lds_limits_for() {
  const void* scat[] = {reinterpret_cast<const void*>(k_scatter<kScatterBlock, true, kPng>),
                        reinterpret_cast<const void*>(k_scatter<kScatterBlock, false, kPng>)};
  const void* gath[] = {reinterpret_cast<const void*>(k_gather<kGatherBlock, 0, kPng>),
                        reinterpret_cast<const void*>(k_gather<kGatherBlock, 1, kPng>),
                        reinterpret_cast<const void*>(k_gather<kGatherBlock, 2, kPng>)};
  for (const void* f : scat)
    PCPM_TRY_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (2 << kMaxLog2) * 4));
  for (const void* f : gath)
    PCPM_TRY_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (1 << kMaxLog2) * 8));
  PCPM_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_persist<kPng>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (1 << kMaxLog2) * 8));
  return PCPM_OK;
}

pcpm_status_t iter_lds_limits() {
  static bool done = false;
  if (done) return PCPM_OK;
  PCPM_TRY(iter_lds_limits_for<false>());
  PCPM_TRY(iter_lds_limits_for<true>());
  done = true;
  return PCPM_OK;
}

// Start of a solve: the control block reset for damping d and tolerance tol,
// and the start vector's statistics.  fill: x0 receives the uniform start
// vector (1/n_g per group) instead of holding the caller's.
static pcpm_status_t start_solve(pcpm_png* g, float* x0, bool fill, double tol, double d, hipStream_t st) {
  const unsigned kk = static_cast<unsigned>(g->k);
  PCPM_LAUNCH("pcpm_init", k_start_parts, dim3(kk), dim3(256), 0, st, x0, g->dmask, g->n, g->part_log2,
              g->part_valid, g->red_start, fill, g->gctl, g->part_group);
  PCPM_LAUNCH("pcpm_init", k_start_finalize, dim3(1), dim3(1024), 0, st, g->ctl, g->gctl, g->group_slots,
              g->red_start, g->k, static_cast<int>(g->ngroups), tol, d);
  return PCPM_OK;
}

// Scatter and gather of one pass in the handle's update order; kScale and
// kMode as in k_scatter / k_gather.
// The scatter stages the rows' values (n_rows of them), the gather writes
// the columns' (n_cols): both n for a graph.
template <bool kScale, int kMode, bool kPng>
static pcpm_status_t scatter_gather(pcpm_png* g, const float* in, float* out, const char* sname, const char* gname,
                                    hipStream_t st) {
  if (g->n_sc)
    PCPM_LAUNCH(sname, (k_scatter<kScatterBlock, kScale, kPng>), dim3(static_cast<unsigned>(g->n_sc)),
                dim3(kScatterBlock), static_cast<size_t>(g->q) * 8, st, g->ctl, g->n_rows, g->part_log2, g->sc_items,
                in, g->outdeg, g->png_src, g->png_blk, g->seg_delta, g->upd, g->eprime);
  PCPM_LAUNCH(gname, (k_gather<kGatherBlock, kMode, kPng>), dim3(static_cast<unsigned>(g->n_ga)), dim3(kGatherBlock),
              static_cast<size_t>(g->q) * 8, st, g->ctl, g->n_cols, g->part_log2, g->ga_items, g->did, g->did_blk,
              g->did_sblk, g->seg_delta, g->upd, in, out, g->dmask, g->partial, g->red, g->gctl, g->part_group,
              g->part_valid, g->wbin);
  return PCPM_OK;
}

template <bool kScale, int kMode>
static pcpm_status_t scatter_gather(pcpm_png* g, const float* in, float* out, const char* sname, const char* gname,
                                    hipStream_t st) {
  return g->png_order ? scatter_gather<kScale, kMode, true>(g, in, out, sname, gname, st)
                      : scatter_gather<kScale, kMode, false>(g, in, out, sname, gname, st);
}

static pcpm_status_t run_iteration(pcpm_png* g, const float* in, float* out, hipStream_t st) {
  PCPM_TRY((scatter_gather<true, 0>(g, in, out, "pcpm_scatter", "pcpm_gather", st)));
  if (g->n_mg)
    PCPM_LAUNCH("pcpm_merge", k_merge<kMergeNodes>, dim3(static_cast<unsigned>(g->n_mg)), dim3(kMergeNodes), 0,
                st, g->ctl, g->n, g->part_log2, g->mg_items, g->partial, in, out, g->dmask, g->red, g->k, g->gctl,
                g->part_group, g->part_valid);
  PCPM_LAUNCH("pcpm_finalize", k_finalize, dim3(1), dim3(1024), 0, st, g->ctl, g->gctl, g->group_slots, g->red,
              g->k, g->k + g->n_mg, g->hist);
  return PCPM_OK;
}

// Workgroups of the persistent solve: as many as can be resident at once
// (one per CU at a 128 KB slice), or 0 if the device cannot launch
// cooperatively.
static pcpm_status_t persist_grid(pcpm_png* g) {
  if (g->persist_grid >= 0) return PCPM_OK;
  PCPM_TRY(iter_lds_limits());
  int cus = 0, coop = 0, per = 0;
  PCPM_TRY_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, g->device));
  PCPM_TRY_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, g->device));
  const void* f = g->png_order ? reinterpret_cast<const void*>(k_persist<true>)
                               : reinterpret_cast<const void*>(k_persist<false>);
  PCPM_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, 1024, static_cast<size_t>(g->q) * 8));
  // every XCD's scatter range needs workgroups of its own (b % 8 for b < grid)
  g->persist_grid = (coop && per * cus >= static_cast<int>(kXcds)) ? per * cus : 0;
  return PCPM_OK;
}

// Mode 0 takes one launch per phase: on MI355X back-to-back launches queue
// with gaps of a few microseconds, while the persistent solve pays for its
// grid barriers and per-unit handoffs (measured slower on every workload).
static bool use_persistent(const pcpm_png* g) { return g->persist_grid > 0 && g->launch_mode == 2; }

// All iterations of a solve in one cooperative launch (a = pr_out holds the
// start vector, b = tmp_pr).
static pcpm_status_t run_persistent(pcpm_png* g, float* a, float* b, int32_t max_iters, hipStream_t st) {
  PCPM_LAUNCH("pcpm_init", k_persist_init, dim3(1), dim3(256), 0, st, g->psync, g->bin_done, g->k);
  PersistArgs pa;
  pa.ctl = g->ctl;
  pa.gctl = g->gctl;
  pa.ps = g->psync;
  pa.bin_done = g->bin_done;
  pa.n = g->n;
  pa.k = g->k;
  pa.s = g->part_log2;
  pa.n_sc = g->n_sc;
  pa.n_ga = g->n_ga;
  pa.n_mg = g->n_mg;
  pa.n_apply = static_cast<int32_t>(g->k - g->n_split_bins) + g->n_mg;
  pa.max_iters = max_iters;
  pa.spin_limit = g->spin_limit;
  pa.sc_items = g->sc_items;
  pa.ga_items = g->ga_items;
  pa.mg_items = g->mg_items;
  pa.outdeg = g->outdeg;
  pa.png_src = g->png_src;
  pa.png_blk = g->png_blk;
  pa.seg_delta = g->seg_delta;
  pa.upd = g->upd;
  pa.spare = g->eprime;
  pa.did = g->did;
  pa.did_blk = g->did_blk;
  pa.did_sblk = g->did_sblk;
  pa.dmask = g->dmask;
  pa.partial = g->partial;
  pa.red = g->red;
  pa.part_group = g->part_group;
  pa.part_valid = g->part_valid;
  pa.group_slots = g->group_slots;
  pa.hist = g->hist;
  pa.x0 = a;
  pa.x1 = b;
  void* args[] = {&pa};
  const void* f = g->png_order ? reinterpret_cast<const void*>(k_persist<true>)
                               : reinterpret_cast<const void*>(k_persist<false>);
  {
    TimerScope ts("pcpm_persist", st);
    PCPM_TRY_HIP(hipLaunchCooperativeKernel(f, dim3(static_cast<unsigned>(g->persist_grid)), dim3(1024), args,
                                            static_cast<unsigned>(g->q * 8), st));
  }
  PCPM_TRY_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipMemcpyAsync(g->psync_host, g->psync, sizeof(PSync), hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  if (g->psync_host->err)
    return set_error(PCPM_ERR_DEVICE, "a device-side wait of the persistent solve ran past its limit of %u polls",
                     g->spin_limit);
  return PCPM_OK;
}

// The PageRank calls take graphs, not matrix handles.
static pcpm_status_t check_graph(const pcpm_png* g) {
  if (g->matrix)
    return set_error(PCPM_ERR_INVALID_ARG, "the handle holds a matrix (num_cols or allow_diagonal): pcpm_spmv only");
  return PCPM_OK;
}

static pcpm_status_t check_device(pcpm_png* g) {
  int dev = -1;
  PCPM_TRY_HIP(hipGetDevice(&dev));
  if (dev != g->device)
    return set_error(PCPM_ERR_INVALID_ARG, "handle lives on device %d but device %d is current", g->device, dev);
  return PCPM_OK;
}

// End of a solve with final control block c: results to the caller, the
// last iterate into a.
static pcpm_status_t finish_solve(pcpm_png* g, const Ctl& c, float* a, const float* b, double tol, int32_t* iters,
                                  double* resid, double* res_hist, hipStream_t st) {
  *iters = c.iter;
  *resid = c.res;
  if (c.iter > 0 && ((c.iter - 1) % 2) == 0)  // last output went to b
    PCPM_TRY_HIP(hipMemcpyAsync(a, b, static_cast<size_t>(g->n) * 4, hipMemcpyDeviceToDevice, st));
  if (res_hist && c.iter > 0)
    PCPM_TRY_HIP(hipMemcpyAsync(res_hist, g->hist, static_cast<size_t>(c.iter) * 8, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  if (c.nonfinite) return set_error(PCPM_ERR_NUMERIC, "non-finite rank, residual or dangling mass");
  if (tol > 0.0 && !c.done)
    return set_error(PCPM_ERR_NOT_CONVERGED, "residual %.3e still above tol %.3e after %d iterations", c.res, tol,
                     c.iter);
  return PCPM_OK;
}

}  // namespace pcpm

extern "C" {

pcpm_status_t pcpm_set_launch(pcpm_png_t g, int32_t mode, uint32_t spin_limit) {
  using namespace pcpm;
  if (!g) return set_error(PCPM_ERR_INVALID_ARG, "NULL handle");
  PCPM_TRY(check_graph(g));
  if (mode < 0 || mode > 2) return set_error(PCPM_ERR_INVALID_ARG, "launch mode %d is not 0, 1 or 2", mode);
  PCPM_TRY(check_device(g));
  PCPM_TRY(persist_grid(g));
  if (mode == 2 && g->persist_grid <= 0)
    return set_error(PCPM_ERR_INVALID_ARG, "the device cannot run the persistent solve (no cooperative launch)");
  g->launch_mode = mode;
  g->spin_limit = spin_limit ? spin_limit : (1u << 22);
  return PCPM_OK;
}

int32_t pcpm_launch_grid(pcpm_png_t g) {
  if (!g || pcpm::persist_grid(g) != PCPM_OK) return 0;
  return g->persist_grid;
}

pcpm_status_t pcpm_iterate(pcpm_png_t g, double d, const float* pr_in, float* pr_out, double* resid, void* stream) {
  using namespace pcpm;
  if (!g || !pr_in || !pr_out) return set_error(PCPM_ERR_INVALID_ARG, "NULL handle or vector");
  if (!(d >= 0.0 && d < 1.0)) return set_error(PCPM_ERR_INVALID_ARG, "d must lie in [0, 1)");
  if (pr_in == pr_out) return set_error(PCPM_ERR_INVALID_ARG, "pr_in and pr_out must differ");
  PCPM_TRY(check_graph(g));
  PCPM_TRY(check_device(g));
  hipStream_t st = static_cast<hipStream_t>(stream);
  // the start statistics clear padding entries, so they run on a copy
  PCPM_TRY_HIP(hipMemcpyAsync(g->tmp_pr, pr_in, static_cast<size_t>(g->n) * 4, hipMemcpyDeviceToDevice, st));
  PCPM_TRY(start_solve(g, g->tmp_pr, false, 0.0, d, st));
  PCPM_TRY(run_iteration(g, g->tmp_pr, pr_out, st));
  if (!resid) {
    const unsigned nb = static_cast<unsigned>(std::min<int64_t>((g->n + 255) / 256, 1024));
    PCPM_LAUNCH("pcpm_init", k_nan_if_nonfinite, dim3(nb), dim3(256), 0, st, g->ctl, pr_out, g->n);
  } else {
    PCPM_TRY_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    PCPM_TRY_HIP(hipStreamSynchronize(st));
    *resid = g->ctl_host->res;
    if (g->ctl_host->nonfinite) return set_error(PCPM_ERR_NUMERIC, "non-finite rank, residual or dangling mass");
  }
  return PCPM_OK;
}

pcpm_status_t pcpm_spmv(pcpm_png_t g, const float* x, float* y, void* stream) {
  using namespace pcpm;
  if (!g || !x || !y) return set_error(PCPM_ERR_INVALID_ARG, "NULL handle or vector");
  {
    const uintptr_t xa = reinterpret_cast<uintptr_t>(x), ya = reinterpret_cast<uintptr_t>(y);
    const uintptr_t xbytes = static_cast<uintptr_t>(g->n_rows) * sizeof(float);
    const uintptr_t ybytes = static_cast<uintptr_t>(g->n_cols) * sizeof(float);
    if (xa < ya + ybytes && ya < xa + xbytes) return set_error(PCPM_ERR_INVALID_ARG, "x and y must not overlap");
  }
  PCPM_TRY(check_device(g));
  hipStream_t st = static_cast<hipStream_t>(stream);
  constexpr int kMaxBlocks = 1024;
  if (!g->spmv_blockmax) PCPM_TRY(dalloc(g, &g->spmv_blockmax, kMaxBlocks));
  const int nb = static_cast<int>(std::min<int64_t>((g->n_rows + 255) / 256, kMaxBlocks));
  PCPM_LAUNCH("pcpm_spmv_scale", k_spmv_absmax, dim3(nb), dim3(256), 0, st, x, g->n_rows, g->spmv_blockmax);
  if (!g->wstats_ready) PCPM_TRY(weight_stats(g, st));  // unweighted handle, first call
  PCPM_LAUNCH("pcpm_spmv_scale", k_spmv_scale, dim3(1), dim3(1024), 0, st, g->ctl, g->spmv_blockmax, nb, g->wstats);
  if (g->wbin)
    PCPM_TRY((scatter_gather<false, 2>(g, x, y, "pcpm_spmv_scatter", "pcpm_spmv_gather", st)));
  else
    PCPM_TRY((scatter_gather<false, 1>(g, x, y, "pcpm_spmv_scatter", "pcpm_spmv_gather", st)));
  if (g->n_mg)
    PCPM_LAUNCH("pcpm_spmv_merge", k_spmv_merge, dim3(static_cast<unsigned>(g->n_mg)), dim3(kMergeNodes), 0, st,
                g->ctl, g->n_cols, g->part_log2, g->mg_items, g->partial, y);
  return PCPM_OK;
}

pcpm_status_t pcpm_pagerank(pcpm_png_t g, double d, double tol, int32_t max_iters, const float* init,
                            float* pr_out, int32_t* iters, double* resid, double* res_hist, void* stream) {
  using namespace pcpm;
  if (!g || !pr_out || !iters || !resid) return set_error(PCPM_ERR_INVALID_ARG, "NULL handle or output");
  if (!(d >= 0.0 && d < 1.0)) return set_error(PCPM_ERR_INVALID_ARG, "d must lie in [0, 1)");
  if (max_iters < 1 || max_iters > kMaxHist)
    return set_error(PCPM_ERR_INVALID_ARG, "max_iters must lie in [1, %d]", kMaxHist);
  if (!(tol == tol)) return set_error(PCPM_ERR_INVALID_ARG, "tol is NaN");
  PCPM_TRY(check_graph(g));
  PCPM_TRY(check_device(g));
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* a = pr_out;
  float* b = g->tmp_pr;
  if (init && init != pr_out)
    PCPM_TRY_HIP(hipMemcpyAsync(a, init, static_cast<size_t>(g->n) * 4, hipMemcpyDeviceToDevice, st));
  PCPM_TRY(start_solve(g, a, !init, tol, d, st));
  PCPM_TRY(persist_grid(g));
  if (use_persistent(g)) {
    PCPM_TRY(run_persistent(g, a, b, max_iters, st));
    return finish_solve(g, g->ctl_host[0], a, b, tol, iters, resid, res_hist, st);
  }
  Ctl c{};
  PCPM_TRY(pipelined_iterations(
      g, tol, max_iters, st,
      [&](int64_t it) { return (it % 2) == 0 ? run_iteration(g, a, b, st) : run_iteration(g, b, a, st); }, &c));
  return finish_solve(g, c, a, b, tol, iters, resid, res_hist, st);
}

pcpm_status_t pcpm_graph_results(pcpm_png_t g, int32_t* iters, double* resid) {
  using namespace pcpm;
  if (!g) return set_error(PCPM_ERR_INVALID_ARG, "NULL handle");
  PCPM_TRY_HIP(hipMemcpy(g->gctl_host, g->gctl, sizeof(GCtl) * g->ngroups, hipMemcpyDeviceToHost));
  for (int grp = 0; grp < g->ngroups; ++grp) {
    if (iters) iters[grp] = g->gctl_host[grp].iter;
    if (resid) resid[grp] = g->gctl_host[grp].res;
  }
  return PCPM_OK;
}

}  // extern "C"
