// Partition-Node Graph construction (Sec. 3.1 write offsets, Sec. 3.3 merged
// compression + transposition) on the GPU.
//
// Pipeline (all on the caller's stream):
//   node pass    validate rows, out-degrees, dangling bitmask, edge -> source
//                (node-parallel: the row of each tile's first edge; then
//                edge-parallel tiles with row marks in LDS)
//   count        per source partition p (one workgroup, LDS histograms):
//                |U(p,p')| and raw edges p -> p' for every p'
//   scans        write offsets (column prefix over source partitions),
//                partition-local PNG offsets (row prefix), bin starts
//   fill         per chunk of a source partition's edges, one wavefront walks
//                them in CSR order; a ballot multisplit ranks each edge among
//                the edges of the same destination partition, so every bin is
//                written in the canonical (p, u, v) order without atomics and
//                the PNG in (p, p', u) order; records go first to at most 64
//                buckets of destination partitions, then to their slots
//   tile flags   flags before every 1024-entry tile of both arrays
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pcpm_device.hpp"
#include "pcpm_internal.hpp"

namespace pcpm {

enum : int32_t {
  kErrOffsets = 1,   // row_off entries out of [0,m] or decreasing
  kErrRange = 2,     // column outside [0,n)
  kErrSelfLoop = 4,
  kErrOrder = 8,     // row not strictly ascending (unsorted or duplicate)
  kErrEnds = 16,     // row_off[0] != 0 or row_off[n] != m
  kErrInternal = 32,
  kErrGraphs = 64,   // an edge leaves its graph, or a padding node has edges
};

// Node pass, in two kernels.  Nodes (one lane per node, coalesced):
// out-degree, dangling bit, offset checks, and for every 1024-edge tile the
// row holding its first edge (tile_row[t]; only rows that contain a tile
// start write, about one per tile).  Edges (one wavefront per tile): the
// rows from tile_row[t] to tile_row[t + 1] put a mark at their first edge in
// LDS, a wavefront max-scan over the marks gives every edge its source, then
// the edge checks.
// Edge u -> c stays inside u's graph and avoids padding nodes.
__device__ __forceinline__ bool same_graph(int64_t u, int32_t c, int s, const int32_t* __restrict__ part_group,
                                           const int32_t* __restrict__ part_valid) {
  const int32_t pc = c >> s;
  const int32_t mask = (1 << s) - 1;
  return part_group[pc] == part_group[u >> s] && (c & mask) < part_valid[pc];
}

__global__ __launch_bounds__(256) void k_node_pass(int64_t n, int64_t m, const int32_t* __restrict__ row_off,
                                                   int32_t* __restrict__ outdeg, uint32_t* __restrict__ dmask,
                                                   int32_t* __restrict__ tile_row,
                                                   int32_t* __restrict__ counters /* [0]=err [2]=ndang */, int s,
                                                   const int32_t* __restrict__ part_valid) {
  __shared__ int32_t wdang[256 / kWave];
  const int64_t nwords = (n + 31) >> 5;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int32_t ndang = 0;  // dangling nodes seen by this wavefront (lane 0)
  for (int64_t base = static_cast<int64_t>(blockIdx.x) * blockDim.x; base < n; base += stride) {
    const int64_t u = base + threadIdx.x;
    bool dang = false;
    int32_t err = 0;
    if (u < n) {
      const int32_t lo = row_off[u], hi = row_off[u + 1];
      if (lo < 0 || hi < lo || static_cast<int64_t>(hi) > m) {
        err |= kErrOffsets;
        outdeg[u] = 0;
      } else {
        outdeg[u] = hi - lo;
        dang = (hi == lo);
        if (hi > lo && (u & ((int64_t{1} << s) - 1)) >= part_valid[u >> s]) err |= kErrGraphs;
        // tiles whose first edge lies in [lo, hi): all below ceil(m / kTile)
        for (int64_t t = (static_cast<int64_t>(lo) + kTile - 1) / kTile; t * kTile < hi; ++t)
          tile_row[t] = static_cast<int32_t>(u);
      }
      if (u == n - 1) tile_row[(m + kTile - 1) / kTile] = static_cast<int32_t>(u);  // end of the last tile's rows
    }
    if (err) atomicOr(&counters[0], err);
    const uint64_t bal = wave_ballot(dang);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t first = base + (threadIdx.x & ~(kWave - 1));
    if (lane == 0 && first < n) {
      const int64_t w = first >> 5;
      dmask[w] = static_cast<uint32_t>(bal);
      if (w + 1 < nwords) dmask[w + 1] = static_cast<uint32_t>(bal >> 32);
      ndang += __popcll(bal);
    }
  }
  // one atomic per workgroup (one per wavefront on a single counter serialised the pass)
  if ((threadIdx.x & (kWave - 1)) == 0) wdang[threadIdx.x / kWave] = ndang;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t b = 0;
    for (int i = 0; i < static_cast<int>(blockDim.x) / kWave; ++i) b += wdang[i];
    if (b) atomicAdd(&counters[2], b);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (row_off[0] != 0 || static_cast<int64_t>(row_off[n]) != m) atomicOr(&counters[0], kErrEnds);
  }
}

// With valid offsets (non-decreasing in [0, m], which the node pass checked
// on the same stream; otherwise this kernel returns at once) the rows of
// tile t are tile_row[t] .. tile_row[t + 1]: the first holds the tile's first
// edge, the others start inside the tile or at its end.  A row's mark is
// kept with an LDS max, so among empty rows that share an offset the
// non-empty row after them wins.  Rows visited over all tiles: n + ntiles.
constexpr int kEdgeBlock = 256;
// ncols: columns must lie in [0, ncols); self_loops: 1 rejects u -> u.
__global__ __launch_bounds__(kEdgeBlock) void k_edge_pass(int64_t ncols, int self_loops, int64_t m,
                                                          const int32_t* __restrict__ row_off,
                                                          const int32_t* __restrict__ col, int32_t* __restrict__ src,
                                                          const int32_t* __restrict__ tile_row,
                                                          int32_t* __restrict__ counters, int s,
                                                          const int32_t* __restrict__ part_group,
                                                          const int32_t* __restrict__ part_valid) {
  __shared__ int32_t marks[kEdgeBlock / kWave][kTile];
  if (counters[0] != 0) return;  // invalid offsets: the build fails, src is not used
  const int lane = threadIdx.x & (kWave - 1);
  int32_t* mk_l = marks[threadIdx.x / kWave];
  const int64_t ntiles = (m + kTile - 1) / kTile;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  int32_t err = 0;
  for (int64_t t = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave; t < ntiles; t += nwaves) {
    const int64_t e0 = t * kTile, e_end = min(m, e0 + kTile);
    const int32_t r0 = tile_row[t], r1 = tile_row[t + 1];
    const int64_t lo0 = row_off[r0];  // the first row's start: at or before e0
    for (int j = 0; j < kSub; ++j) mk_l[j * kWave + lane] = -1;
    __builtin_amdgcn_wave_barrier();
    for (int64_t u = static_cast<int64_t>(r0) + 1 + lane; u <= r1; u += kWave) {
      const int64_t lo = row_off[u];
      if (lo >= e0 && lo < e_end) atomicMax(&mk_l[lo - e0], static_cast<int32_t>(u));
    }
    __builtin_amdgcn_wave_barrier();
    int32_t carry = r0;
    for (int j = 0; j < kSub; ++j) {
      const int64_t e = e0 + j * kWave + lane;
      const bool in = e < m;
      const int32_t mk = mk_l[j * kWave + lane];
      int32_t v = mk;  // inclusive max-scan over the wavefront
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const int32_t o = __shfl_up(v, off);
        if (lane >= off) v = max(v, o);
      }
      const int32_t u = max(v, carry);
      carry = __shfl(u, kWave - 1);
      if (in) {
        src[e] = u;
        const int32_t c = col[e];
        // first edge of its row (a mark, or the tile's first row starting here): no predecessor
        const bool row_start = mk >= 0 || e == lo0;
        const int32_t prev = row_start ? -1 : col[e - 1];
        if (c < 0 || static_cast<int64_t>(c) >= ncols) err |= kErrRange;
        else if (!same_graph(u, c, s, part_group, part_valid)) err |= kErrGraphs;
        if (self_loops && c == u) err |= kErrSelfLoop;
        if (c <= prev) err |= kErrOrder;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  if (err) atomicOr(&counters[0], err);
}

// ---------------------------------------------------------------------------------
// The count and fill passes work on chunks of one source partition's edges
// (CSR order), so that a partition with many edges (hubs under in-degree
// labels) is spread over many workgroups.  For chunk c of partition p,
// ccnt[c][p'] / craw[c][p'] count its first-of-message edges (the PNG edges
// it contributes to U(p,p')) and all its edges into p'.

// Partition edge bounds: pe[p] = row_off[min(n, p q)], p = 0..k.
__global__ __launch_bounds__(256) void k_part_edges(int64_t n, int s, int32_t k, const int32_t* __restrict__ row_off,
                                                    int32_t* __restrict__ pe) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p <= k) pe[p] = row_off[min(n, p << s)];
}

// Count: workgroup c histograms the destination partitions of chunk c's
// edges.  An edge is the first of its message when it starts its row or its
// destination partition differs from the previous edge's (rows are sorted).
__global__ __launch_bounds__(1024) void k_count(int s, int32_t k, const Item* __restrict__ chunks,
                                                const int32_t* __restrict__ col, const int32_t* __restrict__ src,
                                                int32_t* __restrict__ ccnt, int32_t* __restrict__ craw) {
  extern __shared__ int32_t sh[];
  int32_t* c_l = sh;
  int32_t* r_l = sh + k;
  for (int32_t i = threadIdx.x; i < 2 * k; i += blockDim.x) sh[i] = 0;
  __syncthreads();
  const int64_t c = blockIdx.x;
  const Item ch = chunks[c];
  for (int32_t e = ch.lo + static_cast<int32_t>(threadIdx.x); e < ch.hi; e += blockDim.x) {
    const int32_t u = src[e];
    const int32_t pp = col[e] >> s;
    const bool first = (e == 0) || (src[e - 1] != u) || ((col[e - 1] >> s) != pp);
    atomicAdd(&r_l[pp], 1);
    if (first) atomicAdd(&c_l[pp], 1);
  }
  __syncthreads();
  for (int32_t i = threadIdx.x; i < k; i += blockDim.x) {
    ccnt[c * k + i] = c_l[i];
    craw[c * k + i] = r_l[i];
  }
}

// Per partition p and destination p': exclusive prefix of the chunk counts
// over p's chunks (in place: each chunk's starting rank and position inside
// the (p, p') segment and its run of the bin) and the totals cnt/raw[p][p'].
__global__ __launch_bounds__(256) void k_chunk_scan(int32_t k, const int32_t* __restrict__ cfirst,
                                                    int32_t* __restrict__ ccnt, int32_t* __restrict__ craw,
                                                    int32_t* __restrict__ cnt, int32_t* __restrict__ raw) {
  const int64_t p = blockIdx.x;
  const int32_t j = static_cast<int32_t>(blockIdx.y * blockDim.x + threadIdx.x);
  if (j >= k) return;
  int32_t sc = 0, sr = 0;
  for (int64_t c = cfirst[p]; c < cfirst[p + 1]; ++c) {
    const int64_t idx = c * k + j;
    const int32_t a = ccnt[idx], b = craw[idx];
    ccnt[idx] = sc;
    craw[idx] = sr;
    sc += a;
    sr += b;
  }
  cnt[p * k + j] = sc;
  raw[p * k + j] = sr;
}

// Column prefix over source partitions: write offsets wo[p][p'] (updates) and
// dwo[p][p'] (destination IDs); column totals.  One lane per column p'.
__global__ __launch_bounds__(256) void k_colscan(int32_t k, const int32_t* __restrict__ cnt,
                                                 const int32_t* __restrict__ raw, int32_t* __restrict__ wo,
                                                 int32_t* __restrict__ dwo, int32_t* __restrict__ coltot,
                                                 int32_t* __restrict__ coltot_raw) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  int32_t s = 0, sr = 0;
  for (int64_t p = 0; p < k; ++p) {
    const int64_t idx = p * k + j;
    const int32_t c = cnt[idx], r = raw[idx];
    wo[idx] = s;
    dwo[idx] = sr;
    s += c;
    sr += r;
  }
  coltot[j] = s;
  coltot_raw[j] = sr;
}

// Block-wide exclusive scan of one value per thread (blockDim <= 1024).
__device__ int64_t block_excl_scan(int64_t v, int64_t* total) {
  __shared__ int64_t sh[1024];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < static_cast<int>(blockDim.x); off <<= 1) {
    int64_t t = (threadIdx.x >= static_cast<unsigned>(off)) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  const int64_t incl = sh[threadIdx.x];
  *total = sh[blockDim.x - 1];
  __syncthreads();
  return incl - v;
}

// Exclusive scan of long arrays (the tile flag counts) in three launches:
// every workgroup sums kScanSpan values, one workgroup scans the sums
// (k_scan_excl), every workgroup scans its values from its offset, 1024 at a
// time with coalesced loads.  out[L] = total.
constexpr int kScanSpan = 8192;
__global__ __launch_bounds__(1024) void k_scan_sums(const int32_t* __restrict__ in, int64_t L,
                                                    int32_t* __restrict__ bsum) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanSpan + threadIdx.x;
  int64_t sum = 0;
  for (int j = 0; j < kScanSpan / 1024; ++j) {
    const int64_t i = base + j * 1024;
    if (i < L) sum += in[i];
  }
  int64_t tot = 0;
  (void)block_excl_scan(sum, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = static_cast<int32_t>(tot);
}

__global__ __launch_bounds__(1024) void k_scan_apply(const int32_t* __restrict__ in, int64_t L,
                                                     const int32_t* __restrict__ boff, int32_t* __restrict__ out) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanSpan + threadIdx.x;
  int64_t carry = boff[blockIdx.x];
  for (int j = 0; j < kScanSpan / 1024; ++j) {
    const int64_t i = base + j * 1024;
    const int64_t v = i < L ? in[i] : 0;
    int64_t tot = 0;
    const int64_t ex = block_excl_scan(v, &tot);
    if (i < L) out[i] = static_cast<int32_t>(carry + ex);
    carry += tot;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[L] = static_cast<int32_t>(carry);
}

// Row prefix over destination partitions: png_off[p][0..k], row totals and the
// number of non-empty segments of each row.  One workgroup per row.
__global__ __launch_bounds__(256) void k_rowscan(int32_t k, const int32_t* __restrict__ cnt,
                                                 int32_t* __restrict__ png_off, int32_t* __restrict__ rowtot,
                                                 int32_t* __restrict__ rowseg) {
  const int64_t p = blockIdx.x;
  const int32_t per = (k + blockDim.x - 1) / blockDim.x;
  const int32_t j0 = min(k, static_cast<int32_t>(threadIdx.x) * per), j1 = min(k, j0 + per);
  int64_t sum = 0, nz = 0;
  for (int32_t j = j0; j < j1; ++j) {
    const int32_t c = cnt[p * k + j];
    sum += c;
    nz += (c > 0);
  }
  int64_t tot = 0, ntot = 0;
  int64_t run = block_excl_scan(sum, &tot);
  (void)block_excl_scan(nz, &ntot);
  for (int32_t j = j0; j < j1; ++j) {
    png_off[p * (k + 1) + j] = static_cast<int32_t>(run);
    run += cnt[p * k + j];
  }
  if (threadIdx.x == 0) {
    png_off[p * (k + 1) + k] = static_cast<int32_t>(tot);
    rowtot[p] = static_cast<int32_t>(tot);
    rowseg[p] = static_cast<int32_t>(ntot);
  }
}

// Exclusive scan of in[0..L) into out[0..L] (out[L] = total), one workgroup.
__global__ __launch_bounds__(1024) void k_scan_excl(const int32_t* __restrict__ in, int32_t* __restrict__ out,
                                                    int64_t L) {
  const int64_t per = (L + blockDim.x - 1) / blockDim.x;
  const int64_t i0 = min(L, static_cast<int64_t>(threadIdx.x) * per), i1 = min(L, i0 + per);
  int64_t sum = 0;
  for (int64_t i = i0; i < i1; ++i) sum += in[i];
  int64_t tot = 0;
  int64_t run = block_excl_scan(sum, &tot);
  for (int64_t i = i0; i < i1; ++i) {
    const int32_t v = in[i];
    out[i] = static_cast<int32_t>(run);
    run += v;
  }
  if (threadIdx.x == 0) out[L] = static_cast<int32_t>(tot);
}

// The scatter walks source partitions in pairs (P = {2P', 2P'+1}): for each
// destination p', the segments (2P', p') and (2P'+1, p') are adjacent in bin
// p' (the write offset of the second starts where the first ends), so the pair
// writes them as one run.  PNG edges are stored in (pair, p', node) order and
// a "pair segment" is the union of the two.  The bins, and the canonical
// per-partition layout that pcpm_png_export returns, are unchanged.
__device__ __forceinline__ int32_t pair_cnt(const int32_t* __restrict__ cnt, int32_t k, int64_t pair, int32_t j) {
  const int64_t p0 = 2 * pair, p1 = 2 * pair + 1;
  return cnt[p0 * k + j] + (p1 < k ? cnt[p1 * k + j] : 0);
}

// Non-empty (bin, source pair) segments of each destination bin.  One
// workgroup per bin.
__global__ __launch_bounds__(256) void k_binseg(int32_t k, const int32_t* __restrict__ cnt,
                                                int32_t* __restrict__ binseg) {
  const int32_t j = blockIdx.x;
  const int64_t npairs = (k + 1) / 2;
  int64_t nz = 0;
  for (int64_t pr = threadIdx.x; pr < npairs; pr += blockDim.x) nz += (pair_cnt(cnt, k, pr, j) > 0);
  int64_t tot = 0;
  (void)block_excl_scan(nz, &tot);
  if (threadIdx.x == 0) binseg[j] = static_cast<int32_t>(tot);
}

// PNG order of the updates: seg_delta[s] for the s-th non-empty segment in
// (bin p', pair) order: the
// PNG position of the pair segment's first update minus the bin-order index
// of its first message.  The updates of one segment are consecutive in both
// orders (U(2P', p') then U(2P'+1, p'), nodes ascending), so a message's
// update sits at its bin-order index plus its segment's delta.  One
// workgroup per bin.
__global__ __launch_bounds__(256) void k_segdelta_bins(int32_t k, const int32_t* __restrict__ cnt,
                                                  const int32_t* __restrict__ wo, const int32_t* __restrict__ png_off,
                                                  const int32_t* __restrict__ upd_start,
                                                  const int32_t* __restrict__ png_base,
                                                  const int32_t* __restrict__ segbase, int32_t* __restrict__ seg_delta) {
  const int32_t j = blockIdx.x;
  const int64_t npairs = (k + 1) / 2;
  const int64_t per = (npairs + blockDim.x - 1) / blockDim.x;
  const int64_t q0 = min(npairs, static_cast<int64_t>(threadIdx.x) * per), q1 = min(npairs, q0 + per);
  int64_t nz = 0;
  for (int64_t pr = q0; pr < q1; ++pr) nz += (pair_cnt(cnt, k, pr, j) > 0);
  int64_t tot = 0;
  int64_t idx = segbase[j] + block_excl_scan(nz, &tot);
  for (int64_t pr = q0; pr < q1; ++pr) {
    if (pair_cnt(cnt, k, pr, j) > 0) {
      const int64_t p0 = 2 * pr, p1 = 2 * pr + 1;
      const int64_t msg = static_cast<int64_t>(upd_start[j]) + wo[p0 * k + j];
      const int64_t pos = static_cast<int64_t>(png_base[p0]) + png_off[p0 * (k + 1) + j] +
                          (p1 < k ? png_off[p1 * (k + 1) + j] : 0);
      seg_delta[idx++] = static_cast<int32_t>(pos - msg);
    }
  }
}

// Non-empty pair segments of each pair.  One workgroup per pair.
__global__ __launch_bounds__(256) void k_pairseg(int32_t k, const int32_t* __restrict__ cnt,
                                                 int32_t* __restrict__ pairseg) {
  const int64_t pr = blockIdx.x;
  int64_t nz = 0;
  for (int32_t j = threadIdx.x; j < k; j += blockDim.x) nz += (pair_cnt(cnt, k, pr, j) > 0);
  int64_t tot = 0;
  (void)block_excl_scan(nz, &tot);
  if (threadIdx.x == 0) pairseg[pr] = static_cast<int32_t>(tot);
}

// Bin order of the updates: seg_delta[s] for the s-th non-empty pair segment
// in (pair, p') order, the update slot of its first entry minus its position
// in the pair-ordered PNG edges.  One workgroup per pair.
__global__ __launch_bounds__(256) void k_segdelta_pairs(int32_t k, const int32_t* __restrict__ cnt,
                                                  const int32_t* __restrict__ wo, const int32_t* __restrict__ png_off,
                                                  const int32_t* __restrict__ upd_start,
                                                  const int32_t* __restrict__ png_base,
                                                  const int32_t* __restrict__ segbase, int32_t* __restrict__ seg_delta) {
  const int64_t pr = blockIdx.x, p0 = 2 * pr, p1 = 2 * pr + 1;
  const int32_t per = (k + blockDim.x - 1) / blockDim.x;
  const int32_t j0 = min(k, static_cast<int32_t>(threadIdx.x) * per), j1 = min(k, j0 + per);
  int64_t nz = 0;
  for (int32_t j = j0; j < j1; ++j) nz += (pair_cnt(cnt, k, pr, j) > 0);
  int64_t tot = 0;
  int64_t idx = segbase[pr] + block_excl_scan(nz, &tot);
  for (int32_t j = j0; j < j1; ++j) {
    if (pair_cnt(cnt, k, pr, j) > 0) {
      const int64_t slot = static_cast<int64_t>(upd_start[j]) + wo[p0 * k + j];
      const int64_t pos = static_cast<int64_t>(png_base[p0]) + png_off[p0 * (k + 1) + j] +
                          (p1 < k ? png_off[p1 * (k + 1) + j] : 0);
      seg_delta[idx++] = static_cast<int32_t>(slot - pos);
    }
  }
}

// Fill, in two passes that write each bin and PNG region in long runs.  A
// direct fill stores every edge's 2-byte ID into one of k bins; with
// thousands of wavefronts each holding k half-written cache lines, the lines
// leave L2 before they are complete and every store costs a partial-line
// write to memory.
//
// Pass 1 (k_fill): one wavefront per chunk, edges in CSR order, 64 at a time.
// Lanes with the same destination partition form a peer group (one ballot
// per key bit, high bits first); an edge's destination-ID slot is its group's
// cursor plus the number of peer lanes below it (a stable multisplit, no
// atomics), and likewise its PNG slot for a message's first edge.  The
// lowest peer advances the cursors, which start at the chunk's prefixes of
// its partition's counts (the PNG cursor holds the absolute slot in the
// pair-ordered PNG edges, and in its top bit whether the next message
// starts the (pair, p') segment).  The edge's record (ID slot and value;
// PNG slot and value for a message's first edge; weight) goes to the region
// of its bucket, the 2^bbits destination partitions that share their high
// bits (64 buckets at most).  A bucket's region is the bucket's span of the
// ID array, so its cursor is the same prefix summed over the bucket's bins,
// and the records of a bucket lie in CSR order.
#ifndef PCPM_FILL_SETS
#define PCPM_FILL_SETS 4
#endif
constexpr int kFillSets = PCPM_FILL_SETS;  // 64-edge sets whose loads are issued together
#ifndef PCPM_FILL_BUCKETS
#define PCPM_FILL_BUCKETS 64
#endif
constexpr int kFillBuckets = PCPM_FILL_BUCKETS;  // most buckets of pass 1
__global__ __launch_bounds__(64) void k_fill(int s, int32_t k, int nbits, int bbits, const Item* __restrict__ chunks,
                                             const int32_t* __restrict__ col, const int32_t* __restrict__ src,
                                             const int32_t* __restrict__ did_start, const int32_t* __restrict__ dwo,
                                             const int32_t* __restrict__ ccnt, const int32_t* __restrict__ craw,
                                             const int32_t* __restrict__ png_base,
                                             const int32_t* __restrict__ png_off, const float* __restrict__ weights,
                                             uint64_t* __restrict__ rec, uint32_t* __restrict__ rpng,
                                             float* __restrict__ rw) {
  extern __shared__ int32_t sh[];
  int32_t* cur_did = sh;                                     // absolute destination-ID slot per p'
  uint32_t* cur_png = reinterpret_cast<uint32_t*>(sh + k);  // PNG slot per p' | segment-start bit
  int32_t* bcur = sh + 2 * k;                                // record slot per bucket
  const int32_t nb = ((k - 1) >> bbits) + 1;
  const int64_t c = blockIdx.x;
  const Item ch = chunks[c];
  const int64_t p = ch.part;
  const int lane = threadIdx.x;
  for (int32_t j = lane; j < nb; j += kWave) bcur[j] = 0;
  __syncthreads();
  // PNG slots: the pair's earlier pair segments, for the odd partition the
  // even one's run, then the chunk's rank inside U(p, p')
  const int64_t p0 = p & ~int64_t{1}, p1 = p0 + 1;
  const bool odd = (p & 1) != 0;
  const int32_t pbase = png_base[p0];
  for (int32_t j = lane; j < k; j += kWave) {
    const int32_t before = dwo[p * k + j] + craw[c * k + j];  // earlier edges into p' in CSR order
    cur_did[j] = did_start[j] + before;
    atomicAdd(&bcur[j >> bbits], before);
    const int32_t rank = ccnt[c * k + j];
    const int32_t even_off = png_off[p0 * (k + 1) + j];
    const int32_t even_cnt = png_off[p0 * (k + 1) + j + 1] - even_off;
    const int32_t odd_off = p1 < k ? png_off[p1 * (k + 1) + j] : 0;
    const uint32_t slot = static_cast<uint32_t>(pbase + even_off + odd_off + (odd ? even_cnt : 0) + rank);
    const bool seg_open = rank == 0 && (!odd || even_cnt == 0);
    cur_png[j] = slot | (seg_open ? kFlag : 0u);
  }
  __syncthreads();
  for (int32_t j = lane; j < nb; j += kWave) bcur[j] += did_start[j << bbits];
  __syncthreads();
  const int32_t e0 = ch.lo, e1 = ch.hi;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const uint32_t lmask = (1u << s) - 1u;
  // the edge before the current set; a source of -1 makes the next edge a
  // message start
  int32_t cu = -1, cv = 0;
  if (e0 > 0) {
    cu = src[e0 - 1];
    cv = col[e0 - 1];
  }
  // the next batch's loads are in flight while a batch is processed
  int32_t nu[kFillSets], nv[kFillSets];
  float nw[kFillSets];
#pragma unroll
  for (int t = 0; t < kFillSets; ++t) {
    const int32_t e = e0 + t * kWave + lane;
    nu[t] = e < e1 ? src[e] : 0;
    nv[t] = e < e1 ? col[e] : 0;
    nw[t] = (rw && e < e1) ? weights[e] : 0.0f;
  }
  for (int32_t cb = e0; cb < e1; cb += kFillSets * kWave) {
    int32_t us[kFillSets], vs[kFillSets], pps[kFillSets];
    float ws[kFillSets];
#pragma unroll
    for (int t = 0; t < kFillSets; ++t) {
      us[t] = nu[t];
      vs[t] = nv[t];
      ws[t] = nw[t];
    }
    if (cb + kFillSets * kWave < e1) {
#pragma unroll
      for (int t = 0; t < kFillSets; ++t) {
        const int32_t e = cb + (kFillSets + t) * kWave + lane;
        nu[t] = e < e1 ? src[e] : 0;
        nv[t] = e < e1 ? col[e] : 0;
        nw[t] = (rw && e < e1) ? weights[e] : 0.0f;
      }
    }
    // message starts and peer groups of all sets first (independent work,
    // one ballot per key bit and set), then the cursor updates in order
    bool firsts[kFillSets];
    uint64_t peers[kFillSets], bpeers[kFillSets], fmask[kFillSets];
#pragma unroll
    for (int t = 0; t < kFillSets; ++t) {
      const bool valid = cb + t * kWave + lane < e1;
      int32_t pu = __shfl_up(us[t], 1), pv = __shfl_up(vs[t], 1);
      if (lane == 0) {
        pu = cu;
        pv = cv;
      }
      cu = __builtin_amdgcn_readlane(us[t], 63);
      cv = __builtin_amdgcn_readlane(vs[t], 63);
      pps[t] = vs[t] >> s;
      firsts[t] = valid && (pu != us[t] || (pv >> s) != pps[t]);
      peers[t] = wave_ballot(valid);
      fmask[t] = wave_ballot(firsts[t]);
    }
    for (int b = nbits - 1; b >= bbits; --b) {
#pragma unroll
      for (int t = 0; t < kFillSets; ++t) {
        const bool bit = (pps[t] >> b) & 1;
        const uint64_t bb = wave_ballot(bit);
        peers[t] &= bit ? bb : ~bb;
      }
    }
#pragma unroll
    for (int t = 0; t < kFillSets; ++t) bpeers[t] = peers[t];  // same bucket
    for (int b = bbits - 1; b >= 0; --b) {
#pragma unroll
      for (int t = 0; t < kFillSets; ++t) {
        const bool bit = (pps[t] >> b) & 1;
        const uint64_t bb = wave_ballot(bit);
        peers[t] &= bit ? bb : ~bb;
      }
    }
#pragma unroll
    for (int t = 0; t < kFillSets; ++t) {
      if (cb + t * kWave >= e1) break;
      const bool valid = cb + t * kWave + lane < e1;
      const int32_t pp = pps[t];
      const uint64_t fpeers = peers[t] & fmask[t];
      const int32_t hb = pp >> bbits;
      int32_t cd = 0, bc = 0;
      uint32_t cp = 0;
      if (valid) {
        cd = cur_did[pp];
        cp = cur_png[pp];
        bc = bcur[hb];
      }
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        const int32_t ri = bc + __popcll(bpeers[t] & below);
        uint32_t flags = firsts[t] ? kDidFlag : 0u;
        uint32_t pval = 0;
        if (firsts[t]) {
          const int frank = __popcll(fpeers & below);
          const bool seg_first = (cp & kFlag) && frank == 0;
          // source ID local to the pair's 2q nodes, flag on the pair segment's first node
          pval = (static_cast<uint32_t>(us[t]) & ((2u << s) - 1u)) | (seg_first ? kDidFlag : 0u);
          rpng[ri] = (cp & kIdMask) + static_cast<uint32_t>(frank);
          // in bin p', the same edge starts the (p', pair) segment of destination IDs
          if (seg_first) flags |= kSegFlag;
        }
        const uint32_t dval = (static_cast<uint32_t>(vs[t]) & lmask) | flags;
        rec[ri] = static_cast<uint64_t>(static_cast<uint32_t>(cd + __popcll(peers[t] & below))) |
                  (static_cast<uint64_t>(dval) << 32) | (static_cast<uint64_t>(pval) << 48);
        if (rw) rw[ri] = ws[t];  // the weight travels with its destination ID (Sec. 3.5)
        if ((peers[t] & below) == 0) {
          cur_did[pp] = cd + __popcll(peers[t]);
          const int nf = __popcll(fpeers);
          if (nf) cur_png[pp] = (cp & kIdMask) + static_cast<uint32_t>(nf);
        }
        if ((bpeers[t] & below) == 0) bcur[hb] = bc + __popcll(bpeers[t]);
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// Pass 2 (k_place): workgroups take consecutive runs of records and store
// each ID (and PNG source ID, and weight) at its slot.  A run lies in one or
// two buckets, so its stores fall on at most 2 * 2^bbits bins, a long
// stretch of each; workgroups of neighbouring runs share an XCD (xcd_block),
// so the lines that two runs share fill in one L2.
constexpr int kPlaceBlock = 1024;
constexpr int kPlaceRecs = 16;  // records per thread
__global__ __launch_bounds__(kPlaceBlock) void k_place(int64_t m, const uint64_t* __restrict__ rec,
                                                       const uint32_t* __restrict__ rpng,
                                                       const float* __restrict__ rw, uint16_t* __restrict__ did,
                                                       uint16_t* __restrict__ png_src, float* __restrict__ wbin) {
  const int64_t base = static_cast<int64_t>(xcd_block(blockIdx.x, gridDim.x)) * (kPlaceBlock * kPlaceRecs) +
                       threadIdx.x;
  uint64_t r[kPlaceRecs];
  uint32_t pp[kPlaceRecs];
#pragma unroll
  for (int j = 0; j < kPlaceRecs; ++j) {
    const int64_t i = base + static_cast<int64_t>(j) * kPlaceBlock;
    r[j] = i < m ? rec[i] : 0;
    pp[j] = i < m ? rpng[i] : 0;  // read for every record; used for a message's first edge only
  }
#pragma unroll
  for (int j = 0; j < kPlaceRecs; ++j) {
    const int64_t i = base + static_cast<int64_t>(j) * kPlaceBlock;
    if (i < m) {
      const uint32_t dpos = static_cast<uint32_t>(r[j]);
      const uint32_t dval = static_cast<uint32_t>(r[j] >> 32) & 0xFFFFu;
      did[tile_pos(dpos)] = static_cast<uint16_t>(dval);
      if (dval & kDidFlag) png_src[tile_pos(pp[j])] = static_cast<uint16_t>(r[j] >> 48);
      if (wbin) wbin[dpos] = rw[i];
    }
  }
}

// Weight statistics for the SpMV's fixed-point scale: the largest |w| and
// the largest sum over v of |w(u,v)| (1 per edge when unweighted), as the
// bit patterns of non-negative doubles, whose order is that of the values;
// out[2] counts non-finite weights.  One workgroup per gather item (big bins
// are split over several): FP64 sums in an LDS slice; a whole bin takes its
// largest sum at once, the items of a split bin store their slices (as
// doubles in the partial-sum buffer) for k_w_stats_merge.
__global__ __launch_bounds__(1024) void k_w_stats(int64_t n, int s, const Item* __restrict__ items,
                                                  const uint16_t* __restrict__ did, const float* __restrict__ wbin,
                                                  int64_t* __restrict__ partial, unsigned long long* __restrict__ out) {
  extern __shared__ double csum[];
  const Item it = items[blockIdx.x];
  const int64_t q = int64_t{1} << s;
  const int64_t v0 = static_cast<int64_t>(it.part) << s;
  const int qn = static_cast<int>(min(q, n - v0));
  for (int i = threadIdx.x; i < qn; i += 1024) csum[i] = 0.0;
  __syncthreads();
  double wm = 0.0;
  int bad = 0;
  const uint32_t qmask = static_cast<uint32_t>(q - 1);
  for (int64_t e = it.lo + threadIdx.x; e < it.hi; e += 1024) {
    const uint32_t x = did[tile_pos(e)] & qmask;
    const float wf = wbin ? wbin[e] : 1.0f;
    if (!isfinite(wf)) {
      bad = 1;
      continue;
    }
    const double w = fabs(static_cast<double>(wf));
    wm = fmax(wm, w);
    atomicAdd(&csum[x], w);
  }
  __syncthreads();
  double cm = 0.0;
  if (it.aux >= 0) {
    double* dst = reinterpret_cast<double*>(partial + static_cast<int64_t>(it.aux) * q);
    for (int i = threadIdx.x; i < qn; i += 1024) dst[i] = csum[i];
  } else {
    for (int i = threadIdx.x; i < qn; i += 1024) cm = fmax(cm, csum[i]);
  }
  cm = block_max<1024>(cm);
  wm = block_max<1024>(wm);
  if (bad) atomicAdd(&out[2], 1ull);
  if (threadIdx.x == 0) {
    atomicMax(&out[0], static_cast<unsigned long long>(__double_as_longlong(cm)));
    atomicMax(&out[1], static_cast<unsigned long long>(__double_as_longlong(wm)));
  }
}

// Split bins: the sums of the items' slices, node by node, in slot order;
// one workgroup per merge unit (256 nodes).
__global__ __launch_bounds__(256) void k_w_stats_merge(int64_t n, int s, const Merge* __restrict__ mg,
                                                       const int64_t* __restrict__ partial,
                                                       unsigned long long* __restrict__ out) {
  const Merge mu = mg[blockIdx.x];
  const int64_t q = int64_t{1} << s;
  const int64_t v0 = static_cast<int64_t>(mu.part) << s;
  const int qn = static_cast<int>(min(q, n - v0));
  const int i = mu.node_lo + static_cast<int>(threadIdx.x);
  double sum = 0.0;
  if (i < qn) {
    const double* base = reinterpret_cast<const double*>(partial + static_cast<int64_t>(mu.first) * q);
    for (int c = 0; c < mu.count; ++c) sum += base[static_cast<int64_t>(c) * q + i];
  }
  const double cm = block_max<256>(sum);
  if (threadIdx.x == 0) atomicMax(&out[0], static_cast<unsigned long long>(__double_as_longlong(cm)));
}

// Number of entries with a flag bit (`flag`) set in each kTile tile of
// destination IDs (one wavefront per tile; the count does not depend on the
// storage order inside a tile).
__global__ __launch_bounds__(256) void k_tile_flags(const uint16_t* __restrict__ a, int64_t ntiles, uint32_t flag,
                                                    int32_t* __restrict__ cnt) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t t = wave; t < ntiles; t += nwaves) {
    int32_t c = 0;
    for (int j = 0; j < kSub; ++j) c += __popcll(wave_ballot((a[t * kTile + j * kWave + lane] & flag) != 0));
    if (lane == 0) cnt[t] = c;
  }
}

pcpm_status_t set_lds_limits() {
  static bool done = false;
  if (done) return PCPM_OK;
  PCPM_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_count),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 2 * kMaxParts * 4));
  PCPM_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_fill),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (2 * kMaxParts + kFillBuckets) * 4));
  done = true;
  return PCPM_OK;
}

// Exclusive scan of L int32 values: out[0..L), out[L] = total (in == out is
// allowed).  One workgroup up to kScanSpan values, else three launches;
// tmp holds scan_tmp_ints(L) ints.
int64_t scan_tmp_ints(int64_t L) { return 2 * ((L + kScanSpan - 1) / kScanSpan + 1); }

pcpm_status_t scan_excl_i32(const int32_t* in, int32_t* out, int64_t L, int32_t* tmp, hipStream_t st) {
  if (L <= kScanSpan) {
    PCPM_LAUNCH("pcpm_scan", k_scan_excl, dim3(1), dim3(1024), 0, st, in, out, L);
    return PCPM_OK;
  }
  const int64_t nblk = (L + kScanSpan - 1) / kScanSpan;
  int32_t* boff = tmp + nblk + 1;
  PCPM_LAUNCH("pcpm_scan", k_scan_sums, dim3(static_cast<unsigned>(nblk)), dim3(1024), 0, st, in, L, tmp);
  PCPM_LAUNCH("pcpm_scan", k_scan_excl, dim3(1), dim3(1024), 0, st, tmp, boff, nblk);
  PCPM_LAUNCH("pcpm_scan", k_scan_apply, dim3(static_cast<unsigned>(nblk)), dim3(1024), 0, st, in, L, boff, out);
  return PCPM_OK;
}

pcpm_status_t weight_stats(pcpm_png* g, hipStream_t st) {
  if (!g->wstats) PCPM_TRY(dalloc(g, &g->wstats, 3));
  PCPM_TRY_HIP(hipMemsetAsync(g->wstats, 0, 3 * sizeof(unsigned long long), st));
  PCPM_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_w_stats),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(g->q * 8)));
  if (g->n_ga)
    PCPM_LAUNCH("pcpm_wstats", k_w_stats, dim3(static_cast<unsigned>(g->n_ga)), dim3(1024),
                static_cast<size_t>(g->q * 8), st, g->n, g->part_log2, g->ga_items, g->did, g->wbin, g->partial,
                g->wstats);
  if (g->n_mg)
    PCPM_LAUNCH("pcpm_wstats", k_w_stats_merge, dim3(static_cast<unsigned>(g->n_mg)), dim3(256), 0, st, g->n,
                g->part_log2, g->mg_items, g->partial, g->wstats);
  g->wstats_ready = true;
  return PCPM_OK;
}

pcpm_status_t iter_lds_limits();  // pcpm_iter.hip

static bool is_device_ptr(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// Graphs of a multi-graph handle ("groups"): partition -> group, real nodes
// per partition, per-group 1/n_g.
static pcpm_status_t setup_groups(pcpm_png* g, const pcpm_build_opts_t* opts, hipStream_t st) {
  const int64_t G = (opts && opts->num_graphs > 1) ? opts->num_graphs : 1;
  const int64_t q = g->q, k = g->k, n = g->n;
  g->group_off.assign(G + 1, 0);
  g->group_n.assign(G, 0);
  if (G == 1) {
    g->group_off[1] = n;
    g->group_n[0] = n;
  } else {
    if (!opts->graph_node_off || !opts->graph_nodes)
      return set_error(PCPM_ERR_INVALID_ARG, "num_graphs > 1 needs graph_node_off and graph_nodes");
    for (int64_t i = 0; i <= G; ++i) g->group_off[i] = opts->graph_node_off[i];
    for (int64_t i = 0; i < G; ++i) g->group_n[i] = opts->graph_nodes[i];
    if (g->group_off[0] != 0 || g->group_off[G] != n)
      return set_error(PCPM_ERR_INVALID_ARG, "graph_node_off must start at 0 and end at n");
    for (int64_t i = 0; i < G; ++i) {
      if (g->group_off[i] % q != 0 || g->group_off[i + 1] <= g->group_off[i])
        return set_error(PCPM_ERR_INVALID_ARG, "graph %lld: offsets must increase in multiples of q",
                         static_cast<long long>(i));
      if (g->group_n[i] < 1 || g->group_n[i] > g->group_off[i + 1] - g->group_off[i])
        return set_error(PCPM_ERR_INVALID_ARG, "graph %lld: node count outside its range",
                         static_cast<long long>(i));
    }
  }
  g->ngroups = static_cast<int32_t>(G);
  std::vector<int32_t> pg(k), pv(k);
  for (int64_t grp = 0, p = 0; p < k; ++p) {
    while (p * q >= g->group_off[grp + 1]) ++grp;
    pg[p] = static_cast<int32_t>(grp);
    const int64_t real_end = g->group_off[grp] + g->group_n[grp];
    pv[p] = static_cast<int32_t>(std::max<int64_t>(0, std::min<int64_t>({q, n - p * q, real_end - p * q})));
  }
  std::vector<GCtl> gc(G);
  for (int64_t i = 0; i < G; ++i) {
    memset(&gc[i], 0, sizeof(GCtl));
    gc[i].inv_n = 1.0 / static_cast<double>(g->group_n[i]);
  }
  PCPM_TRY(dalloc(g, &g->part_group, k));
  PCPM_TRY(dalloc(g, &g->part_valid, k));
  PCPM_TRY(dalloc(g, &g->gctl, G));
  PCPM_TRY_HIP(hipHostMalloc(reinterpret_cast<void**>(&g->gctl_host), sizeof(GCtl) * G, hipHostMallocDefault));
  PCPM_TRY_HIP(hipMemcpyAsync(g->part_group, pg.data(), k * 4, hipMemcpyHostToDevice, st));
  PCPM_TRY_HIP(hipMemcpyAsync(g->part_valid, pv.data(), k * 4, hipMemcpyHostToDevice, st));
  PCPM_TRY_HIP(hipMemcpyAsync(g->gctl, gc.data(), sizeof(GCtl) * G, hipMemcpyHostToDevice, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  return PCPM_OK;
}

static pcpm_status_t build_items(pcpm_png* g, const pcpm_build_opts_t* opts, hipStream_t st) {
  const int64_t k = g->k;
  std::vector<int32_t> png_base(k + 1), did_start(k + 1);
  PCPM_TRY_HIP(hipMemcpyAsync(png_base.data(), g->png_base, (k + 1) * 4, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipMemcpyAsync(did_start.data(), g->did_start, (k + 1) * 4, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));

  auto chunk_for = [&](int64_t total, int64_t requested) -> int64_t {
    if (requested > 0) return requested;
    const int64_t mean = (total + k - 1) / std::max<int64_t>(k, 1);
    return std::max<int64_t>(2 * mean, 65536);
  };
  const int64_t sc = chunk_for(g->eprime, opts ? opts->scatter_chunk : 0);
  const int64_t gc = chunk_for(g->m, opts ? opts->gather_chunk : 0);

  std::vector<Item> sc_items, ga_items;
  std::vector<Merge> mg;
  for (int64_t pr = 0; 2 * pr < k; ++pr) {  // scatter items: ranges of one partition pair's PNG edges
    const int64_t a = png_base[2 * pr], b = png_base[std::min<int64_t>(2 * pr + 2, k)];
    if (b == a) continue;
    const int64_t nch = (b - a + 2 * sc - 1) / (2 * sc);
    const int64_t step = (b - a + nch - 1) / nch;
    for (int64_t lo = a; lo < b; lo += step)
      sc_items.push_back({static_cast<int32_t>(pr), static_cast<int32_t>(lo),
                          static_cast<int32_t>(std::min(b, lo + step)), 0});
  }
  int32_t slot = 0;
  const int64_t k_dst = (g->n_cols + g->q - 1) / g->q;  // column partitions (k for a graph)
  for (int64_t p = 0; p < k_dst; ++p) {
    const int64_t a = did_start[p], b = did_start[p + 1];
    const int64_t nch = std::max<int64_t>(1, (b - a + gc - 1) / gc);
    if (nch == 1) {
      ga_items.push_back({static_cast<int32_t>(p), static_cast<int32_t>(a), static_cast<int32_t>(b), -1});
      continue;
    }
    const int64_t step = (b - a + nch - 1) / nch;
    const int32_t first = slot;
    for (int64_t lo = a; lo < b; lo += step)
      ga_items.push_back({static_cast<int32_t>(p), static_cast<int32_t>(lo),
                          static_cast<int32_t>(std::min(b, lo + step)), slot++});
    ++g->n_split_bins;
    const int64_t qn = std::min<int64_t>(g->q, g->n_cols - p * g->q);
    for (int64_t nl = 0; nl < qn; nl += 256) mg.push_back({static_cast<int32_t>(p), first, slot - first,
                                                           static_cast<int32_t>(nl)});
  }
  // Workgroup b of a scatter or gather launch runs array entry xcd_block(b, n),
  // so XCD x runs one contiguous range of the array.  Scatter: with items in
  // source-partition order, pairs p and p+1, whose segments lie next to each
  // other in every bin, run together on one XCD and the cache lines they
  // share fill in its L2 once.  That order suits pairs of similar work; if it
  // would load one XCD more than 10% above the mean, the array instead holds
  // the items largest first in dispatch order.  Gather: always largest first.
  // Neighbouring bins together on one XCD would share lines too, but with
  // PNG-ordered updates their segments of a source pair are neighbours, so
  // 32 workgroups would read one small region of the update array at a time
  // (measured: the RMAT-24 gather 350 -> 461 us); bins in size order spread
  // the reads over the whole run of each pair.
  auto largest_first = [](std::vector<Item>& items) {
    const unsigned ni = static_cast<unsigned>(items.size());
    std::vector<Item> lpt = items;
    std::stable_sort(lpt.begin(), lpt.end(), [](const Item& x, const Item& y) { return (x.hi - x.lo) > (y.hi - y.lo); });
    for (unsigned b = 0; b < ni; ++b) items[xcd_block(b, ni)] = lpt[b];
  };
  {
    const unsigned ni = static_cast<unsigned>(sc_items.size());
    std::vector<int64_t> xw(kXcds, 0);
    int64_t tot = 0;
    for (unsigned b = 0; b < ni; ++b) {
      const Item& it = sc_items[xcd_block(b, ni)];
      xw[b % kXcds] += it.hi - it.lo;
      tot += it.hi - it.lo;
    }
    const int64_t worst = ni ? *std::max_element(xw.begin(), xw.end()) : 0;
    if (ni && worst * 10 > 11 * ((tot + kXcds - 1) / kXcds)) {
      largest_first(sc_items);
      g->scatter_order = 1;
    }
  }
  largest_first(ga_items);

  g->n_sc = static_cast<int32_t>(sc_items.size());
  g->n_ga = static_cast<int32_t>(ga_items.size());
  g->n_mg = static_cast<int32_t>(mg.size());
  g->n_split_slots = slot;
  PCPM_TRY(dalloc(g, &g->sc_items, g->n_sc));
  PCPM_TRY(dalloc(g, &g->ga_items, g->n_ga));
  PCPM_TRY(dalloc(g, &g->mg_items, g->n_mg));
  PCPM_TRY(dalloc(g, &g->partial, static_cast<int64_t>(slot) * g->q));  // int64 slices
  // one (residual, dangling, mass) triple per apply unit: bins applied by the
  // gather use slot p, merge units use k + unit; slots of split bins stay zero
  PCPM_TRY(dalloc(g, &g->red, 3 * (k + g->n_mg)));
  PCPM_TRY(dalloc(g, &g->red_start, 4 * k));
  PCPM_TRY_HIP(hipMemsetAsync(g->red, 0, static_cast<size_t>(3 * (k + g->n_mg)) * sizeof(double), st));
  // per group: first partition and first merge unit (units are in partition order)
  {
    const int64_t G = g->ngroups;
    std::vector<int32_t> gs(2 * (G + 1));
    size_t u = 0;
    for (int64_t grp = 0; grp <= G; ++grp) {
      const int64_t p0 = g->group_off[grp] / g->q;
      gs[2 * grp] = static_cast<int32_t>(grp == G ? k : p0);
      while (u < mg.size() && mg[u].part < (grp == G ? k : p0)) ++u;
      gs[2 * grp + 1] = static_cast<int32_t>(grp == G ? mg.size() : u);
    }
    PCPM_TRY(dalloc(g, &g->group_slots, 2 * (G + 1)));
    PCPM_TRY_HIP(hipMemcpyAsync(g->group_slots, gs.data(), gs.size() * 4, hipMemcpyHostToDevice, st));
  }
  if (g->n_sc)
    PCPM_TRY_HIP(hipMemcpyAsync(g->sc_items, sc_items.data(), sc_items.size() * sizeof(Item),
                                hipMemcpyHostToDevice, st));
  if (g->n_ga)
    PCPM_TRY_HIP(hipMemcpyAsync(g->ga_items, ga_items.data(), ga_items.size() * sizeof(Item),
                                hipMemcpyHostToDevice, st));
  if (g->n_mg)
    PCPM_TRY_HIP(hipMemcpyAsync(g->mg_items, mg.data(), mg.size() * sizeof(Merge), hipMemcpyHostToDevice, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  return PCPM_OK;
}

static pcpm_status_t build(int64_t n, int64_t m, const int32_t* row_off, const int32_t* col,
                           const pcpm_build_opts_t* opts, hipStream_t st, pcpm_png* g) {
  const int s = opts ? opts->part_log2 : 14;  // part_log2 = 0 (autotune) is handled by pcpm_build_png
  if (s < kMinLog2 || s > kMaxLog2)
    return set_error(PCPM_ERR_INVALID_ARG, "part_log2 %d outside [%d, %d]", s, kMinLog2, kMaxLog2);
  const int64_t q = int64_t{1} << s;
  const int64_t k = (n + q - 1) / q;
  if (k > kMaxParts)
    return set_error(PCPM_ERR_INVALID_ARG, "k = ceil(n/q) = %lld exceeds %d partitions",
                     static_cast<long long>(k), kMaxParts);
  g->n = n;
  g->m = m;
  g->q = q;
  g->k = k;
  g->part_log2 = s;
  PCPM_TRY(set_lds_limits());
  PCPM_TRY(iter_lds_limits());
  PCPM_TRY(setup_groups(g, opts, st));

  // ---- node pass -------------------------------------------------------------
  int32_t* src = nullptr;
  int32_t* counters = nullptr;
  int32_t* tile_row = nullptr;
  const int64_t ntiles_e = (m + kTile - 1) / kTile;
  PCPM_TRY(dalloc(g, &g->outdeg, n));
  PCPM_TRY(dalloc(g, &g->dmask, (n + 31) / 32));
  PCPM_TRY(dalloc(g, &src, m));
  PCPM_TRY(dalloc(g, &counters, 4));
  PCPM_TRY(dalloc(g, &tile_row, ntiles_e + 1));
  PCPM_TRY_HIP(hipMemsetAsync(counters, 0, 16, st));
  PCPM_TRY_HIP(hipMemsetAsync(tile_row, 0, static_cast<size_t>(ntiles_e + 1) * 4, st));
  {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    PCPM_LAUNCH("pcpm_build_nodes", k_node_pass, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, st, n, m,
                row_off, g->outdeg, g->dmask, tile_row, counters, s, g->part_valid);
    const int64_t eblocks = std::min<int64_t>((ntiles_e + kEdgeBlock / kWave - 1) / (kEdgeBlock / kWave), 65536);
    if (m > 0)
      PCPM_LAUNCH("pcpm_build_nodes", k_edge_pass, dim3(static_cast<unsigned>(eblocks)), dim3(kEdgeBlock), 0, st,
                  g->n_cols, g->matrix ? 0 : 1, m, row_off, col, src, tile_row, counters, s, g->part_group,
                  g->part_valid);
  }
  int32_t hc[4] = {0, 0, 0, 0};
  PCPM_TRY_HIP(hipMemcpyAsync(hc, counters, 16, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  if (hc[0]) {
    const char* what = (hc[0] & kErrOffsets)    ? "row offsets out of range or decreasing"
                       : (hc[0] & kErrEnds)     ? "row_off[0] != 0 or row_off[n] != m"
                       : (hc[0] & kErrRange)    ? "column index outside [0, n)"
                       : (hc[0] & kErrSelfLoop) ? "self-loop"
                       : (hc[0] & kErrOrder)    ? "row not strictly ascending (unsorted or duplicate edge)"
                       : (hc[0] & kErrGraphs)   ? "an edge leaves its graph or a padding node has edges"
                                                : "internal queue overflow";
    return set_error(hc[0] & kErrInternal ? PCPM_ERR_DEVICE : PCPM_ERR_GRAPH, "invalid CSR: %s (flags 0x%x)",
                     what, hc[0]);
  }
  g->n_dangling = hc[2];

  // ---- counts and scans ----------------------------------------------------------
  int32_t *cnt, *raw, *dwo, *coltot, *coltot_raw, *rowtot, *rowseg, *segbase;
  PCPM_TRY(dalloc(g, &cnt, k * k));
  PCPM_TRY(dalloc(g, &raw, k * k));
  PCPM_TRY(dalloc(g, &g->wo, k * k));
  PCPM_TRY(dalloc(g, &dwo, k * k));
  PCPM_TRY(dalloc(g, &coltot, k));
  PCPM_TRY(dalloc(g, &coltot_raw, k));
  PCPM_TRY(dalloc(g, &rowtot, k));
  PCPM_TRY(dalloc(g, &rowseg, k));
  PCPM_TRY(dalloc(g, &segbase, k + 1));
  PCPM_TRY(dalloc(g, &g->png_off, k * (k + 1)));
  PCPM_TRY(dalloc(g, &g->upd_start, k + 1));
  PCPM_TRY(dalloc(g, &g->did_start, k + 1));
  PCPM_TRY(dalloc(g, &g->png_base, k + 1));
  const unsigned kk = static_cast<unsigned>(k);
  // chunks of each source partition's edges, about m / max(k, 4096) edges each
  // (at least 16384), so that skewed partitions spread over many workgroups
  int32_t* pe_d = nullptr;
  PCPM_TRY(dalloc(g, &pe_d, k + 1));
  PCPM_LAUNCH("pcpm_build_chunks", k_part_edges, dim3(static_cast<unsigned>((k + 1 + 255) / 256)), dim3(256), 0, st,
              n, s, static_cast<int32_t>(k), row_off, pe_d);
  std::vector<int32_t> pe(k + 1), cfirst(k + 1);
  PCPM_TRY_HIP(hipMemcpyAsync(pe.data(), pe_d, (k + 1) * 4, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  const int64_t chunk_len = (opts && opts->build_chunk > 0)
                                ? opts->build_chunk
                                : std::max<int64_t>(16384, (m + std::max<int64_t>(k, 4096) - 1) / std::max<int64_t>(k, 4096));
  std::vector<Item> chunks;
  for (int64_t p = 0; p < k; ++p) {
    cfirst[p] = static_cast<int32_t>(chunks.size());
    const int64_t a = pe[p], b = pe[p + 1];
    const int64_t nch = std::max<int64_t>(1, (b - a + chunk_len - 1) / chunk_len);
    const int64_t step = std::max<int64_t>(1, (b - a + nch - 1) / nch);
    if (b == a) chunks.push_back({static_cast<int32_t>(p), static_cast<int32_t>(a), static_cast<int32_t>(a), 0});
    for (int64_t lo = a; lo < b; lo += step)
      chunks.push_back({static_cast<int32_t>(p), static_cast<int32_t>(lo), static_cast<int32_t>(std::min(b, lo + step)), 0});
  }
  cfirst[k] = static_cast<int32_t>(chunks.size());
  const int64_t nchunks = static_cast<int64_t>(chunks.size());
  Item* chunks_d = nullptr;
  int32_t *cfirst_d = nullptr, *ccnt = nullptr, *craw = nullptr;
  PCPM_TRY(dalloc(g, &chunks_d, nchunks));
  PCPM_TRY(dalloc(g, &cfirst_d, k + 1));
  PCPM_TRY(dalloc(g, &ccnt, nchunks * k));
  PCPM_TRY(dalloc(g, &craw, nchunks * k));
  PCPM_TRY_HIP(hipMemcpyAsync(chunks_d, chunks.data(), nchunks * sizeof(Item), hipMemcpyHostToDevice, st));
  PCPM_TRY_HIP(hipMemcpyAsync(cfirst_d, cfirst.data(), (k + 1) * 4, hipMemcpyHostToDevice, st));
  PCPM_LAUNCH("pcpm_build_count", k_count, dim3(static_cast<unsigned>(nchunks)), dim3(1024),
              static_cast<size_t>(2 * k * 4), st, s, static_cast<int32_t>(k), chunks_d, col, src, ccnt, craw);
  PCPM_LAUNCH("pcpm_build_count", k_chunk_scan, dim3(kk, static_cast<unsigned>((k + 255) / 256)), dim3(256), 0, st,
              static_cast<int32_t>(k), cfirst_d, ccnt, craw, cnt, raw);
  PCPM_LAUNCH("pcpm_build_colscan", k_colscan, dim3((kk + 255) / 256), dim3(256), 0, st, static_cast<int32_t>(k),
              cnt, raw, g->wo, dwo, coltot, coltot_raw);
  PCPM_LAUNCH("pcpm_build_rowscan", k_rowscan, dim3(kk), dim3(256), 0, st, static_cast<int32_t>(k), cnt,
              g->png_off, rowtot, rowseg);
  PCPM_LAUNCH("pcpm_build_scan", k_scan_excl, dim3(1), dim3(1024), 0, st, coltot, g->upd_start, k);
  PCPM_LAUNCH("pcpm_build_scan", k_scan_excl, dim3(1), dim3(1024), 0, st, coltot_raw, g->did_start, k);
  PCPM_LAUNCH("pcpm_build_scan", k_scan_excl, dim3(1), dim3(1024), 0, st, rowtot, g->png_base, k);
  PCPM_LAUNCH("pcpm_build_pairseg", k_binseg, dim3(kk), dim3(256), 0, st, static_cast<int32_t>(k), cnt, rowseg);
  PCPM_LAUNCH("pcpm_build_scan", k_scan_excl, dim3(1), dim3(1024), 0, st, rowseg, segbase, k);
  int32_t tot[2] = {0, 0};
  PCPM_TRY_HIP(hipMemcpyAsync(&tot[0], g->upd_start + k, 4, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipMemcpyAsync(&tot[1], segbase + k, 4, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  g->eprime = tot[0];
  g->nseg = tot[1];

  // Update order: PNG order when (pair, bin) segments are short on average
  // (the scatter's writes then break into many partial runs), else bin order.
  const int64_t order = opts ? opts->update_order : 0;
  if (order < 0 || order > 2) return set_error(PCPM_ERR_INVALID_ARG, "update_order must be 0, 1 or 2");
  g->png_order = order == 2 || (order == 0 && g->eprime < kPngOrderRun * g->nseg);
  PCPM_TRY(dalloc(g, &g->seg_delta, g->nseg + kWave));  // padded for the gathers' 64-wide delta loads
  PCPM_TRY_HIP(hipMemsetAsync(g->seg_delta + g->nseg, 0, kWave * sizeof(int32_t), st));
  if (g->png_order) {
    PCPM_LAUNCH("pcpm_build_segdelta", k_segdelta_bins, dim3(kk), dim3(256), 0, st, static_cast<int32_t>(k), cnt,
                g->wo, g->png_off, g->upd_start, g->png_base, segbase, g->seg_delta);
  } else {
    const int64_t npairs = (k + 1) / 2;
    PCPM_LAUNCH("pcpm_build_pairseg", k_pairseg, dim3(static_cast<unsigned>(npairs)), dim3(256), 0, st,
                static_cast<int32_t>(k), cnt, rowseg);
    PCPM_LAUNCH("pcpm_build_scan", k_scan_excl, dim3(1), dim3(1024), 0, st, rowseg, segbase, npairs);
    PCPM_LAUNCH("pcpm_build_segdelta", k_segdelta_pairs, dim3(static_cast<unsigned>(npairs)), dim3(256), 0, st,
                static_cast<int32_t>(k), cnt, g->wo, g->png_off, g->upd_start, g->png_base, segbase, g->seg_delta);
  }

  // ---- fill --------------------------------------------------------------------
  const int64_t ntp = (g->eprime + kTile - 1) / kTile;
  const int64_t ntd = (m + kTile - 1) / kTile;
  PCPM_TRY(dalloc(g, &g->png_src, std::max<int64_t>(ntp, 1) * kTile));
  PCPM_TRY(dalloc(g, &g->did, std::max<int64_t>(ntd, 1) * kTile));
  PCPM_TRY_HIP(hipMemsetAsync(g->png_src, 0, std::max<int64_t>(ntp, 1) * kTile * 2, st));
  PCPM_TRY_HIP(hipMemsetAsync(g->did, 0, std::max<int64_t>(ntd, 1) * kTile * 2, st));
  int nbits = 0;
  while ((int64_t{1} << nbits) < k) ++nbits;
  int bbits = 0;  // destination partitions per bucket: 2^bbits, at most kFillBuckets buckets
  while ((int64_t{1} << (nbits - bbits)) > kFillBuckets) ++bbits;
  const int64_t nbuckets = ((k - 1) >> bbits) + 1;
  const float* weights = opts ? opts->weights : nullptr;
  if (weights) {
    if (!is_device_ptr(weights)) return set_error(PCPM_ERR_INVALID_ARG, "weights must be a device pointer");
    // padded to whole tiles (zeros): the gather reads a tile's weights without a predicate
    PCPM_TRY(dalloc(g, &g->wbin, std::max<int64_t>(ntd, 1) * kTile));
    PCPM_TRY_HIP(hipMemsetAsync(g->wbin, 0, std::max<int64_t>(ntd, 1) * kTile * 4, st));
  }
  if (m > 0) {
    uint64_t* rec = nullptr;
    uint32_t* rpng = nullptr;
    float* rw = nullptr;
    PCPM_TRY(dalloc(g, &rec, m));
    PCPM_TRY(dalloc(g, &rpng, m));
    if (weights) PCPM_TRY(dalloc(g, &rw, m));
    PCPM_LAUNCH("pcpm_build_fill", k_fill, dim3(static_cast<unsigned>(nchunks)), dim3(64),
                static_cast<size_t>((2 * k + nbuckets) * 4), st, s, static_cast<int32_t>(k), nbits, bbits, chunks_d,
                col, src, g->did_start, dwo, ccnt, craw, g->png_base, g->png_off, weights, rec, rpng, rw);
    const int64_t per = int64_t{kPlaceBlock} * kPlaceRecs;
    PCPM_LAUNCH("pcpm_build_place", k_place, dim3(static_cast<unsigned>((m + per - 1) / per)), dim3(kPlaceBlock), 0,
                st, m, rec, rpng, rw, g->did, g->png_src, g->wbin);
    PCPM_TRY_HIP(hipStreamSynchronize(st));
    dfree(g, rec);
    dfree(g, rpng);
    if (rw) dfree(g, rw);
  }

  // ---- tile flag prefixes ----------------------------------------------------
  // Messages (bit 15) before every tile of destination IDs; with PNG-ordered
  // updates also (bin, pair) segments (bit 14), with bin-ordered updates the
  // pair segments (bit 15) before every tile of PNG edges.
  int32_t* tcnt = nullptr;
  int32_t* tsum = nullptr;  // per-workgroup sums of the long scans, then their offsets
  PCPM_TRY(dalloc(g, &tcnt, std::max(ntd, ntp) + 1));
  PCPM_TRY(dalloc(g, &tsum, scan_tmp_ints(std::max(ntd, ntp))));
  PCPM_TRY(dalloc(g, &g->did_blk, ntd + 1));
  if (g->png_order) PCPM_TRY(dalloc(g, &g->did_sblk, ntd + 1));
  else PCPM_TRY(dalloc(g, &g->png_blk, ntp + 1));
  for (int f = 0; f < 2; ++f) {
    const uint16_t* a = (f == 0 || g->png_order) ? g->did : g->png_src;
    const int64_t nt = (f == 0 || g->png_order) ? ntd : ntp;
    int32_t* out = f == 0 ? g->did_blk : (g->png_order ? g->did_sblk : g->png_blk);
    if (nt > 0)
      PCPM_LAUNCH("pcpm_build_tiles", k_tile_flags, dim3(static_cast<unsigned>(std::min<int64_t>((nt + 3) / 4, 16384))),
                  dim3(256), 0, st, a, nt, (f == 1 && g->png_order) ? kSegFlag : kDidFlag, tcnt);
    PCPM_TRY(scan_excl_i32(tcnt, out, nt, tsum, st));
  }

  // ---- iteration buffers -----------------------------------------------------------
  PCPM_TRY(dalloc(g, &g->upd, g->eprime + 1));  // + spare slot for masked stores
  PCPM_TRY(dalloc(g, &g->hist, kMaxHist));
  PCPM_TRY(dalloc(g, &g->ctl, 1));
  PCPM_TRY(dalloc(g, &g->psync, 1));
  PCPM_TRY(dalloc(g, &g->bin_done, g->k));
  PCPM_TRY(dalloc(g, &g->tmp_pr, n));
  PCPM_TRY_HIP(hipHostMalloc(reinterpret_cast<void**>(&g->ctl_host), 2 * sizeof(Ctl), hipHostMallocDefault));
  for (hipEvent_t& e : g->ctl_ev) PCPM_TRY_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  PCPM_TRY_HIP(hipHostMalloc(reinterpret_cast<void**>(&g->psync_host), sizeof(PSync), hipHostMallocDefault));
  PCPM_TRY(build_items(g, opts, st));

  // ---- weight statistics (scale of pcpm_spmv) -----------------------------------
  // weighted handles: now, to reject non-finite weights; unweighted ones on
  // their first pcpm_spmv (PageRank does not use them)
  if (g->wbin) {
    PCPM_TRY(weight_stats(g, st));
    unsigned long long bad = 0;
    PCPM_TRY_HIP(hipMemcpyAsync(&bad, g->wstats + 2, sizeof(bad), hipMemcpyDeviceToHost, st));
    PCPM_TRY_HIP(hipStreamSynchronize(st));
    if (bad) return set_error(PCPM_ERR_INVALID_ARG, "weights hold %llu non-finite values", bad);
  }

  // ---- release build-only buffers ------------------------------------------------
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  for (void* p : {static_cast<void*>(pe_d), static_cast<void*>(chunks_d), static_cast<void*>(cfirst_d),
                  static_cast<void*>(ccnt), static_cast<void*>(craw)})
    dfree(g, p);
  for (void* p : {static_cast<void*>(src), static_cast<void*>(counters), static_cast<void*>(tile_row),
                  static_cast<void*>(raw), static_cast<void*>(dwo), static_cast<void*>(coltot),
                  static_cast<void*>(coltot_raw), static_cast<void*>(rowtot), static_cast<void*>(rowseg),
                  static_cast<void*>(segbase), static_cast<void*>(tcnt), static_cast<void*>(tsum),
                  static_cast<void*>(cnt)})
    dfree(g, p);
  return PCPM_OK;
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t* __restrict__ a, int64_t len, int32_t v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * 256)
    a[i] = v;
}

// ---- measured choice of the configuration (part_log2 = 0) --------------------------
// The paper chooses its partition size from a sweep of execution time over
// partition sizes (Sec. 5.3.2, Figs. 11-14); the same sweep runs here on the
// GPU at build time: every candidate q and update order is built and a few
// iterations are timed, then the work-item chunks of the fastest are varied
// (the items are rebuilt on the same PNG) and timed.  The winner is kept per
// process, keyed by the graph's content hash, the options and the device.

// Order-dependent 64-bit hash of an int32 array: the wrapping sum over i of
// a mix of (salt, i, a[i]); equal arrays give equal sums whatever the order
// of the additions.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void k_hash(const int32_t* __restrict__ a, int64_t len, uint64_t salt,
                                              unsigned long long* __restrict__ out) {
  uint64_t h = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * 256)
    h += mix64(salt ^ mix64(static_cast<uint64_t>(i) * 0x100000001B3ull + static_cast<uint32_t>(a[i])));
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) h += __shfl_xor(h, off);
  if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(out, static_cast<unsigned long long>(h));
}

static pcpm_status_t graph_hash(int64_t n, int64_t m, const int32_t* row_off, const int32_t* col, hipStream_t st,
                                uint64_t* out) {
  unsigned long long* d = nullptr;
  PCPM_TRY_HIP(hipMalloc(&d, 16));
  pcpm_status_t rc = PCPM_OK;
  do {
    if (hipMemsetAsync(d, 0, 16, st) != hipSuccess) { rc = set_error(PCPM_ERR_DEVICE, "hash: memset failed"); break; }
    const unsigned b1 = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((n + 256) / 256, 4096)));
    hipLaunchKernelGGL(k_hash, dim3(b1), dim3(256), 0, st, row_off, n + 1, uint64_t{0x726F775F6F6666ull}, d);
    if (m > 0) {
      const unsigned b2 = static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((m + 255) / 256, 8192)));
      hipLaunchKernelGGL(k_hash, dim3(b2), dim3(256), 0, st, col, m, uint64_t{0x636F6C756D6Eull}, d + 1);
    }
    if (hipGetLastError() != hipSuccess) { rc = set_error(PCPM_ERR_DEVICE, "hash: launch failed"); break; }
    unsigned long long h[2] = {0, 0};
    if (hipMemcpyAsync(h, d, 16, hipMemcpyDeviceToHost, st) != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
      rc = set_error(PCPM_ERR_DEVICE, "hash: copy failed");
      break;
    }
    *out = h[0] * 0x9E3779B97F4A7C15ull ^ h[1] ^ static_cast<uint64_t>(n) << 1 ^ static_cast<uint64_t>(m) << 33;
  } while (false);
  (void)hipFree(d);
  return rc;
}

struct TuneRecord {
  std::vector<pcpm_tune_entry_t> table;
  int32_t best = -1;
};
static std::mutex g_tune_mu;
static std::map<std::string, TuneRecord> g_tune_cache;

static std::string tune_key(int64_t n, int64_t m, uint64_t h, const pcpm_build_opts_t& o, int64_t mask, int device) {
  hipDeviceProp_t prop;
  std::string name = hipGetDeviceProperties(&prop, device) == hipSuccess ? prop.name : "?";
  char buf[512];
  uint64_t gh = 0;
  if (o.num_graphs > 1)
    for (int64_t i = 0; i <= o.num_graphs; ++i) gh = gh * 1000003ull + static_cast<uint64_t>(o.graph_node_off[i]);
  std::snprintf(buf, sizeof buf, "dev=%d:%s;n=%lld;m=%lld;h=%016llx;G=%d;gh=%016llx;w=%d;v=%lld;mask=%llx;o=%lld;sc=%lld;"
                "gc=%lld;bc=%lld", device, name.c_str(), static_cast<long long>(n), static_cast<long long>(m),
                static_cast<unsigned long long>(h), o.num_graphs, static_cast<unsigned long long>(gh),
                o.weights ? 1 : 0, static_cast<long long>(o.tune_vectors), static_cast<unsigned long long>(mask),
                static_cast<long long>(o.update_order), static_cast<long long>(o.scatter_chunk),
                static_cast<long long>(o.gather_chunk), static_cast<long long>(o.build_chunk));
  return buf;
}

// Work items again with other chunk sizes on the same PNG (the buffers that
// depend on the items are reallocated; the batched working set is dropped).
static pcpm_status_t rebuild_items(pcpm_png* g, const pcpm_build_opts_t& o, hipStream_t st) {
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  for (void* p : {static_cast<void*>(g->sc_items), static_cast<void*>(g->ga_items), static_cast<void*>(g->mg_items),
                  static_cast<void*>(g->partial), static_cast<void*>(g->red), static_cast<void*>(g->red_start),
                  static_cast<void*>(g->group_slots)})
    if (p) dfree(g, p);
  g->sc_items = g->ga_items = nullptr;
  g->mg_items = nullptr;
  g->partial = nullptr;
  g->red = g->red_start = nullptr;
  g->group_slots = nullptr;
  g->n_split_bins = g->n_split_slots = 0;
  g->scatter_order = 0;
  if (g->ppr_kt) {
    for (void* p : {static_cast<void*>(g->ppr_x[0]), static_cast<void*>(g->ppr_x[1]),
                    static_cast<void*>(g->ppr_upd), static_cast<void*>(g->ppr_partial),
                    static_cast<void*>(g->ppr_red), static_cast<void*>(g->ppr_vctl), static_cast<void*>(g->ppr_mask)})
      if (p) dfree(g, p);
    g->ppr_x[0] = g->ppr_x[1] = g->ppr_upd = nullptr;
    g->ppr_partial = nullptr;
    g->ppr_red = nullptr;
    g->ppr_vctl = nullptr;
    g->ppr_mask = nullptr;
    g->ppr_kt = 0;
  }
  return build_items(g, &o, st);
}

// Time per iteration (per vector-iteration for vectors > 1) of a handle:
// a warm-up, then `reps` runs of `iters` iterations.
static pcpm_status_t time_handle(pcpm_png* g, int64_t vectors, float* work, hipStream_t st, double* ms) {
  // the fastest of kReps runs of kIters iterations: the minimum is robust to
  // interference, and runs of a few ms keep launch noise small
  constexpr int kIters = 6, kReps = 3;
  int kv = 1;
  std::vector<int32_t> off, seeds;
  if (vectors > 1) {  // kv seed sets of `per` consecutive nodes
    kv = static_cast<int>(std::min<int64_t>(vectors, pcpm_ppr_tile_width(g)));
    const int per = static_cast<int>(std::min<int64_t>(8, g->n));
    for (int j = 0; j <= kv; ++j) off.push_back(j * per);
    for (int j = 0; j < kv; ++j)
      for (int i = 0; i < per; ++i)
        seeds.push_back(static_cast<int32_t>((static_cast<int64_t>(j) * 7919 * per + i) % g->n));
  }
  std::vector<int32_t> it(kv);
  std::vector<double> res(kv);
  auto run = [&](int iters) -> pcpm_status_t {
    int32_t i1 = 0;
    double r1 = 0.0;
    if (g->matrix) {  // a matrix: the SpMV itself (x and y in the two halves of work)
      for (int i = 0; i < iters; ++i) PCPM_TRY(pcpm_spmv(g, work, work + g->n, st));
      return hipStreamSynchronize(st) == hipSuccess ? PCPM_OK : set_error(PCPM_ERR_DEVICE, "sync failed");
    }
    if (vectors > 1)
      return pcpm_ppr_batch(g, 0.85, kv, off.data(), seeds.data(), 0.0, iters, work, it.data(), res.data(), st);
    return pcpm_pagerank(g, 0.85, 0.0, iters, nullptr, work, &i1, &r1, nullptr, st);
  };
  PCPM_TRY(run(2));
  double best = 0.0;
  for (int r = 0; r < kReps; ++r) {
    const auto t0 = std::chrono::steady_clock::now();
    PCPM_TRY(run(kIters));
    const double t = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    best = r == 0 ? t : std::min(best, t);
  }
  *ms = best / kIters / kv;
  return PCPM_OK;
}

static pcpm_status_t tuned_build(int64_t n, int64_t m, const int32_t* row_off, const int32_t* col,
                                 const pcpm_build_opts_t* opts, hipStream_t st, pcpm_png** out) {
  pcpm_build_opts_t o{};
  if (opts) o = *opts;
  int device = 0;
  PCPM_TRY_HIP(hipGetDevice(&device));
  const int64_t mask = o.tune_log2_mask ? o.tune_log2_mask : ((1 << 12) | (1 << 13) | (1 << 14));
  if (mask & ~((int64_t{1} << (kMaxLog2 + 1)) - (int64_t{1} << kMinLog2)))
    return set_error(PCPM_ERR_INVALID_ARG, "tune_log2_mask 0x%llx has bits outside [%d, %d]",
                     static_cast<unsigned long long>(mask), kMinLog2, kMaxLog2);
  if (o.num_graphs > 1 && !o.graph_node_off) return set_error(PCPM_ERR_INVALID_ARG, "graph_node_off is NULL");
  uint64_t h = 0;
  PCPM_TRY(graph_hash(n, m, row_off, col, st, &h));
  const std::string key = tune_key(n, m, h, o, mask, device);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto hit = g_tune_cache.find(key);
    if (hit != g_tune_cache.end()) {
      const pcpm_tune_entry_t& e = hit->second.table[hit->second.best];
      pcpm_build_opts_t b = o;
      b.part_log2 = e.part_log2;
      b.update_order = e.update_order;
      b.scatter_chunk = e.scatter_chunk;
      b.gather_chunk = e.gather_chunk;
      pcpm_png* g = nullptr;
      PCPM_TRY(pcpm_build_png(n, m, row_off, col, &b, st, &g));
      g->tune_table = hit->second.table;
      g->tune_best = hit->second.best;
      g->tune_cached = 1;
      *out = g;
      return PCPM_OK;
    }
  }
  // timing output: n * min(v, 16) floats
  float* work = nullptr;
  const int64_t wv = o.tune_vectors > 1 ? std::min<int64_t>(o.tune_vectors, 16) : 2;
  const int64_t wn = std::max<int64_t>(n, o.num_cols);
  PCPM_TRY_HIP(hipMalloc(&work, static_cast<size_t>(wn) * wv * sizeof(float)));
  PCPM_TRY_HIP(hipMemsetAsync(work, 0, static_cast<size_t>(wn) * wv * sizeof(float), st));
  struct Guard {
    float* w;
    pcpm_png* best = nullptr;
    ~Guard() {
      if (w) (void)hipFree(w);
      if (best) free_handle(best);
    }
  } guard{work};
  std::vector<pcpm_tune_entry_t> table;
  int32_t best = -1;
  pcpm_build_opts_t best_opts = o;
  const int64_t orders[2] = {1, 2};
  for (int s = kMinLog2; s <= kMaxLog2; ++s) {
    if (!((mask >> s) & 1)) continue;
    const int64_t q = int64_t{1} << s;
    if ((n + q - 1) / q > kMaxParts) continue;
    bool aligned = true;
    for (int64_t i = 0; o.num_graphs > 1 && i <= o.num_graphs; ++i) aligned &= (o.graph_node_off[i] % q) == 0;
    if (!aligned) continue;
    for (int64_t order : orders) {
      if (o.update_order && order != o.update_order) continue;
      pcpm_build_opts_t b = o;
      b.part_log2 = s;
      b.update_order = order;
      pcpm_png* g = nullptr;
      const auto t0 = std::chrono::steady_clock::now();
      PCPM_TRY(pcpm_build_png(n, m, row_off, col, &b, st, &g));
      const double bms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      double ms = 0.0;
      const pcpm_status_t rc = time_handle(g, o.tune_vectors, work, st, &ms);
      if (rc != PCPM_OK) {
        free_handle(g);
        return rc;
      }
      table.push_back({s, static_cast<int32_t>(order), o.scatter_chunk, o.gather_chunk, ms, bms});
      if (best < 0 || ms < table[best].ms_per_iter) {
        best = static_cast<int32_t>(table.size() - 1);
        best_opts = b;
        if (guard.best) free_handle(guard.best);
        guard.best = g;
      } else {
        free_handle(g);
      }
    }
  }
  if (best < 0) return set_error(PCPM_ERR_INVALID_ARG, "no autotune candidate fits this graph");
  // work-item chunks of the fastest PNG: the automatic value, half and double
  pcpm_png* g = guard.best;
  const int64_t auto_sc = std::max<int64_t>(2 * ((g->eprime + g->k - 1) / g->k), 65536);
  const int64_t auto_gc = std::max<int64_t>(2 * ((g->m + g->k - 1) / g->k), 65536);
  for (int field = 0; field < 2; ++field) {
    if ((field == 0 ? o.gather_chunk : o.scatter_chunk) != 0) continue;  // fixed by the caller
    const int64_t a = field == 0 ? auto_gc : auto_sc;
    for (int64_t c : {a / 2, a * 2}) {
      pcpm_build_opts_t b = best_opts;
      (field == 0 ? b.gather_chunk : b.scatter_chunk) = std::max<int64_t>(c, 4096);
      PCPM_TRY(rebuild_items(g, b, st));
      double ms = 0.0;
      PCPM_TRY(time_handle(g, o.tune_vectors, work, st, &ms));
      table.push_back({b.part_log2, static_cast<int32_t>(b.update_order), b.scatter_chunk, b.gather_chunk, ms, 0.0});
      if (ms < table[best].ms_per_iter) {
        best = static_cast<int32_t>(table.size() - 1);
        best_opts = b;
      }
    }
  }
  PCPM_TRY(rebuild_items(g, best_opts, st));
  g->tune_table = table;
  g->tune_best = best;
  g->tune_cached = 0;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    TuneRecord& rec = g_tune_cache[key];
    rec.table = table;
    rec.best = best;
  }
  guard.best = nullptr;
  *out = g;
  return PCPM_OK;
}

}  // namespace pcpm

extern "C" {

pcpm_status_t pcpm_build_png(int64_t n, int64_t m, const int32_t* row_off, const int32_t* col,
                             const pcpm_build_opts_t* opts, void* stream, pcpm_png_t* out) {
  using namespace pcpm;
  if (!out) return set_error(PCPM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n < 1 || m < 0) return set_error(PCPM_ERR_INVALID_ARG, "n must be >= 1 and m >= 0");
  if (n >= (int64_t{1} << 31) || m >= (int64_t{1} << 31))
    return set_error(PCPM_ERR_OVERFLOW, "n and m must be below 2^31 (the top ID bit is the message flag)");
  if (!row_off || (m > 0 && !col)) return set_error(PCPM_ERR_INVALID_ARG, "row_off or col is NULL");
  if (!is_device_ptr(row_off) || (m > 0 && !is_device_ptr(col)))
    return set_error(PCPM_ERR_INVALID_ARG, "row_off and col must be device pointers");
  const auto t0 = std::chrono::steady_clock::now();
  if (opts && opts->part_log2 == 0) {  // autotune: the sweep builds and times candidates
    pcpm_png* tg = nullptr;
    PCPM_TRY(tuned_build(n, m, row_off, col, opts, static_cast<hipStream_t>(stream), &tg));
    tg->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = tg;
    return PCPM_OK;
  }
  // a matrix (generic SpMV, Sec. 3.5): n rows, num_cols columns, possibly
  // diagonal entries; its node slots cover max(rows, cols), rows past n empty
  const int64_t ncols = (opts && opts->num_cols > 0) ? opts->num_cols : n;
  const bool matrix = ncols != n || (opts && opts->allow_diagonal);
  if (ncols >= (int64_t{1} << 31)) return set_error(PCPM_ERR_OVERFLOW, "num_cols must be below 2^31");
  if (matrix && opts->num_graphs > 1) return set_error(PCPM_ERR_INVALID_ARG, "a matrix handle holds one matrix");
  pcpm_png* g = new (std::nothrow) pcpm_png();
  if (!g) return set_error(PCPM_ERR_OOM, "host allocation failed");
  if (hipGetDevice(&g->device) != hipSuccess) {
    delete g;
    return set_error(PCPM_ERR_DEVICE, "no current HIP device");
  }
  g->n_rows = n;
  g->n_cols = ncols;
  g->matrix = matrix;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nslots = std::max(n, ncols);
  int32_t* ext = nullptr;  // row offsets over every node slot
  pcpm_status_t rc = PCPM_OK;
  if (nslots > n) {
    if (hipMalloc(&ext, static_cast<size_t>(nslots + 1) * 4) != hipSuccess) {
      (void)hipGetLastError();
      free_handle(g);
      return set_error(PCPM_ERR_OOM, "row offset extension of %lld entries", static_cast<long long>(nslots + 1));
    }
    if (hipMemcpyAsync(ext, row_off, static_cast<size_t>(n + 1) * 4, hipMemcpyDeviceToDevice, st) != hipSuccess)
      rc = set_error(PCPM_ERR_DEVICE, "row offset copy failed");
    else
      hipLaunchKernelGGL(k_fill_i32, dim3(static_cast<unsigned>(std::min<int64_t>((nslots - n + 255) / 256, 4096))),
                         dim3(256), 0, st, ext + n + 1, nslots - n, static_cast<int32_t>(m));
  }
  if (rc == PCPM_OK) rc = build(nslots, m, ext ? ext : row_off, col, opts, st, g);
  if (ext) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(ext);
  }
  if (rc != PCPM_OK) {
    (void)hipStreamSynchronize(st);
    free_handle(g);
    return rc;
  }
  g->build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = g;
  return PCPM_OK;
}

int32_t pcpm_tune_table(pcpm_png_t g, pcpm_tune_entry_t* out, int32_t max_entries, int32_t* best, int32_t* cached) {
  if (!g) return 0;
  const int32_t cnt = static_cast<int32_t>(g->tune_table.size());
  for (int32_t i = 0; out && i < std::min(cnt, max_entries); ++i) out[i] = g->tune_table[i];
  if (best) *best = g->tune_best;
  if (cached) *cached = g->tune_cached;
  return cnt;
}

void pcpm_tune_cache_clear(void) {
  std::lock_guard<std::mutex> lock(pcpm::g_tune_mu);
  pcpm::g_tune_cache.clear();
}

pcpm_status_t pcpm_graph_hash(int64_t n, int64_t m, const int32_t* row_off, const int32_t* col, void* stream,
                              uint64_t* out) {
  using namespace pcpm;
  if (!out || n < 1 || m < 0 || !row_off || (m > 0 && !col))
    return set_error(PCPM_ERR_INVALID_ARG, "bad size, NULL array or NULL output");
  if (!is_device_ptr(row_off) || (m > 0 && !is_device_ptr(col)))
    return set_error(PCPM_ERR_INVALID_ARG, "row_off and col must be device pointers");
  return graph_hash(n, m, row_off, col, static_cast<hipStream_t>(stream), out);
}

pcpm_status_t pcpm_png_info(pcpm_png_t g, pcpm_png_info_t* out) {
  using namespace pcpm;
  if (!g || !out) return set_error(PCPM_ERR_INVALID_ARG, "NULL handle or output");
  out->n = g->n;
  out->m = g->m;
  out->q = g->q;
  out->k = g->k;
  out->eprime = g->eprime;
  out->nseg = g->nseg;
  out->n_dangling = g->n_dangling;
  out->scatter_items = g->n_sc;
  out->gather_items = g->n_ga;
  out->split_bins = g->n_split_bins;
  out->device_bytes = g->device_bytes;
  out->num_graphs = g->ngroups;
  out->build_ms = g->build_ms;
  out->weighted = g->wbin ? 1 : 0;
  out->update_order = g->png_order ? 2 : 1;
  out->num_cols = g->n_cols;
  out->matrix = g->matrix ? 1 : 0;
  if (g->matrix) out->n = g->n_rows;
  return PCPM_OK;
}

pcpm_status_t pcpm_png_export_weights(pcpm_png_t g, float* w) {
  using namespace pcpm;
  if (!g || !w) return set_error(PCPM_ERR_INVALID_ARG, "NULL handle or output");
  if (!g->wbin) return set_error(PCPM_ERR_INVALID_ARG, "the handle has no edge weights");
  PCPM_TRY_HIP(hipSetDevice(g->device));
  PCPM_TRY_HIP(hipDeviceSynchronize());
  if (g->m > 0) PCPM_TRY_HIP(hipMemcpy(w, g->wbin, static_cast<size_t>(g->m) * 4, hipMemcpyDeviceToHost));
  return PCPM_OK;
}

pcpm_status_t pcpm_png_export(pcpm_png_t g, int64_t* png_off, int32_t* png_src, int64_t* upd_start, int64_t* wo,
                              int64_t* did_start, uint32_t* did) {
  using namespace pcpm;
  if (!g) return set_error(PCPM_ERR_INVALID_ARG, "NULL handle");
  PCPM_TRY_HIP(hipSetDevice(g->device));
  PCPM_TRY_HIP(hipDeviceSynchronize());
  const int64_t k = g->k;
  auto widen = [](const std::vector<int32_t>& a, int64_t* out) {
    for (size_t i = 0; i < a.size(); ++i) out[i] = a[i];
  };
  if (png_off) {
    std::vector<int32_t> t(k * (k + 1));
    PCPM_TRY_HIP(hipMemcpy(t.data(), g->png_off, t.size() * 4, hipMemcpyDeviceToHost));
    widen(t, png_off);
  }
  if (wo) {
    std::vector<int32_t> t(k * k);
    PCPM_TRY_HIP(hipMemcpy(t.data(), g->wo, t.size() * 4, hipMemcpyDeviceToHost));
    widen(t, wo);
  }
  if (upd_start) {
    std::vector<int32_t> t(k + 1);
    PCPM_TRY_HIP(hipMemcpy(t.data(), g->upd_start, t.size() * 4, hipMemcpyDeviceToHost));
    widen(t, upd_start);
  }
  if (did_start) {
    std::vector<int32_t> t(k + 1);
    PCPM_TRY_HIP(hipMemcpy(t.data(), g->did_start, t.size() * 4, hipMemcpyDeviceToHost));
    widen(t, did_start);
  }
  if (png_src && g->eprime > 0) {
    // stored partition-local with a 16-bit flag; exported as global node IDs
    // (in the tile storage order of tile_pos, up to the end of the last 128-entry block)
    std::vector<uint16_t> loc((g->eprime + 127) / 128 * 128);
    std::vector<int32_t> pb(k + 1);
    std::vector<int32_t> po(k * (k + 1));
    PCPM_TRY_HIP(hipMemcpy(loc.data(), g->png_src, loc.size() * 2, hipMemcpyDeviceToHost));
    PCPM_TRY_HIP(hipMemcpy(pb.data(), g->png_base, (k + 1) * 4, hipMemcpyDeviceToHost));
    PCPM_TRY_HIP(hipMemcpy(po.data(), g->png_off, po.size() * 4, hipMemcpyDeviceToHost));
    // stored in partition-pair order (see k_segdelta); exported per partition
    for (int64_t p = 0; p < k; ++p) {
      const int64_t p0 = p & ~int64_t{1}, p1 = p0 + 1;
      for (int64_t j = 0; j < k; ++j) {
        const int64_t a = po[p * (k + 1) + j], c = po[p * (k + 1) + j + 1] - a;
        const int64_t even_off = po[p0 * (k + 1) + j], even_cnt = po[p0 * (k + 1) + j + 1] - even_off;
        const int64_t odd_off = p1 < k ? po[p1 * (k + 1) + j] : 0;
        const int64_t src = pb[p0] + even_off + odd_off + ((p & 1) ? even_cnt : 0);
        for (int64_t r = 0; r < c; ++r)
          png_src[pb[p] + a + r] = static_cast<int32_t>(p0 * g->q + (loc[tile_pos(src + r)] & (kDidFlag - 1u)));
      }
    }
  }
  if (did && g->m > 0) {
    // stored partition-local with a 16-bit flag; exported as global IDs with the top-bit flag
    std::vector<uint16_t> loc((g->m + 127) / 128 * 128);
    std::vector<int32_t> ds(k + 1);
    PCPM_TRY_HIP(hipMemcpy(loc.data(), g->did, loc.size() * 2, hipMemcpyDeviceToHost));
    PCPM_TRY_HIP(hipMemcpy(ds.data(), g->did_start, (k + 1) * 4, hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < k; ++p) {
      const uint32_t base = static_cast<uint32_t>(p * g->q);
      for (int64_t e = ds[p]; e < ds[p + 1]; ++e) {
        const uint16_t x = loc[tile_pos(e)];
        did[e] = (base + (x & (kSegFlag - 1u))) | ((x & kDidFlag) ? kFlag : 0u);
      }
    }
  }
  return PCPM_OK;
}

}  // extern "C"
