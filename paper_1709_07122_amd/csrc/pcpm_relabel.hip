// Degree-ordered relabelling of a CSR graph on the GPU.  Sec. 5.3.1 and
// Table 6: the compression ratio r of the PNG, and with it the traffic of
// Sec. 4, rises with a labelling that puts related nodes close; in-degree
// order gathers the hubs (most destination IDs) into the first partitions.
//
// Pipeline (caller's stream):
//   nodes      offset checks, out-degrees, the row of every 1024-edge tile's
//              first edge
//   columns    range check; in-degrees as run lengths of the sorted columns
//              (a 32-bit radix sort: no atomics)
//   node sort  keys (maxdeg - deg) << idbits | id, LSD radix sort over the
//              degree bits only: the IDs are already in order, so equal
//              degrees keep increasing old ID
//   perm       perm[old] = new label; new out-degrees -> new row offsets
//   edge sort  keys perm[u] << idbits | perm[v] (sources from LDS row marks
//              per tile), LSD radix sort over 2 idbits bits: rows in new
//              order, columns ascending
//
// The radix sort is stable and 8 bits per pass: a histogram per 2048-key
// tile (digit-major, so one exclusive scan gives every tile's start in
// every digit), then each tile ranks its keys in LDS (one ballot per digit
// bit gives the lanes of a wavefront with the same digit; per-wavefront
// counts and a running cursor per digit keep tile order) and writes them out
// in digit order, so consecutive lanes store consecutive addresses.
#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

#include "pcpm_device.hpp"
#include "pcpm_internal.hpp"

namespace pcpm {
namespace {

constexpr int kRsBlock = 256;                 // threads per radix workgroup (= digits)
#ifndef PCPM_RS_PER
#define PCPM_RS_PER 8
#endif
constexpr int kRsPer = PCPM_RS_PER;           // keys per thread
constexpr int kRsTile = kRsBlock * kRsPer;    // keys per workgroup
constexpr int kRsBits = 8;
constexpr int kRsDigits = 1 << kRsBits;
constexpr int kRsWaves = kRsBlock / kWave;
static_assert(kRsBlock == kRsDigits, "one thread per digit");

// Exclusive scan of one value per thread of a 256-thread workgroup.
__device__ int32_t block256_excl_scan(int32_t v, int32_t* wtot /* kRsWaves */) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  int32_t x = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int32_t o = __shfl_up(x, off);
    if (lane >= off) x += o;
  }
  if (lane == kWave - 1) wtot[w] = x;
  __syncthreads();
  int32_t before = 0;
  for (int i = 0; i < w; ++i) before += wtot[i];
  __syncthreads();
  return before + x - v;
}

template <class K>
__global__ __launch_bounds__(kRsBlock) void k_rs_hist(const K* __restrict__ keys, int64_t L, int shift,
                                                      int64_t nblk, int32_t* __restrict__ hist) {
  __shared__ int32_t h[kRsDigits];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kRsTile + threadIdx.x;
#pragma unroll
  for (int j = 0; j < kRsPer; ++j) {
    const int64_t i = base + static_cast<int64_t>(j) * kRsBlock;
    if (i < L) atomicAdd(&h[(keys[i] >> shift) & (kRsDigits - 1)], 1);
  }
  __syncthreads();
  hist[static_cast<int64_t>(threadIdx.x) * nblk + blockIdx.x] = h[threadIdx.x];  // digit-major
}

// off: exclusive scan of the digit-major histogram (keys of smaller digits,
// then of the same digit in earlier tiles).
template <class K>
__global__ __launch_bounds__(kRsBlock) void k_rs_scatter(const K* __restrict__ in, K* __restrict__ out,
                                                         int64_t L, int shift, int64_t nblk,
                                                         const int32_t* __restrict__ off) {
  __shared__ K sk[kRsTile];                     // the tile in digit order
  __shared__ int32_t lstart[kRsDigits];         // tile-local start of each digit
  __shared__ int32_t cur[kRsDigits];            // next tile-local slot of each digit
  __shared__ int32_t cnt[kRsWaves][kRsDigits];  // keys of each digit in a wavefront's 64
  __shared__ int32_t ofs[kRsWaves][kRsDigits];  // their first slot
  __shared__ int32_t wtot[kRsWaves];
  const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid / kWave;
  const int64_t t0 = static_cast<int64_t>(blockIdx.x) * kRsTile;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  cur[tid] = 0;
#pragma unroll
  for (int i = 0; i < kRsWaves; ++i) cnt[i][tid] = 0;
  __syncthreads();
  K k[kRsPer];
#pragma unroll
  for (int j = 0; j < kRsPer; ++j) {
    const int64_t i = t0 + static_cast<int64_t>(j) * kRsBlock + tid;
    k[j] = i < L ? in[i] : K{0};
    if (i < L) atomicAdd(&cur[(k[j] >> shift) & (kRsDigits - 1)], 1);
  }
  __syncthreads();
  const int32_t start = block256_excl_scan(cur[tid], wtot);
  lstart[tid] = start;
  cur[tid] = start;
  __syncthreads();
  // round j: keys t0 + 256 j + (64 w + lane), i.e. wavefronts in tile order
  for (int j = 0; j < kRsPer; ++j) {
    const bool valid = t0 + static_cast<int64_t>(j) * kRsBlock + tid < L;
    const int d = static_cast<int>((k[j] >> shift) & (kRsDigits - 1));
    uint64_t peers = wave_ballot(valid);
#pragma unroll
    for (int b = 0; b < kRsBits; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t bb = wave_ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    if (valid && (peers & below) == 0) cnt[w][d] = __popcll(peers);
    __syncthreads();
    {
      int32_t base = cur[tid];
#pragma unroll
      for (int i = 0; i < kRsWaves; ++i) {
        ofs[i][tid] = base;
        base += cnt[i][tid];
        cnt[i][tid] = 0;
      }
      cur[tid] = base;
    }
    __syncthreads();
    if (valid) sk[ofs[w][d] + __popcll(peers & below)] = k[j];
  }
  __syncthreads();
  const int64_t nvalid = L - t0 < kRsTile ? L - t0 : kRsTile;
#pragma unroll
  for (int j = 0; j < kRsPer; ++j) {
    const int i = j * kRsBlock + tid;
    if (i < nvalid) {
      const K key = sk[i];
      const int d = static_cast<int>((key >> shift) & (kRsDigits - 1));
      out[static_cast<int64_t>(off[static_cast<int64_t>(d) * nblk + blockIdx.x]) + (i - lstart[d])] = key;
    }
  }
}

enum : int32_t { kRlErrOffsets = 1, kRlErrRange = 2 };

// Offsets, out-degrees, and the row of every tile's first edge (rows that
// contain a tile start write it; all below ceil(m / kTile) when the offsets
// are valid); tile_row[ntiles] = n - 1.
__global__ __launch_bounds__(256) void k_rl_nodes(int64_t n, int64_t m, const int32_t* __restrict__ row_off,
                                                  int32_t* __restrict__ outdeg, int32_t* __restrict__ tile_row,
                                                  int32_t* __restrict__ flags) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int32_t err = 0;
  for (int64_t u = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; u < n; u += stride) {
    const int32_t lo = row_off[u], hi = row_off[u + 1];
    if (lo < 0 || hi < lo || static_cast<int64_t>(hi) > m) {
      err = kRlErrOffsets;
      outdeg[u] = 0;
    } else {
      outdeg[u] = hi - lo;
      for (int64_t t = (static_cast<int64_t>(lo) + kTile - 1) / kTile; t * kTile < hi; ++t)
        tile_row[t] = static_cast<int32_t>(u);
    }
    if (u == n - 1) tile_row[(m + kTile - 1) / kTile] = static_cast<int32_t>(u);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (row_off[0] != 0 || static_cast<int64_t>(row_off[n]) != m))
    err = kRlErrOffsets;
  if (err) atomicOr(flags, err);
}

// Column range check; a copy of the columns as sort keys when ckeys is given.
__global__ __launch_bounds__(256) void k_rl_cols(int64_t n, int64_t m, const int32_t* __restrict__ col,
                                                 uint32_t* __restrict__ ckeys, int32_t* __restrict__ flags) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int32_t err = 0;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < m; e += stride) {
    const int32_t c = col[e];
    if (c < 0 || static_cast<int64_t>(c) >= n) err = kRlErrRange;
    if (ckeys) ckeys[e] = static_cast<uint32_t>(c);
  }
  if (err) atomicOr(flags, err);
}

// In-degrees from the sorted columns: node v's entries are one run, whose
// first and last index are stored by the entries at the run's two ends
// (rstart and rend start at 0, so a node without in-edges gets 0).
__global__ __launch_bounds__(256) void k_rl_runs(int64_t m, const uint32_t* __restrict__ sc,
                                                 int32_t* __restrict__ rstart, int32_t* __restrict__ rend) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += stride) {
    const uint32_t v = sc[i];
    if (i == 0 || sc[i - 1] != v) rstart[v] = static_cast<int32_t>(i);
    if (i == m - 1 || sc[i + 1] != v) rend[v] = static_cast<int32_t>(i + 1);
  }
}

__global__ __launch_bounds__(256) void k_rl_indeg(int64_t n, const int32_t* __restrict__ rstart,
                                                  int32_t* __restrict__ rend_indeg) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; v < n; v += stride)
    rend_indeg[v] -= rstart[v];
}

__global__ __launch_bounds__(256) void k_rl_max(int64_t n, const int32_t* __restrict__ deg, int32_t* __restrict__ mx) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  int32_t v = 0;
  for (int64_t u = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; u < n; u += stride)
    v = max(v, deg[u]);
  for (int off = kWave / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off));
  if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(mx, v);
}

__global__ __launch_bounds__(256) void k_rl_node_keys(int64_t n, const int32_t* __restrict__ deg, int32_t maxdeg,
                                                      int idbits, uint64_t* __restrict__ keys) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t u = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; u < n; u += stride)
    keys[u] = (static_cast<uint64_t>(maxdeg - deg[u]) << idbits) | static_cast<uint64_t>(u);
}

// New label i = position of the old node in the sorted keys; the new row i
// has the old node's out-degree.
__global__ __launch_bounds__(256) void k_rl_perm(int64_t n, const uint64_t* __restrict__ keys, uint64_t idmask,
                                                 const int32_t* __restrict__ outdeg, int32_t* __restrict__ perm,
                                                 int32_t* __restrict__ newdeg) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t old = static_cast<int64_t>(keys[i] & idmask);
    perm[old] = static_cast<int32_t>(i);
    newdeg[i] = outdeg[old];
  }
}

// Edge keys: one wavefront per 1024-edge tile.  The rows tile_row[t] ..
// tile_row[t + 1] mark their first edges in LDS (max over rows that share an
// offset: the non-empty one), a wavefront max-scan gives each edge its row.
constexpr int kRlEdgeBlock = 256;
__global__ __launch_bounds__(kRlEdgeBlock) void k_rl_edge_keys(int64_t m, const int32_t* __restrict__ row_off,
                                                               const int32_t* __restrict__ col,
                                                               const int32_t* __restrict__ tile_row,
                                                               const int32_t* __restrict__ perm, int idbits,
                                                               uint64_t* __restrict__ keys) {
  __shared__ int32_t marks[kRlEdgeBlock / kWave][kTile];
  const int lane = threadIdx.x & (kWave - 1);
  int32_t* mk = marks[threadIdx.x / kWave];
  const int64_t ntiles = (m + kTile - 1) / kTile;
  const int64_t nwaves = static_cast<int64_t>(gridDim.x) * blockDim.x / kWave;
  for (int64_t t = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave; t < ntiles; t += nwaves) {
    const int64_t e0 = t * kTile, e_end = min(m, e0 + kTile);
    const int32_t r0 = tile_row[t], r1 = tile_row[t + 1];
    for (int j = 0; j < kSub; ++j) mk[j * kWave + lane] = -1;
    __builtin_amdgcn_wave_barrier();
    for (int64_t u = static_cast<int64_t>(r0) + 1 + lane; u <= r1; u += kWave) {
      const int64_t lo = row_off[u];
      if (lo >= e0 && lo < e_end) atomicMax(&mk[lo - e0], static_cast<int32_t>(u));
    }
    __builtin_amdgcn_wave_barrier();
    int32_t carry = r0;
    for (int j = 0; j < kSub; ++j) {
      const int64_t e = e0 + j * kWave + lane;
      int32_t v = mk[j * kWave + lane];
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const int32_t o = __shfl_up(v, off);
        if (lane >= off) v = max(v, o);
      }
      const int32_t u = max(v, carry);
      carry = __shfl(u, kWave - 1);
      if (e < m)
        keys[e] = (static_cast<uint64_t>(perm[u]) << idbits) | static_cast<uint64_t>(perm[col[e]]);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

__global__ __launch_bounds__(256) void k_rl_cols_out(int64_t m, const uint64_t* __restrict__ keys, uint64_t idmask,
                                                     int32_t* __restrict__ col_out) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
  for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < m; e += stride)
    col_out[e] = static_cast<int32_t>(keys[e] & idmask);
}

// Device buffers of one call, freed on every return path.
struct Scratch {
  std::vector<void*> ptrs;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  pcpm_status_t get(T** p, int64_t count) {
    void* q = nullptr;
    const size_t bytes = static_cast<size_t>(count > 0 ? count : 1) * sizeof(T);
    if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return set_error(PCPM_ERR_OOM, "hipMalloc of %zu bytes failed", bytes);
    }
    ptrs.push_back(q);
    *p = static_cast<T*>(q);
    return PCPM_OK;
  }
};

unsigned grid_for(int64_t items, int64_t per_block, int64_t cap = 65536) {
  return static_cast<unsigned>(std::max<int64_t>(1, std::min<int64_t>((items + per_block - 1) / per_block, cap)));
}

// Stable LSD sort of a[0..L) by bits [lo, hi); b is the second buffer.
// *result is the buffer holding the sorted keys.
template <class K>
pcpm_status_t radix_sort(K* a, K* b, int64_t L, int lo, int hi, int32_t* hist, int32_t* tmp, hipStream_t st,
                         K** result) {
  const int64_t nblk = (L + kRsTile - 1) / kRsTile;
  for (int shift = lo; shift < hi && L > 0; shift += kRsBits) {
    PCPM_LAUNCH("pcpm_relabel_sort", k_rs_hist<K>, dim3(static_cast<unsigned>(nblk)), dim3(kRsBlock), 0, st, a, L,
                shift, nblk, hist);
    PCPM_TRY(scan_excl_i32(hist, hist, kRsDigits * nblk, tmp, st));
    PCPM_LAUNCH("pcpm_relabel_sort", k_rs_scatter<K>, dim3(static_cast<unsigned>(nblk)), dim3(kRsBlock), 0, st, a, b,
                L, shift, nblk, hist);
    std::swap(a, b);
  }
  *result = a;
  return PCPM_OK;
}

bool on_device(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

}  // namespace
}  // namespace pcpm

extern "C" pcpm_status_t pcpm_relabel(int64_t n, int64_t m, const int32_t* row_off, const int32_t* col, int32_t key,
                                      int32_t* perm, int32_t* row_off_out, int32_t* col_out, void* stream) {
  using namespace pcpm;
  if (n < 1 || m < 0) return set_error(PCPM_ERR_INVALID_ARG, "n must be >= 1 and m >= 0");
  if (n >= (int64_t{1} << 31) || m >= (int64_t{1} << 31))
    return set_error(PCPM_ERR_OVERFLOW, "n and m must be below 2^31");
  if (key != 0 && key != 1) return set_error(PCPM_ERR_INVALID_ARG, "key must be 0 (in-degree) or 1 (out-degree)");
  if (!row_off || !perm || !row_off_out || (m > 0 && (!col || !col_out)))
    return set_error(PCPM_ERR_INVALID_ARG, "NULL array");
  if (!on_device(row_off) || !on_device(perm) || !on_device(row_off_out) ||
      (m > 0 && (!on_device(col) || !on_device(col_out))))
    return set_error(PCPM_ERR_INVALID_ARG, "arrays must be device pointers");
  {
    // outputs are written while inputs are still read: no overlap
    auto span = [](const void* p, int64_t bytes) {
      const uintptr_t a = reinterpret_cast<uintptr_t>(p);
      return std::make_pair(a, a + static_cast<uintptr_t>(bytes));
    };
    const std::pair<uintptr_t, uintptr_t> ins[2] = {span(row_off, (n + 1) * 4), span(col, m * 4)};
    const std::pair<uintptr_t, uintptr_t> outs[3] = {span(perm, n * 4), span(row_off_out, (n + 1) * 4),
                                                     span(col_out, m * 4)};
    for (const auto& o : outs) {
      for (const auto& i : ins)
        if (o.first < i.second && i.first < o.second) return set_error(PCPM_ERR_INVALID_ARG, "outputs overlap inputs");
      for (const auto& o2 : outs)
        if (&o2 != &o && o.first < o2.second && o2.first < o.second)
          return set_error(PCPM_ERR_INVALID_ARG, "outputs overlap each other");
    }
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  Scratch sc;
  int idbits = 1;
  while ((int64_t{1} << idbits) < n) ++idbits;
  const uint64_t idmask = (uint64_t{1} << idbits) - 1;
  const int64_t ntiles = (m + kTile - 1) / kTile;
  const int64_t nk = std::max(n, m);
  const int64_t nh = kRsDigits * ((nk + kRsTile - 1) / kRsTile) + 1;
  int32_t *outdeg, *indeg = nullptr, *rstart = nullptr, *tile_row, *flags, *newdeg, *tmp, *hist;
  uint64_t *ka, *kb, *sorted;
  PCPM_TRY(sc.get(&outdeg, n));
  PCPM_TRY(sc.get(&tile_row, ntiles + 1));
  PCPM_TRY(sc.get(&flags, 2));
  PCPM_TRY(sc.get(&newdeg, n));
  PCPM_TRY(sc.get(&ka, nk));
  PCPM_TRY(sc.get(&kb, nk));
  PCPM_TRY(sc.get(&hist, nh));
  PCPM_TRY(sc.get(&tmp, scan_tmp_ints(std::max(nh, n))));
  if (key == 0) {
    PCPM_TRY(sc.get(&indeg, n));
    PCPM_TRY(sc.get(&rstart, n));
  }
  // in-degrees: the columns (as 32-bit keys in the first key buffer) sorted,
  // then each node's run length
  uint32_t* ca = key == 0 && m > 0 ? reinterpret_cast<uint32_t*>(ka) : nullptr;
  uint32_t* cb = reinterpret_cast<uint32_t*>(kb);
  PCPM_TRY_HIP(hipMemsetAsync(flags, 0, 8, st));
  PCPM_TRY_HIP(hipMemsetAsync(tile_row, 0, static_cast<size_t>(ntiles + 1) * 4, st));
  PCPM_LAUNCH("pcpm_relabel_nodes", k_rl_nodes, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, n, m, row_off,
              outdeg, tile_row, flags);
  if (m > 0)
    PCPM_LAUNCH("pcpm_relabel_nodes", k_rl_cols, dim3(grid_for(m, 256 * 16, 8192)), dim3(256), 0, st, n, m, col, ca,
                flags);
  int32_t hf[2] = {0, 0};
  PCPM_TRY_HIP(hipMemcpyAsync(hf, flags, 8, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  if (hf[0] & kRlErrOffsets) return set_error(PCPM_ERR_GRAPH, "invalid CSR: row offsets");
  if (hf[0] & kRlErrRange) return set_error(PCPM_ERR_GRAPH, "invalid CSR: column index outside [0, n)");
  if (indeg) {
    PCPM_TRY_HIP(hipMemsetAsync(indeg, 0, static_cast<size_t>(n) * 4, st));
    PCPM_TRY_HIP(hipMemsetAsync(rstart, 0, static_cast<size_t>(n) * 4, st));
    if (m > 0) {
      uint32_t* sc_sorted = nullptr;
      PCPM_TRY(radix_sort<uint32_t>(ca, cb, m, 0, idbits, hist, tmp, st, &sc_sorted));
      PCPM_LAUNCH("pcpm_relabel_nodes", k_rl_runs, dim3(grid_for(m, 256 * 16, 8192)), dim3(256), 0, st, m, sc_sorted,
                  rstart, indeg);
      PCPM_LAUNCH("pcpm_relabel_nodes", k_rl_indeg, dim3(grid_for(n, 256 * 4, 8192)), dim3(256), 0, st, n, rstart,
                  indeg);
    }
  }
  const int32_t* deg = indeg ? indeg : outdeg;
  PCPM_LAUNCH("pcpm_relabel_nodes", k_rl_max, dim3(grid_for(n, 256 * 16, 4096)), dim3(256), 0, st, n, deg,
              flags + 1);
  PCPM_TRY_HIP(hipMemcpyAsync(hf, flags, 8, hipMemcpyDeviceToHost, st));
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  const int32_t maxdeg = hf[1];
  int degbits = 0;
  while ((int64_t{1} << degbits) <= maxdeg) ++degbits;

  // nodes: largest degree first, equal degrees in old-ID order
  PCPM_LAUNCH("pcpm_relabel_nodes", k_rl_node_keys, dim3(grid_for(n, 256)), dim3(256), 0, st, n, deg, maxdeg, idbits,
              ka);
  PCPM_TRY(radix_sort(ka, kb, n, idbits, idbits + degbits, hist, tmp, st, &sorted));
  PCPM_LAUNCH("pcpm_relabel_nodes", k_rl_perm, dim3(grid_for(n, 256)), dim3(256), 0, st, n, sorted, idmask, outdeg,
              perm, newdeg);
  PCPM_TRY(scan_excl_i32(newdeg, row_off_out, n, tmp, st));
  if (m > 0) {
    // edges: (new source, new destination) ascending
    PCPM_LAUNCH("pcpm_relabel_edges", k_rl_edge_keys, dim3(grid_for(ntiles, kRlEdgeBlock / kWave)),
                dim3(kRlEdgeBlock), 0, st, m, row_off, col, tile_row, perm, idbits, ka);
    PCPM_TRY(radix_sort(ka, kb, m, 0, 2 * idbits, hist, tmp, st, &sorted));
    PCPM_LAUNCH("pcpm_relabel_edges", k_rl_cols_out, dim3(grid_for(m, 256 * 16)), dim3(256), 0, st, m, sorted, idmask,
                col_out);
  }
  PCPM_TRY_HIP(hipStreamSynchronize(st));
  return PCPM_OK;
}
