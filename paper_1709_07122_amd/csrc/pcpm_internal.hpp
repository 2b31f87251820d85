// Internal declarations of libpcpm (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "pcpm.h"

namespace pcpm {

// Destination IDs and PNG source IDs carry a flag in their top bit: the first
// ID of a message (Sec. 3.2) and the first node of a (source, destination)
// partition segment respectively.
constexpr uint32_t kFlag = 0x80000000u;
constexpr uint32_t kIdMask = 0x7FFFFFFFu;
// Destination IDs and PNG source IDs are stored partition-local in 16 bits:
// v - p'q or u - pq (< q <= 2^14), with bit 15 marking the first ID of each
// message or the first node of each segment.
constexpr uint32_t kDidFlag = 0x8000u;
// Bit 14 of a destination ID marks the first ID of each (destination bin,
// source pair) segment: the gather finds an update's position in the
// PNG-ordered update array from its message index and its segment.
constexpr uint32_t kSegFlag = 0x4000u;

// Flag-decoding tile: 16 sub-blocks of one wavefront (64 lanes) each.  The
// running flag count before every tile is stored, so any wavefront can decode
// any tile on its own.
constexpr int kWave = 64;
constexpr int kSub = 16;
constexpr int kTile = kWave * kSub;

constexpr int kMaxHist = 100000;   // residual history kept on the device
// Updates go in PNG order when the average non-empty (pair, bin) segment is
// shorter than this many updates (measured on MI355X with the non-temporal
// PNG-order stores: RMAT-24 with random labels, 333 per segment, ran 1.5%
// faster in PNG order; with in-degree labels, 399 per segment, 7% slower).
constexpr int64_t kPngOrderRun = 360;
constexpr int kMaxParts = 16384;   // k limit (LDS cursors of the fill kernel)
constexpr int kMinLog2 = 1;
constexpr int kMaxLog2 = 14;       // 16384 * 8 B = 128 KB fixed-point slice in LDS
static_assert(kMaxLog2 <= 14, "partition-local destination IDs use 14 bits (bits 14, 15 are flags)");
#ifndef PCPM_SCATTER_BLOCK
#define PCPM_SCATTER_BLOCK 1024
#endif
#ifndef PCPM_GATHER_BLOCK
#define PCPM_GATHER_BLOCK 1024
#endif
constexpr int kScatterBlock = PCPM_SCATTER_BLOCK;  // threads per scatter workgroup
constexpr int kGatherBlock = PCPM_GATHER_BLOCK;    // threads per gather / merge workgroup

// MI355X has 8 XCDs (32 CUs and one L2 each), and the workgroups of a launch
// are dealt to them in turn: workgroup b runs on XCD b % 8.  xcd_block(b, nb)
// renumbers the workgroups so that each XCD takes one contiguous range of
// [0, nb) (a bijection): work items that are neighbours in memory then run
// together on one XCD and share its L2.
constexpr unsigned kXcds = 8;
__host__ __device__ inline unsigned xcd_block(unsigned b, unsigned nb) {
  const unsigned x = b % kXcds, j = b / kXcds;
  const unsigned per = nb / kXcds, rem = nb % kXcds;
  return x * per + (x < rem ? x : rem) + j;
}

// Device control block of one handle (one solve at a time).
struct Ctl {
  double res;       // largest residual over groups, last iteration
  double res_prev;  // the same one iteration before
  double tol;       // stop threshold (<= 0: never)
  double d;         // damping factor
  int32_t iter;     // iterations completed
  int32_t done;     // every group converged, or a non-finite value appeared
  int32_t nonfinite;
  int32_t fx_shift; // gather sums are kept as integers in units of 2^-fx_shift
  int32_t ngroups;
  int32_t fx_cap;   // largest fx_shift the start vector's mass allows
};

// Per-group state: a group is one graph of a multi-graph handle (the whole
// graph for a single one).
struct GCtl {
  double base;      // (1-d)/n_g + d*D_g/n_g: jump plus dangling share per node
  double dmass;     // dangling mass D_g of the current input
  double res;       // residual of the group's last iteration
  double inv_n;     // 1/n_g
  int32_t iter;     // iterations the group has run
  int32_t done;     // residual fell below tol: the group keeps its iterate
};

// Per-vector state of batched personalised PageRank.
struct VCtl {
  double coef;      // ((1-d) + d*D_j)/|S_j|: jump plus dangling share of each seed node
  double inv_s;     // 1/|S_j|
  double dmass;     // dangling mass D_j of the current iterate
  double res;       // residual of the vector's last iteration
  int32_t iter;     // iterations the vector has run
  int32_t done;     // residual fell below tol: the vector keeps its iterate
  int32_t vec;      // vector of the batch in this slot, -1 = idle
  int32_t pad;
};

// Queue of the batch's vectors over the kt slots of a tile: a slot whose
// vector has finished takes the next one.  old_vec / new_vec describe the
// refill planned by the last iteration (-1 = none).
struct PprQueue {
  int32_t head;       // next vector to start
  int32_t k;          // vectors in the batch
  int32_t max_iters;  // iteration limit per vector
  int32_t pending;    // a refill is planned
  int32_t old_vec[16];
  int32_t new_vec[16];
};

// Device state of a persistent solve (one cooperative launch runs all of a
// solve's iterations): a grid barrier, work counters, and the flag of a
// bounded wait that gave up.  On cache lines of its own, away from the
// control block that every workgroup reads.
struct alignas(256) PSync {
  uint32_t bar_count;       // workgroups arrived at the current barrier
  uint32_t bar_gen;         // barriers completed
  int32_t err;              // a wait ran past its spin limit
  int32_t applied;          // apply units finished, counted over the whole solve
  int32_t ga_next;          // next gather item of this iteration
  int32_t mg_next;          // next merge unit of this iteration
  int32_t sc_next[kXcds];   // next scatter item of each XCD's range
};

// A unit of scatter or gather work: a contiguous range [lo, hi) of PNG edges
// (scatter, part = source partition) or of destination IDs (gather, part =
// destination partition).  aux: gather partial slot (-1 = whole bin).
struct Item {
  int32_t part, lo, hi, aux;
};

// Merge work: nodes [node_lo, node_lo + 256) of a destination bin split over
// `count` gather items whose partial sums sit in consecutive partial slots
// starting at `first`.
struct Merge {
  int32_t part, first, count, node_lo;
};

// Arguments of the persistent kernels (passed by value).
struct PersistArgs {
  Ctl* ctl;
  GCtl* gctl;
  PSync* ps;
  int32_t* bin_done;
  int64_t n, k;
  int32_t s, n_sc, n_ga, n_mg, n_apply, max_iters;
  uint32_t spin_limit;
  const Item* sc_items;
  const Item* ga_items;
  const Merge* mg_items;
  const int32_t* outdeg;
  const uint16_t* png_src;
  const int32_t* png_blk;
  const int32_t* seg_delta;
  float* upd;
  int64_t spare;
  const uint16_t* did;
  const int32_t* did_blk;
  const int32_t* did_sblk;
  const uint32_t* dmask;
  int64_t* partial;
  double* red;
  const int32_t* part_group;
  const int32_t* part_valid;
  const int32_t* group_slots;
  double* hist;
  float* x0;  // input of even iterations (the caller's output vector)
  float* x1;  // input of odd iterations
};

struct PprPersistArgs {
  Ctl* ctl;
  VCtl* vctl;
  PSync* ps;
  int32_t* bin_done;
  PprQueue* queue;
  int64_t n, k, max_loops, spare;
  int32_t s, n_sc, n_ga, n_mg, n_apply, kvec, refill;
  uint32_t spin_limit;
  double d;
  const Item* sc_items;
  const Item* ga_items;
  const Merge* mg_items;
  const int32_t* outdeg;
  const uint16_t* png_src;
  const int32_t* png_blk;
  const int32_t* seg_delta;
  float* upd;
  const uint16_t* did;
  const int32_t* did_blk;
  const int32_t* did_sblk;
  const uint32_t* dmask;
  uint32_t* seedmask;
  int64_t* partial;
  double* red;
  double* hist;
  int32_t* out_it;
  double* out_res;
  int32_t* out_conv;
  float* pr_out;
  const int32_t* seeds;
  const int32_t* seed_off;
  float* x0;  // iterate tile read by even iterations
  float* x1;
};

// ---- errors ----------------------------------------------------------------
pcpm_status_t set_error(pcpm_status_t st, const char* fmt, ...);

#define PCPM_TRY_HIP(expr)                                                              \
  do {                                                                                  \
    hipError_t _e = (expr);                                                             \
    if (_e != hipSuccess)                                                               \
      return ::pcpm::set_error(_e == hipErrorOutOfMemory ? PCPM_ERR_OOM : PCPM_ERR_DEVICE, \
                               "%s failed: %s", #expr, hipGetErrorString(_e));          \
  } while (0)

#define PCPM_TRY(expr)                          \
  do {                                          \
    pcpm_status_t _s = (expr);                  \
    if (_s != PCPM_OK) return _s;               \
  } while (0)

// ---- per-kernel timing -------------------------------------------------------
struct TimerScope {
  TimerScope(const char* name, hipStream_t s);
  ~TimerScope();
  const char* name;
  hipStream_t stream;
  hipEvent_t start = nullptr;
};

// Position in the timing record (the number of launches recorded so far),
// and removal of the records from a position on: a solve drops the launches
// of iterations it queued past convergence (they return at once and would
// dilute the per-kernel averages).  Assumes one thread records at a time.
size_t timing_mark();
void timing_discard_from(size_t pos);

// Launch with optional event timing and a launch-error check.
#define PCPM_LAUNCH(name, kernel, grid, block, shmem, stream, ...)                     \
  do {                                                                                  \
    ::pcpm::TimerScope _ts(name, stream);                                               \
    hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__);                \
    hipError_t _e = hipGetLastError();                                                  \
    if (_e != hipSuccess)                                                               \
      return ::pcpm::set_error(PCPM_ERR_DEVICE, "launch of %s failed: %s", name,       \
                               hipGetErrorString(_e));                                  \
  } while (0)

// ---- wave-level helpers (device) -------------------------------------------------
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __ballot(p); }

// Storage order of the 16-bit tile entries (destination IDs, PNG source IDs):
// inside each 128-entry block, entries i and 64 + i share one 32-bit word
// (low and high half).  A wavefront reads two 64-entry sub-blocks with one
// 4-byte load per lane and still sees 64 consecutive entries per sub-block;
// on MI355X 2-byte loads move about half the bytes per instruction.
__host__ __device__ inline int64_t tile_pos(int64_t e) {
  return (e & ~int64_t{127}) | ((e & 63) << 1) | ((e >> 6) & 1);
}
constexpr int kPairs = kSub / 2;

// This lane's words of one tile.
__device__ __forceinline__ void load_tile_words(const uint16_t* tile, int lane, uint32_t (&w)[kPairs]) {
  const uint32_t* p = reinterpret_cast<const uint32_t*>(tile);
#pragma unroll
  for (int j = 0; j < kPairs; ++j) w[j] = p[j * kWave + lane];
}

// Update slots of one tile of destination IDs (Alg. 5): an ID's message index
// in bin order is the number of message flags so far (inclusive) minus one;
// blk = message flags before the tile.  With updates in PNG order the slot
// adds the delta of the ID's (bin, source pair) segment, the segment index
// counting segment flags the same way (sblk = segment flags before the
// tile).  dl holds, in lane i, the delta of segment max(sblk - 1, 0) + i,
// loaded ahead of the tile; a tile that reaches past those 64 segments reads
// its deltas from seg_delta instead.
template <bool kPng>
__device__ __forceinline__ void tile_slots(const uint32_t (&x)[kSub], int32_t blk, int32_t sblk, int32_t dl,
                                           const int32_t* __restrict__ seg_delta, int32_t (&slot)[kSub]) {
  int32_t run = blk - 1, srun = sblk - 1;
  int32_t seg[kSub];
#pragma unroll
  for (int j = 0; j < kSub; ++j) {
    const bool f = (x[j] & kDidFlag) != 0u;
    const uint64_t bal = wave_ballot(f);
    slot[j] = run + lanes_below(bal) + (f ? 1 : 0);
    run += __popcll(bal);
    if constexpr (kPng) {
      const bool sf = (x[j] & kSegFlag) != 0u;
      const uint64_t sbal = wave_ballot(sf);
      seg[j] = srun + lanes_below(sbal) + (sf ? 1 : 0);
      srun += __popcll(sbal);
    }
  }
  if constexpr (kPng) {
    const int32_t sbase = max(sblk - 1, 0);
    if (srun - sbase < kWave) {
#pragma unroll
      for (int j = 0; j < kSub; ++j) slot[j] += __builtin_amdgcn_ds_bpermute((seg[j] - sbase) << 2, dl);
    } else {
#pragma unroll
      for (int j = 0; j < kSub; ++j) slot[j] += seg_delta[seg[j]];
    }
  }
}

// Deltas of the 64 segments from max(sblk - 1, 0) on, one per lane (the
// array is padded by kWave entries past its last segment).
__device__ __forceinline__ int32_t tile_deltas(const int32_t* __restrict__ seg_delta, int32_t sblk, int lane) {
  return seg_delta[max(sblk - 1, 0) + lane];
}

// Flag counts before tile t, by a vector load that keeps its place among the
// wavefront's other loads: lane 0 gets blk[t], lane 1 sblk[t] (PNG order) or
// blk[t + 1] (bin order, where sblk is NULL).  A scalar load would instead
// make every later wait on LDS results wait for it too.
__device__ __forceinline__ int32_t load_counts(const int32_t* __restrict__ blk, const int32_t* __restrict__ sblk,
                                               int64_t t, int lane) {
  const int32_t* p = sblk ? ((lane & 1) ? sblk + t : blk + t) : blk + t + (lane & 1);
  return *p;
}

// Entry 64j + lane of the tile, j = 0..kSub-1.
__device__ __forceinline__ void unpack_tile(const uint32_t (&w)[kPairs], uint32_t (&x)[kSub]) {
#pragma unroll
  for (int j = 0; j < kSub; ++j) x[j] = (j & 1) ? (w[j >> 1] >> 16) : (w[j >> 1] & 0xFFFFu);
}


}  // namespace pcpm

// ---- the handle ------------------------------------------------------------------
struct pcpm_png {
  int64_t n = 0, m = 0, q = 0, k = 0, eprime = 0, nseg = 0, n_dangling = 0;
  // rows and columns (n for a graph); a matrix handle (generic SpMV, Sec.
  // 3.5: num_cols != rows or diagonal entries) has n = max(rows, cols) node
  // slots, its scatter reading rows and its gather writing columns
  int64_t n_rows = 0, n_cols = 0;
  bool matrix = false;
  int part_log2 = 0;
  int device = 0;
  double build_ms = 0.0;
  int64_t device_bytes = 0;

  // per node
  int32_t* outdeg = nullptr;    // n
  uint32_t* dmask = nullptr;    // ceil(n/32) dangling bitmask

  // scatter side: PNG in (source pair, destination partition, source partition, node) order
  uint16_t* png_src = nullptr;  // ceil(E'/kTile)*kTile, in partition-pair order: u - 2Pq, bit 15 = pair segment start
  int32_t* png_blk = nullptr;   // bin order: pair-segment flags before each PNG tile, ceil(E'/kTile)+1
  int32_t* seg_delta = nullptr; // nseg + kWave (padding), one per non-empty (pair, bin) segment.  Bin order: update slot minus PNG
                                // position, segments in (pair, bin) order.  PNG order: PNG position minus
                                // message index, segments in (bin, pair) order
  bool png_order = false;       // updates stored in PNG order (else bin order)
  int32_t* png_base = nullptr;  // k+1: first PNG edge of each source partition
  int32_t* png_off = nullptr;   // k*(k+1): partition-local PNG offsets
  int32_t* wo = nullptr;        // k*k: write offsets (Sec. 3.1)
  int32_t* upd_start = nullptr; // k+1: first update slot of each bin

  // gather side: destination-ID bins
  uint16_t* did = nullptr;      // ceil(m/kTile)*kTile: v - p'q, bit 15 = first of message, bit 14 = first of segment
  int32_t* did_sblk = nullptr;  // segment flags before each tile, ceil(m/kTile)+1
  float* wbin = nullptr;        // m edge weights in bin order (weighted handles only)
  // weight statistics of the SpMV scale, as bit patterns of non-negative
  // doubles: max over v of sum_{u->v} |w(u,v)|, max |w| (1 if unweighted, 0
  // without edges), then the count of non-finite weights; computed at build
  // for weighted handles, on the first pcpm_spmv for unweighted ones
  unsigned long long* wstats = nullptr;
  bool wstats_ready = false;
  float* spmv_blockmax = nullptr;  // per-block max |x| of pcpm_spmv
  int32_t* did_blk = nullptr;   // flags before each tile, ceil(m/kTile)+1
  int32_t* did_start = nullptr; // k+1
  float* upd = nullptr;         // E'+1: updates in bin or PNG order (rewritten every iteration) + spare slot

  // work lists
  pcpm::Item* sc_items = nullptr;
  pcpm::Item* ga_items = nullptr;
  pcpm::Merge* mg_items = nullptr;
  int32_t n_sc = 0, n_ga = 0, n_mg = 0, n_split_slots = 0, n_split_bins = 0;
  int32_t scatter_order = 0;  // 0: source-partition order per XCD, 1: largest first
  int64_t* partial = nullptr;   // n_split_slots * q fixed-point partial sums

  // groups (graphs of a multi-graph handle)
  int32_t ngroups = 1;
  int32_t* part_group = nullptr;  // k: group of each partition
  int32_t* part_valid = nullptr;  // k: real (non-padding) nodes of each partition
  int32_t* group_slots = nullptr; // 2*(G+1): first partition and first merge unit of each group
  pcpm::GCtl* gctl = nullptr;     // G
  pcpm::GCtl* gctl_host = nullptr;  // pinned mirror
  std::vector<int64_t> group_off, group_n;  // host copies

  // persistent solves: grid barrier and work counters, finished split-bin
  // items per bin (counted over a solve), workgroups of the cooperative
  // launch (0: not possible on this device), launch mode (pcpm_set_launch)
  pcpm::PSync* psync = nullptr;
  pcpm::PSync* psync_host = nullptr;  // pinned mirror
  int32_t* bin_done = nullptr;    // k
  int32_t persist_grid = -1;      // -1: not yet queried
  int32_t launch_mode = 0;
  uint32_t spin_limit = 1u << 22; // polls before a device-side wait gives up

  // reductions and control
  double* red = nullptr;        // 3*(k + n_mg): (residual, dangling, -) partial sums per apply unit
  double* red_start = nullptr;  // 4*k: (non-finite count, dangling, L1 mass) of the start vector per partition,
                                // then the largest |value| per partition
  double* hist = nullptr;       // kMaxHist residuals (largest over groups)
  pcpm::Ctl* ctl = nullptr;
  pcpm::Ctl* ctl_host = nullptr;  // pinned mirrors: two slots, [0] for single reads
  hipEvent_t ctl_ev[2] = {nullptr, nullptr};  // completion of the copy into each slot
  float* tmp_pr = nullptr;      // n: second rank buffer

  // batched personalised PageRank working set (grown by pcpm_ppr_batch)
  int32_t ppr_kt = 0;
  float* ppr_x[2] = {nullptr, nullptr};  // n * kt, vector-minor
  float* ppr_upd = nullptr;              // (E'+1) * kt
  int64_t* ppr_partial = nullptr;        // n_split_slots * q * kt
  double* ppr_red = nullptr;             // (k + n_mg) * kt * 2
  pcpm::VCtl* ppr_vctl = nullptr;        // kt
  pcpm::VCtl* ppr_vctl_host = nullptr;   // pinned mirror (64 entries)
  uint32_t* ppr_mask = nullptr;          // n: seed bits of the tile's vectors
  int32_t* ppr_seeds = nullptr;
  int64_t ppr_seed_cap = 0;
  int32_t* ppr_seed_off = nullptr;
  int64_t ppr_off_cap = 0;
  pcpm::PprQueue* ppr_queue = nullptr;
  int32_t* ppr_out_it = nullptr;         // per vector of the batch: iterations,
  double* ppr_out_res = nullptr;         // last residual
  int32_t* ppr_out_conv = nullptr;       // and whether it fell below tol
  int64_t ppr_vec_cap = 0;

  // warm start: in-degrees (computed once per handle) and two rank vectors
  // for the first iterate from the uniform start
  float2* ws_sfeat = nullptr;            // n: log1p(in-degree), log1p(out-degree)
  float* ws_x = nullptr;                 // 2n
  double ws_indeg_ms = 0.0;

  // autotuned builds (part_log2 = 0): the measurements and the chosen entry
  std::vector<pcpm_tune_entry_t> tune_table;
  int32_t tune_best = -1;
  int32_t tune_cached = 0;

  std::vector<std::pair<void*, size_t>> allocations;
};

namespace pcpm {
// Device allocation tracked by the handle.
template <class T>
pcpm_status_t dalloc(pcpm_png* g, T** p, int64_t count) {
  size_t bytes = static_cast<size_t>(count > 0 ? count : 1) * sizeof(T);
  void* ptr = nullptr;
  hipError_t e = hipMalloc(&ptr, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_error(PCPM_ERR_OOM, "hipMalloc of %zu bytes failed: %s", bytes,
                     hipGetErrorString(e));
  }
  g->allocations.emplace_back(ptr, bytes);
  g->device_bytes += static_cast<int64_t>(bytes);
  *p = static_cast<T*>(ptr);
  return PCPM_OK;
}

// Free one tracked allocation early (build-only buffers).
void dfree(pcpm_png* g, void* p);
void free_handle(pcpm_png* g);
pcpm_status_t set_lds_limits();
// Exclusive scan of L int32 values into out[0..L] (out[L] = total) on st;
// tmp holds scan_tmp_ints(L) ints (pcpm_build.hip).
int64_t scan_tmp_ints(int64_t L);
// Queue the weight statistics into g->wstats on st (pcpm_build.hip).
pcpm_status_t weight_stats(pcpm_png* g, hipStream_t st);
pcpm_status_t scan_excl_i32(const int32_t* in, int32_t* out, int64_t L, int32_t* tmp, hipStream_t st);

// Iterations 0 .. up to max_iters - 1 of a solve whose kernels keep the
// device control block g->ctl and return at once once it says done.  They go
// out in batches, each followed by a copy of the control block into one of
// the two pinned slots of g->ctl_host and an event; the host waits for the
// older of the two batches in flight and sizes the next one from the
// residual decay it shows (tol > 0), counting the iterations already queued,
// so the device always has work queued while the host decides.  step(it)
// queues iteration it.  *last receives the last control block read: the
// final one once it says done, or after max_iters iterations.
template <class Step>
pcpm_status_t pipelined_iterations(pcpm_png* g, double tol, int64_t max_iters, hipStream_t st, Step step,
                                   Ctl* last) {
  int64_t launched = 0;
  int pending[2] = {-1, -1};  // FIFO of slots whose copy is in flight
  int npend = 0;
  std::vector<size_t> marks;  // timing-record position at the start of each iteration
  auto queue = [&](int64_t count) -> pcpm_status_t {
    const int slot = npend == 0 ? 0 : 1 - pending[npend - 1];
    for (int64_t i = 0; i < count; ++i) {
      marks.push_back(timing_mark());
      PCPM_TRY(step(launched + i));
    }
    launched += count;
    PCPM_TRY_HIP(hipMemcpyAsync(&g->ctl_host[slot], g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    PCPM_TRY_HIP(hipEventRecord(g->ctl_ev[slot], st));
    pending[npend++] = slot;
    return PCPM_OK;
  };
  const int64_t batch0 = tol > 0.0 ? 4 : 64;
  PCPM_TRY(queue(std::min(batch0, max_iters)));
  if (launched < max_iters) PCPM_TRY(queue(std::min(batch0, max_iters - launched)));
  for (;;) {
    const int slot = pending[0];
    PCPM_TRY_HIP(hipEventSynchronize(g->ctl_ev[slot]));
    *last = g->ctl_host[slot];
    pending[0] = pending[1];
    --npend;
    if (last->done) {  // what is still in flight returns at once
      if (last->iter >= 0 && static_cast<size_t>(last->iter) < marks.size()) timing_discard_from(marks[last->iter]);
      return PCPM_OK;
    }
    if (launched >= max_iters) {
      if (npend == 0) return PCPM_OK;
      continue;
    }
    int64_t want = 64;
    if (tol > 0.0) {
      const double res = last->res, prev = last->res_prev;
      double rho = (prev > 0.0 && res > 0.0) ? res / prev : 0.5;
      rho = std::min(std::max(rho, 0.05), 0.995);
      const double est = res > 0.0 ? std::ceil(std::log(tol / res) / std::log(rho)) : 1.0;
      const double ahead = static_cast<double>(launched - last->iter);  // queued behind this copy
      want = static_cast<int64_t>(std::min(std::max(est - ahead, 1.0), 16.0));
    }
    PCPM_TRY(queue(std::min(want, max_iters - launched)));
  }
}
}  // namespace pcpm
