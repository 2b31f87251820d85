// One PCPM PageRank iteration on the GPU: scatter (Alg. 3 over the PNG),
// gather (Alg. 5, branch-free) with the apply of Alg. 2 fused into its
// epilogue, and an FP64 reduction of the L1 residual and the dangling mass.
//
// Per iteration, on the caller's stream:
//   k_scatter   one workgroup per scatter item (a range of one source
//               partition's PNG edges): the partition's scaled ranks
//               PR(u)/outdeg(u) are staged in LDS, PNG edges are streamed
//               and each writes its update to its bin slot.
//   k_gather    one workgroup per gather item (a range of one destination
//               bin): destination IDs and updates are streamed, the update of
//               an ID is found from the running count of message flags, and
//               sums build up in an LDS slice of the destination partition.
//               A whole bin is applied in place; a split bin stores its
//               partial slice for k_merge.
//   k_merge     applies split bins, adding their partial slices in order.
//   k_finalize  one workgroup: residual and next dangling mass in FP64, in a
//               fixed order; sets the convergence flag that makes the kernels
//               of later iterations return at once.
#include <algorithm>

#include "pcpm_internal.hpp"

namespace pcpm {

// Sum two FP64 values over the workgroup; the result is valid in thread 0.
template <int BS>
__device__ __forceinline__ void block_sum2(double& a, double& b) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  __shared__ double sh[2 * (BS / kWave)];
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sh[2 * w] = a;
    sh[2 * w + 1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = 0.0;
    b = 0.0;
    for (int i = 0; i < BS / kWave; ++i) {
      a += sh[2 * i];
      b += sh[2 * i + 1];
    }
  }
}

// Apply (Alg. 2) for the nodes v0 .. v0+qn-1 of one destination partition:
//   x_new(v) = d * acc(v) + base,  base = (1-d)/n + d*D/n
// plus this partition's share of sum |x_new - x_old| and of the next
// dangling mass, both FP64.
template <int BS, class AccFn>
__device__ __forceinline__ void apply_partition(const Ctl* __restrict__ ctl, int64_t v0, int qn, AccFn acc,
                                                const float* __restrict__ pr_in, float* __restrict__ pr_out,
                                                const uint32_t* __restrict__ dmask, double* __restrict__ red_slot) {
  const double base = ctl->base;
  const double d = ctl->d;
  double r = 0.0, dm = 0.0;
  for (int i = threadIdx.x; i < qn; i += BS) {
    const int64_t v = v0 + i;
    const float xn = static_cast<float>(fma(d, static_cast<double>(acc(i)), base));
    const float xo = pr_in[v];
    r += fabs(static_cast<double>(xn) - static_cast<double>(xo));
    if ((dmask[v >> 5] >> (v & 31)) & 1u) dm += static_cast<double>(xn);
    pr_out[v] = xn;
  }
  block_sum2<BS>(r, dm);
  if (threadIdx.x == 0) {
    red_slot[0] = r;
    red_slot[1] = dm;
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_scatter(const Ctl* __restrict__ ctl, int64_t n, int s,
                                                const Item* __restrict__ items, const float* __restrict__ pr,
                                                const int32_t* __restrict__ outdeg,
                                                const uint32_t* __restrict__ png_src,
                                                const int32_t* __restrict__ png_blk,
                                                const int32_t* __restrict__ seg_delta, float* __restrict__ upd) {
  if (ctl->done) return;
  extern __shared__ float spr[];
  const Item it = items[blockIdx.x];
  const int64_t v0 = static_cast<int64_t>(it.part) << s;
  const int qn = static_cast<int>(min(int64_t{1} << s, n - v0));
  for (int i = threadIdx.x; i < qn; i += BS) {
    const int od = outdeg[v0 + i];
    spr[i] = od > 0 ? pr[v0 + i] / static_cast<float>(od) : 0.0f;
  }
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t lo = it.lo, hi = it.hi;
  for (int64_t t = lo / kTile + threadIdx.x / kWave; t * kTile < hi; t += BS / kWave) {
    const int64_t tb = t * kTile;
    uint32_t x[kSub];
#pragma unroll
    for (int j = 0; j < kSub; ++j) x[j] = png_src[tb + j * kWave + lane];
    int32_t run = png_blk[t];
    int32_t seg[kSub];
#pragma unroll
    for (int j = 0; j < kSub; ++j) {
      const uint32_t f = x[j] >> 31;
      const uint64_t bal = wave_ballot(f != 0);
      seg[j] = run + lanes_below(bal) + static_cast<int32_t>(f) - 1;
      run += __popcll(bal);
    }
#pragma unroll
    for (int j = 0; j < kSub; ++j) {
      const int64_t e = tb + j * kWave + lane;
      if (e >= lo && e < hi) {
        const int64_t slot = e + seg_delta[seg[j]];
        upd[slot] = spr[static_cast<int64_t>(x[j] & kIdMask) - v0];
      }
    }
  }
}

template <int BS>
__global__ __launch_bounds__(BS) void k_gather(const Ctl* __restrict__ ctl, int64_t n, int s,
                                               const Item* __restrict__ items, const uint32_t* __restrict__ did,
                                               const int32_t* __restrict__ did_blk, const float* __restrict__ upd,
                                               const float* __restrict__ pr_in, float* __restrict__ pr_out,
                                               const uint32_t* __restrict__ dmask, float* __restrict__ partial,
                                               double* __restrict__ red) {
  if (ctl->done) return;
  extern __shared__ float acc[];
  const Item it = items[blockIdx.x];
  const int64_t q = int64_t{1} << s;
  const int64_t v0 = static_cast<int64_t>(it.part) << s;
  const int qn = static_cast<int>(min(q, n - v0));
  for (int i = threadIdx.x; i < qn; i += BS) acc[i] = 0.0f;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t lo = it.lo, hi = it.hi;
  for (int64_t t = lo / kTile + threadIdx.x / kWave; t * kTile < hi; t += BS / kWave) {
    const int64_t tb = t * kTile;
    uint32_t x[kSub];
#pragma unroll
    for (int j = 0; j < kSub; ++j) x[j] = did[tb + j * kWave + lane];
    int32_t run = did_blk[t];
    int32_t ui[kSub];
#pragma unroll
    for (int j = 0; j < kSub; ++j) {
      const uint32_t f = x[j] >> 31;
      const uint64_t bal = wave_ballot(f != 0);
      ui[j] = run + lanes_below(bal) + static_cast<int32_t>(f) - 1;  // Alg. 5 update pointer
      run += __popcll(bal);
    }
    float val[kSub];
#pragma unroll
    for (int j = 0; j < kSub; ++j) {
      const int64_t e = tb + j * kWave + lane;
      val[j] = (e >= lo && e < hi) ? upd[ui[j]] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kSub; ++j) {
      const int64_t e = tb + j * kWave + lane;
      if (e >= lo && e < hi) atomicAdd(&acc[static_cast<int64_t>(x[j] & kIdMask) - v0], val[j]);
    }
  }
  __syncthreads();
  if (it.aux >= 0) {
    float* dst = partial + static_cast<int64_t>(it.aux) * q;
    for (int i = threadIdx.x; i < qn; i += BS) dst[i] = acc[i];
    return;
  }
  apply_partition<BS>(ctl, v0, qn, [&](int i) { return acc[i]; }, pr_in, pr_out, dmask, red + 2 * it.part);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_merge(const Ctl* __restrict__ ctl, int64_t n, int s,
                                              const Merge* __restrict__ mg, const float* __restrict__ partial,
                                              const float* __restrict__ pr_in, float* __restrict__ pr_out,
                                              const uint32_t* __restrict__ dmask, double* __restrict__ red) {
  if (ctl->done) return;
  const Merge mi = mg[blockIdx.x];
  const int64_t q = int64_t{1} << s;
  const int64_t v0 = static_cast<int64_t>(mi.part) << s;
  const int qn = static_cast<int>(min(q, n - v0));
  const float* base = partial + static_cast<int64_t>(mi.first) * q;
  const int cnt = mi.count;
  auto acc = [&](int i) {
    float sum = 0.0f;
    for (int c = 0; c < cnt; ++c) sum += base[static_cast<int64_t>(c) * q + i];
    return sum;
  };
  apply_partition<BS>(ctl, v0, qn, acc, pr_in, pr_out, dmask, red + 2 * mi.part);
}

__global__ __launch_bounds__(1024) void k_finalize(Ctl* __restrict__ ctl, const double* __restrict__ red,
                                                   int64_t k, double* __restrict__ hist, int64_t n) {
  if (ctl->done) return;
  double r = 0.0, dm = 0.0;
  for (int64_t j = threadIdx.x; j < k; j += 1024) {
    r += red[2 * j];
    dm += red[2 * j + 1];
  }
  block_sum2<1024>(r, dm);
  if (threadIdx.x == 0) {
    const double d = ctl->d;
    const int32_t it = ctl->iter;
    ctl->res = r;
    hist[it] = r;
    ctl->iter = it + 1;
    ctl->dmass = dm;
    ctl->base = (1.0 - d) / static_cast<double>(n) + d * dm / static_cast<double>(n);
    if (!isfinite(r) || !isfinite(dm)) {
      ctl->nonfinite = 1;
      ctl->done = 1;
    } else if (ctl->tol > 0.0 && r < ctl->tol) {
      ctl->done = 1;
    }
  }
}

// ---- start of a solve ----------------------------------------------------------------
__global__ void k_ctl_init(Ctl* ctl, double tol, double d) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ctl->base = 0.0;
    ctl->dmass = 0.0;
    ctl->res = 0.0;
    ctl->tol = tol;
    ctl->d = d;
    ctl->iter = 0;
    ctl->done = 0;
    ctl->nonfinite = 0;
    ctl->pad = 0;
  }
}

__global__ __launch_bounds__(256) void k_fill_value(float* __restrict__ x, int64_t n, float v) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    x[i] = v;
}

// Dangling mass of the starting vector: fixed grid, fixed per-thread order.
__global__ __launch_bounds__(256) void k_dangling_partial(const float* __restrict__ x,
                                                          const uint32_t* __restrict__ dmask, int64_t n,
                                                          double* __restrict__ red_init) {
  double dm = 0.0, nonfin = 0.0;
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; v < n;
       v += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float xv = x[v];
    if (!isfinite(xv)) nonfin += 1.0;
    if ((dmask[v >> 5] >> (v & 31)) & 1u) dm += static_cast<double>(xv);
  }
  block_sum2<256>(dm, nonfin);
  if (threadIdx.x == 0) red_init[blockIdx.x] = nonfin > 0.0 ? NAN : dm;
}

__global__ __launch_bounds__(256) void k_init_finalize(Ctl* __restrict__ ctl, const double* __restrict__ red_init,
                                                       int nb, int64_t n) {
  double dm = 0.0, unused = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) dm += red_init[i];
  block_sum2<256>(dm, unused);
  if (threadIdx.x == 0) {
    const double d = ctl->d;
    ctl->dmass = dm;
    ctl->base = (1.0 - d) / static_cast<double>(n) + d * dm / static_cast<double>(n);
    if (!isfinite(dm)) {
      ctl->nonfinite = 1;
      ctl->done = 1;
    }
  }
}

pcpm_status_t iter_lds_limits() {
  static bool done = false;
  if (done) return PCPM_OK;
  const int bytes = (1 << kMaxLog2) * 4;
  PCPM_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_scatter<kIterBlock>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  PCPM_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_gather<kIterBlock>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
  done = true;
  return PCPM_OK;
}

static pcpm_status_t start_solve(pcpm_png* g, double tol, double d, const float* x0, hipStream_t st) {
  PCPM_LAUNCH("pcpm_init", k_ctl_init, dim3(1), dim3(64), 0, st, g->ctl, tol, d);
  PCPM_LAUNCH("pcpm_init", k_dangling_partial, dim3(kInitBlocks), dim3(256), 0, st, x0, g->dmask, g->n,
              g->red_init);
  PCPM_LAUNCH("pcpm_init", k_init_finalize, dim3(1), dim3(256), 0, st, g->ctl, g->red_init, kInitBlocks, g->n);
  return PCPM_OK;
}

static pcpm_status_t run_iteration(pcpm_png* g, const float* in, float* out, hipStream_t st) {
  const size_t lds = static_cast<size_t>(g->q) * 4;
  const dim3 bs(kIterBlock);
  if (g->n_sc)
    PCPM_LAUNCH("pcpm_scatter", k_scatter<kIterBlock>, dim3(static_cast<unsigned>(g->n_sc)), bs, lds, st, g->ctl,
                g->n, g->part_log2, g->sc_items, in, g->outdeg, g->png_src, g->png_blk, g->seg_delta, g->upd);
  PCPM_LAUNCH("pcpm_gather", k_gather<kIterBlock>, dim3(static_cast<unsigned>(g->n_ga)), bs, lds, st, g->ctl, g->n,
              g->part_log2, g->ga_items, g->did, g->did_blk, g->upd, in, out, g->dmask, g->partial, g->red);
  if (g->n_mg)
    PCPM_LAUNCH("pcpm_merge", k_merge<kIterBlock>, dim3(static_cast<unsigned>(g->n_mg)), bs, 0, st, g->ctl, g->n,
                g->part_log2, g->mg_items, g->partial, in, out, g->dmask, g->red);
  PCPM_LAUNCH("pcpm_finalize", k_finalize, dim3(1), dim3(1024), 0, st, g->ctl, g->red, g->k, g->hist, g->n);
  return PCPM_OK;
}

static pcpm_status_t check_device(pcpm_png* g) {
  int dev = -1;
  PCPM_TRY_HIP(hipGetDevice(&dev));
  if (dev != g->device)
    return set_error(PCPM_ERR_INVALID_ARG, "handle lives on device %d but device %d is current", g->device, dev);
  return PCPM_OK;
}

}  // namespace pcpm

extern "C" {

pcpm_status_t pcpm_iterate(pcpm_png_t g, double d, const float* pr_in, float* pr_out, double* resid, void* stream) {
  using namespace pcpm;
  if (!g || !pr_in || !pr_out) return set_error(PCPM_ERR_INVALID_ARG, "NULL handle or vector");
  if (!(d >= 0.0 && d < 1.0)) return set_error(PCPM_ERR_INVALID_ARG, "d must lie in [0, 1)");
  if (pr_in == pr_out) return set_error(PCPM_ERR_INVALID_ARG, "pr_in and pr_out must differ");
  PCPM_TRY(check_device(g));
  hipStream_t st = static_cast<hipStream_t>(stream);
  PCPM_TRY(start_solve(g, 0.0, d, pr_in, st));
  PCPM_TRY(run_iteration(g, pr_in, pr_out, st));
  if (resid) {
    PCPM_TRY_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    PCPM_TRY_HIP(hipStreamSynchronize(st));
    *resid = g->ctl_host->res;
    if (g->ctl_host->nonfinite) return set_error(PCPM_ERR_NUMERIC, "non-finite rank, residual or dangling mass");
  }
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
  PCPM_TRY(check_device(g));
  hipStream_t st = static_cast<hipStream_t>(stream);
  float* a = pr_out;
  float* b = g->tmp_pr;
  if (init) {
    if (init != pr_out)
      PCPM_TRY_HIP(hipMemcpyAsync(a, init, static_cast<size_t>(g->n) * 4, hipMemcpyDeviceToDevice, st));
  } else {
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>((g->n + 255) / 256, 4096));
    PCPM_LAUNCH("pcpm_init", k_fill_value, dim3(blocks), dim3(256), 0, st, a, g->n,
                static_cast<float>(1.0 / static_cast<double>(g->n)));
  }
  PCPM_TRY(start_solve(g, tol, d, a, st));
  // Iterations are queued in small batches; after convergence the queued
  // kernels of the remaining iterations return immediately.
  constexpr int kBatch = 4;
  int launched = 0;
  while (launched < max_iters) {
    const int nb = std::min(kBatch, max_iters - launched);
    for (int i = 0; i < nb; ++i) {
      const int it = launched + i;
      const bool even = (it % 2) == 0;
      PCPM_TRY(run_iteration(g, even ? a : b, even ? b : a, st));
    }
    launched += nb;
    PCPM_TRY_HIP(hipMemcpyAsync(g->ctl_host, g->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, st));
    PCPM_TRY_HIP(hipStreamSynchronize(st));
    if (g->ctl_host->done) break;
  }
  const Ctl c = *g->ctl_host;
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

}  // extern "C"
