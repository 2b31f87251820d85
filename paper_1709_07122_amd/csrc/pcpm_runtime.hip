// Error reporting, per-kernel event timing and handle teardown for libpcpm.
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pcpm_internal.hpp"

namespace pcpm {

static thread_local std::string t_last_error;

pcpm_status_t set_error(pcpm_status_t st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_last_error = buf;
  return st;
}

// ---- timing ---------------------------------------------------------------------
struct TimedLaunch {
  std::string name;
  hipEvent_t start, stop;
};

static std::mutex g_timing_mu;
static bool g_timing_on = false;
static std::vector<TimedLaunch> g_launches;

TimerScope::TimerScope(const char* n, hipStream_t s) : name(n), stream(s) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  if (!g_timing_on) return;
  if (hipEventCreate(&start) != hipSuccess) { start = nullptr; return; }
  if (hipEventRecord(start, stream) != hipSuccess) {
    (void)hipEventDestroy(start);
    start = nullptr;
  }
}

TimerScope::~TimerScope() {
  if (!start) return;
  hipEvent_t stop = nullptr;
  if (hipEventCreate(&stop) != hipSuccess || hipEventRecord(stop, stream) != hipSuccess) {
    (void)hipEventDestroy(start);
    if (stop) (void)hipEventDestroy(stop);
    return;
  }
  std::lock_guard<std::mutex> lk(g_timing_mu);
  g_launches.push_back({name, start, stop});
}

size_t timing_mark() {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  return g_launches.size();
}

void timing_discard_from(size_t pos) {
  std::vector<TimedLaunch> drop;
  {
    std::lock_guard<std::mutex> lk(g_timing_mu);
    if (pos >= g_launches.size()) return;
    drop.assign(g_launches.begin() + static_cast<std::ptrdiff_t>(pos), g_launches.end());
    g_launches.resize(pos);
  }
  for (auto& l : drop) {
    (void)hipEventSynchronize(l.stop);
    (void)hipEventDestroy(l.start);
    (void)hipEventDestroy(l.stop);
  }
}

// ---- plain HBM streams (the measured ceiling of the iteration kernels) ----------
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kStreamBlock = 256;
constexpr int kStreamGrid = 4096;
constexpr int kStreamUnroll = 4;

// kind 0: read (per-workgroup sums to dst), 1/2: write, 3/4: copy; 2 and 4
// with non-temporal stores.  n4 = number of 16-byte vectors.
template <int kKind>
__global__ __launch_bounds__(kStreamBlock) void k_stream(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                                         int64_t n4) {
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kStreamBlock;
  int64_t i = static_cast<int64_t>(blockIdx.x) * kStreamBlock + threadIdx.x;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const f32x4 fill = {1.f, 2.f, 3.f, 4.f};
  for (; i + (kStreamUnroll - 1) * stride < n4; i += kStreamUnroll * stride) {
    f32x4 v[kStreamUnroll];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u)
      if constexpr (kKind == 0 || kKind >= 3) v[u] = src[i + u * stride];
#pragma unroll
    for (int u = 0; u < kStreamUnroll; ++u) {
      if constexpr (kKind == 0) acc += v[u];
      else if constexpr (kKind == 1) dst[i + u * stride] = fill;
      else if constexpr (kKind == 2) __builtin_nontemporal_store(fill, dst + i + u * stride);
      else if constexpr (kKind == 3) dst[i + u * stride] = v[u];
      else __builtin_nontemporal_store(v[u], dst + i + u * stride);
    }
  }
  for (; i < n4; i += stride) {
    if constexpr (kKind == 0) acc += src[i];
    else if constexpr (kKind == 1) dst[i] = fill;
    else if constexpr (kKind == 2) __builtin_nontemporal_store(fill, dst + i);
    else if constexpr (kKind == 3) dst[i] = src[i];
    else __builtin_nontemporal_store(src[i], dst + i);
  }
  if constexpr (kKind == 0) {
    __shared__ float sh[kStreamBlock / 64];
    float t = acc.x + acc.y + acc.z + acc.w;
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x / 64] = t;
    __syncthreads();
    if (threadIdx.x == 0) reinterpret_cast<float*>(dst)[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
  }
}

void dfree(pcpm_png* g, void* p) {
  for (auto it = g->allocations.begin(); it != g->allocations.end(); ++it) {
    if (it->first == p) {
      (void)hipFree(p);
      g->device_bytes -= static_cast<int64_t>(it->second);
      g->allocations.erase(it);
      return;
    }
  }
}

void free_handle(pcpm_png* g) {
  if (!g) return;
  for (auto& a : g->allocations) (void)hipFree(a.first);
  g->allocations.clear();
  if (g->ctl_host) (void)hipHostFree(g->ctl_host);
  for (hipEvent_t& e : g->ctl_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (g->psync_host) (void)hipHostFree(g->psync_host);
  g->psync_host = nullptr;
  if (g->gctl_host) (void)hipHostFree(g->gctl_host);
  if (g->ppr_vctl_host) (void)hipHostFree(g->ppr_vctl_host);
  g->ppr_vctl_host = nullptr;
  g->ctl_host = nullptr;
  g->gctl_host = nullptr;
  delete g;
}

}  // namespace pcpm

extern "C" {

const char* pcpm_last_error(void) { return pcpm::t_last_error.c_str(); }

pcpm_status_t pcpm_hbm_stream(int32_t kind, const void* src, void* dst, int64_t bytes, void* stream) {
  using namespace pcpm;
  if (kind < 0 || kind > 4) return set_error(PCPM_ERR_INVALID_ARG, "stream kind %d is not 0..4", kind);
  if (bytes <= 0 || bytes % 16) return set_error(PCPM_ERR_INVALID_ARG, "bytes must be a positive multiple of 16");
  if (!dst || (kind != 1 && kind != 2 && !src)) return set_error(PCPM_ERR_INVALID_ARG, "NULL buffer");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16)
    return set_error(PCPM_ERR_INVALID_ARG, "buffers must be 16-byte aligned");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const auto* s4 = static_cast<const f32x4*>(src);
  auto* d4 = static_cast<f32x4*>(dst);
  const int64_t n4 = bytes / 16;
  switch (kind) {
    case 0: PCPM_LAUNCH("pcpm_stream_read", k_stream<0>, dim3(kStreamGrid), dim3(kStreamBlock), 0, st, s4, d4, n4); break;
    case 1: PCPM_LAUNCH("pcpm_stream_write", k_stream<1>, dim3(kStreamGrid), dim3(kStreamBlock), 0, st, s4, d4, n4); break;
    case 2: PCPM_LAUNCH("pcpm_stream_write_nt", k_stream<2>, dim3(kStreamGrid), dim3(kStreamBlock), 0, st, s4, d4, n4); break;
    case 3: PCPM_LAUNCH("pcpm_stream_copy", k_stream<3>, dim3(kStreamGrid), dim3(kStreamBlock), 0, st, s4, d4, n4); break;
    default: PCPM_LAUNCH("pcpm_stream_copy_nt", k_stream<4>, dim3(kStreamGrid), dim3(kStreamBlock), 0, st, s4, d4, n4); break;
  }
  return PCPM_OK;
}

void pcpm_png_free(pcpm_png_t g) { pcpm::free_handle(g); }

void pcpm_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(pcpm::g_timing_mu);
  pcpm::g_timing_on = on != 0;
}

int pcpm_timing_collect(pcpm_kernel_time_t* out, int max_entries) {
  std::vector<pcpm::TimedLaunch> launches;
  {
    std::lock_guard<std::mutex> lk(pcpm::g_timing_mu);
    launches.swap(pcpm::g_launches);
  }
  std::map<std::string, std::pair<int64_t, double>> acc;
  for (auto& l : launches) {
    float ms = 0.f;
    if (hipEventSynchronize(l.stop) == hipSuccess && hipEventElapsedTime(&ms, l.start, l.stop) == hipSuccess) {
      auto& a = acc[l.name];
      a.first += 1;
      a.second += ms;
    }
    (void)hipEventDestroy(l.start);
    (void)hipEventDestroy(l.stop);
  }
  int i = 0;
  for (auto& kv : acc) {
    if (out && i < max_entries) {
      memset(out[i].name, 0, sizeof(out[i].name));
      strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
      out[i].launches = kv.second.first;
      out[i].total_ms = kv.second.second;
    }
    ++i;
  }
  return i;
}

}  // extern "C"
