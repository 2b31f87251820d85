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
