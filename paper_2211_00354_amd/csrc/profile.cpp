// Stage profiler: HIP events recorded around each stage on the stream that
// runs it; durations are resolved (after the events complete) on read.
#include <atomic>
#include <map>
#include <mutex>

#include "lens_internal.h"

namespace lensfmm {

namespace {
std::atomic<bool> g_on{false};
std::mutex g_mu;
struct Pending {
  std::string name;
  hipEvent_t a, b;
};
std::vector<Pending> g_pending;
struct Acc {
  double ms = 0;
  int64_t n = 0;
};
std::map<std::string, Acc> g_acc;

void resolve_locked() {
  for (auto &p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto &a = g_acc[p.name];
      a.ms += ms;
      a.n += 1;
    }
    (void)hipGetLastError();
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  g_pending.clear();
}
}  // namespace

thread_local bool t_capturing = false;
thread_local int t_no_timing = 0;
void set_capturing(bool on) { t_capturing = on; }
NoTiming::NoTiming() { ++t_no_timing; }
NoTiming::~NoTiming() { --t_no_timing; }
bool profiling_enabled() {
  return !t_capturing && t_no_timing == 0 && g_on.load(std::memory_order_relaxed);
}

StageTimer::StageTimer(const char *n, hipStream_t s) : name(n), stream(s) {
  if (!profiling_enabled()) return;
  if (hipEventCreate(&ev0) != hipSuccess || hipEventCreate(&ev1) != hipSuccess ||
      hipEventRecord(ev0, s) != hipSuccess) {
    (void)hipGetLastError();
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    ev0 = ev1 = nullptr;
  }
}

StageTimer::~StageTimer() {
  if (!ev0) return;
  if (hipEventRecord(ev1, stream) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
    return;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_pending.push_back({name, ev0, ev1});
}

}  // namespace lensfmm

using namespace lensfmm;

extern "C" {

LENS_API void lens_profile_enable(int32_t on) {
  std::lock_guard<std::mutex> lk(g_mu);
  resolve_locked();
  if (on) g_acc.clear();
  g_on.store(on != 0);
}

LENS_API int32_t lens_profile_read(int32_t cap, const char **names, double *total_ms,
                                   int64_t *launches) {
  std::lock_guard<std::mutex> lk(g_mu);
  resolve_locked();
  int32_t i = 0;
  for (auto &kv : g_acc) {
    if (i < cap) {
      if (names) names[i] = kv.first.c_str();
      if (total_ms) total_ms[i] = kv.second.ms;
      if (launches) launches[i] = kv.second.n;
    }
    ++i;
  }
  return i;
}

}  // extern "C"
