// Optional per-kernel-class timing with HIP events on the launch stream (diagnostics).
// When enabled, each launch of a kernel class is bracketed by two events recorded on the
// stream the kernel runs on; afqmc_kpt_timing_read synchronises on the recorded events and
// returns the accumulated milliseconds and launch count of one class.
#include <mutex>
#include <vector>

#include "internal.h"
#include "timing.h"

namespace afqmc {

namespace {
struct Rec {
  hipEvent_t a, b;
  int kc;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_pool;  // created at enable time
size_t g_used = 0;
double g_ms[KC_COUNT];
long long g_n[KC_COUNT];
long long g_dropped = 0;
}  // namespace

bool timing_on() { return g_on; }

TimedScope::TimedScope(int kc, hipStream_t s) : rec_(-1), s_(s) {
  if (!g_on) return;
  // launches being captured into a graph are not timed
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_used >= g_pool.size()) { ++g_dropped; return; }
  rec_ = (int)g_used++;
  g_pool[rec_].kc = kc;
  (void)hipEventRecord(g_pool[rec_].a, s_);
}

TimedScope::~TimedScope() {
  if (rec_ < 0) return;
  (void)hipEventRecord(g_pool[rec_].b, s_);
}

static void drain_locked() {
  for (size_t i = 0; i < g_used; ++i) {
    float ms = 0.f;
    if (hipEventSynchronize(g_pool[i].b) == hipSuccess &&
        hipEventElapsedTime(&ms, g_pool[i].a, g_pool[i].b) == hipSuccess) {
      g_ms[g_pool[i].kc] += ms;
      g_n[g_pool[i].kc] += 1;
    }
  }
  g_used = 0;
}

}  // namespace afqmc

using namespace afqmc;

extern "C" {

afqmc_status afqmc_kpt_timing_enable(int enable, int capacity) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (enable) {
    if (capacity < 1 || capacity > (1 << 20)) return AFQMC_EINVAL;
    if (g_pool.size() < (size_t)capacity) {
      size_t old = g_pool.size();
      g_pool.resize(capacity);
      for (size_t i = old; i < g_pool.size(); ++i) {
        if (hipEventCreate(&g_pool[i].a) != hipSuccess || hipEventCreate(&g_pool[i].b) != hipSuccess) {
          g_pool.resize(i);
          return AFQMC_EHIP;
        }
      }
    }
    for (int k = 0; k < KC_COUNT; ++k) { g_ms[k] = 0.0; g_n[k] = 0; }
    g_used = 0;
    g_dropped = 0;
    g_on = true;
  } else {
    drain_locked();
    g_on = false;
  }
  return AFQMC_OK;
}

afqmc_status afqmc_kpt_timing_read(int kclass, double* total_ms, long long* launches) {
  if (!total_ms || !launches) return AFQMC_ENULL;
  if (kclass < 0 || kclass >= KC_COUNT) return AFQMC_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  drain_locked();
  *total_ms = g_ms[kclass];
  *launches = g_n[kclass];
  return AFQMC_OK;
}

}  // extern "C"
