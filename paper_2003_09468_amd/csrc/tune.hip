// Autotuner of the tile shapes of the large contractions (Taylor terms, HS potential,
// force bias).  Each stage has a short list of compiled tile candidates; the tuner times
// every candidate on the caller's batch (same grouping of problems as the real launches)
// with HIP events and keeps the fastest in a process-wide cache keyed by the stage and the
// shapes and precisions of the group.  Launches look the cache up and fall back to
// candidate 0, the built-in default, for groups that were never tuned.
#include <float.h>

#include <map>
#include <mutex>

#include "internal.h"

namespace afqmc {

namespace {
std::mutex g_tmu;
std::map<std::string, int> g_cache;
}  // namespace

std::string tune_key(int stage, const Job* jobs, const int* ids, int c) {
  std::string k = std::to_string(stage);
  for (int q = 0; q < c; ++q) {
    const afqmc_kpt_problem& p = jobs[ids[q]].p;
    k += "|" + std::to_string(p.prec) + "," + std::to_string(p.nk) + "," + std::to_string(p.m) +
         "," + std::to_string(p.nocc) + "," + std::to_string(p.nchol) + "," +
         std::to_string(p.nwalk);
  }
  return k;
}

int tune_lookup(const std::string& key) {
  std::lock_guard<std::mutex> lk(g_tmu);
  auto it = g_cache.find(key);
  return it == g_cache.end() ? 0 : it->second;
}

void tune_store(const std::string& key, int choice) {
  std::lock_guard<std::mutex> lk(g_tmu);
  g_cache[key] = choice;
}

int tune_ncand(int stage, int prec) {
  switch (stage) {
    case TS_TAYLOR: return prec == AFQMC_PREC_BF16X3 ? 1 : low_prec(prec) ? 3 : 6;
    case TS_VHS: return prec == AFQMC_PREC_BF16X3 ? 1 : 3;
    case TS_VBIAS: return prec == AFQMC_PREC_BF16X3 ? 1 : 3;
    default: return 1;
  }
}

hipError_t tune_group(int stage, const Job* jobs, const int* ids, int c,
                      const std::function<hipError_t(int)>& run, hipStream_t s) {
  const int nc = tune_ncand(stage, jobs[ids[0]].p.prec);
  if (nc <= 1) {  // a single variant: nothing to time
    tune_store(tune_key(stage, jobs, ids, c), 0);
    return hipSuccess;
  }
  hipEvent_t a, b;
  hipError_t e = hipEventCreate(&a);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&b);
  if (e != hipSuccess) { (void)hipEventDestroy(a); return e; }
  int best = 0;
  float best_ms = FLT_MAX;
  constexpr int kReps = 3;
  for (int ch = 0; ch < nc && e == hipSuccess; ++ch) {
    e = run(ch);  // warm-up
    if (e != hipSuccess) break;
    e = hipEventRecord(a, s);
    for (int r = 0; r < kReps && e == hipSuccess; ++r) e = run(ch);
    if (e != hipSuccess) break;
    e = hipEventRecord(b, s);
    if (e != hipSuccess) break;
    e = hipEventSynchronize(b);
    if (e != hipSuccess) break;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, a, b);
    if (e == hipSuccess && ms < best_ms) { best_ms = ms; best = ch; }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return e;
  tune_store(tune_key(stage, jobs, ids, c), best);
  return hipSuccess;
}

}  // namespace afqmc
