// Stage timing with HIP events (rt_profile_* in include/rtucker.h).
#include <mutex>
#include <vector>

#include "../../include/rtucker.h"
#include "common.hpp"
#include "profile.hpp"

namespace rt {

namespace {

struct Pair {
  hipEvent_t a, b;
  int stage;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Pair> g_live;
std::vector<hipEvent_t> g_pool;
double g_ms[RT_PROFILE_STAGES];
int64_t g_cnt[RT_PROFILE_STAGES];

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

bool prof_enabled() { return g_on; }

ProfScope::ProfScope(int stage, hipStream_t s) : stage_(stage), s_(s) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  a_ = take_event();
  b_ = take_event();
  if (a_ && b_ && hipEventRecord(a_, s_) == hipSuccess) return;
  // no timing for this scope: hand the events back
  if (a_) g_pool.push_back(a_);
  if (b_) g_pool.push_back(b_);
  a_ = b_ = nullptr;
}

ProfScope::~ProfScope() {
  if (!a_ || !b_) return;
  const bool ok = hipEventRecord(b_, s_) == hipSuccess;
  std::lock_guard<std::mutex> lk(g_mu);
  if (ok) {
    g_live.push_back({a_, b_, stage_});
  } else {
    g_pool.push_back(a_);
    g_pool.push_back(b_);
  }
}

}  // namespace rt

using namespace rt;

extern "C" {

int rt_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = on != 0;
  if (g_on) {
    for (int i = 0; i < RT_PROFILE_STAGES; ++i) {
      g_ms[i] = 0.0;
      g_cnt[i] = 0;
    }
  }
  return RT_OK;
}

int rt_profile_read(rt_profile* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  for (const Pair& p : g_live) {
    hipError_t e = hipEventSynchronize(p.b);
    if (e != hipSuccess) return hip_fail(e, "profile event sync");
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, p.a, p.b);
    if (e != hipSuccess) return hip_fail(e, "profile elapsed time");
    if (p.stage >= 0 && p.stage < RT_PROFILE_STAGES) {
      g_ms[p.stage] += ms;
      g_cnt[p.stage] += 1;
    }
    g_pool.push_back(p.a);
    g_pool.push_back(p.b);
  }
  g_live.clear();
  if (out) {
    for (int i = 0; i < RT_PROFILE_STAGES; ++i) {
      out->ms[i] = g_ms[i];
      out->count[i] = g_cnt[i];
    }
  }
  return RT_OK;
}

}  // extern "C"
