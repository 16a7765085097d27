// Optional launch timing per kernel class (bie_profile_enable / bie_profile_read): a pair of HIP
// events around each launch on its own stream, read back only when asked.
#include <hip/hip_runtime.h>

#include <vector>

#include "internal.h"

namespace bie {
namespace {

struct Rec {
  hipEvent_t a, b;
  long long pairs;
};

struct ClassStats {
  std::vector<Rec> pending;
  long long launches = 0, pairs = 0;
  double ms = 0.0;
};

bool g_on = false;
unsigned g_mask = ~0u;
int g_every = 1;                        // record every g_every-th launch of a class
long long g_seen[BIE_K_COUNT] = {};      // launches of each class while enabled
ClassStats g_stats[BIE_K_COUNT];
std::vector<hipEvent_t> g_pool;

hipEvent_t get_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // timing only: no system-scope fence (a cache write-back) at the markers, which would add its
  // own cost to the measured launches and to the work after them
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

int drain(ClassStats &c) {
  for (Rec &r : c.pending) {
    if (hipEventSynchronize(r.b) != hipSuccess) return BIE_EDEVICE;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return BIE_EDEVICE;
    c.ms += ms;
    c.launches += 1;
    c.pairs += r.pairs;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  c.pending.clear();
  return BIE_OK;
}

thread_local int g_suspend = 0;  // > 0 inside a ProfSuspend

}  // namespace

ProfSuspend::ProfSuspend() { ++g_suspend; }
ProfSuspend::~ProfSuspend() { --g_suspend; }

ProfScope::ProfScope(int k, hipStream_t st, long long p)
    : kclass(k), s(st), pairs(p), on(g_on && ((g_mask >> k) & 1u) && g_suspend == 0) {
  if (!on) return;
  on = g_seen[k]++ % g_every == 0;
  if (!on) return;
  hipEvent_t a = get_event();
  if (!a) {
    on = false;
    return;
  }
  hipEventRecord(a, s);
  g_stats[kclass].pending.push_back({a, nullptr, pairs});
}

ProfScope::~ProfScope() {
  if (!on) return;
  hipEvent_t b = get_event();
  Rec &r = g_stats[kclass].pending.back();
  if (!b) {
    g_pool.push_back(r.a);
    g_stats[kclass].pending.pop_back();
    return;
  }
  hipEventRecord(b, s);
  r.b = b;
}

}  // namespace bie

using namespace bie;

extern "C" {

int bie_profile_enable(int on) {
  for (auto &c : g_stats) {
    if (drain(c) != BIE_OK) return BIE_EDEVICE;
    c = ClassStats();
  }
  g_on = on != 0;
  for (auto &n : g_seen) n = 0;
  return BIE_OK;
}

int bie_profile_select(unsigned mask) {
  g_mask = mask;
  return BIE_OK;
}

int bie_profile_sample(int every) {
  if (every < 1) {
    set_error("bie_profile_sample: every must be at least 1");
    return BIE_EINVAL;
  }
  g_every = every;
  return BIE_OK;
}

int bie_profile_read(int kclass, long long *launches, double *ms_total, long long *pairs) {
  if (kclass < 0 || kclass >= BIE_K_COUNT) {
    set_error("bie_profile_read: unknown kernel class");
    return BIE_EINVAL;
  }
  BIE_TRY(drain(g_stats[kclass]));
  if (launches) *launches = g_stats[kclass].launches;
  if (ms_total) *ms_total = g_stats[kclass].ms;
  if (pairs) *pairs = g_stats[kclass].pairs;
  return BIE_OK;
}

}  // extern "C"
