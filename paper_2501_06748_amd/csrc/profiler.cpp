// Live kernel timing with HIP events.
//
// When a kernel id is enabled, every launch of that kernel is bracketed by a
// pair of events recorded on the stream the kernel is launched on; the
// elapsed times are accumulated when the caller reads the profile.  Used to
// measure the average launch duration of the dominant kernel inside a timed
// region without an external profiler.  Not thread-safe (one host thread).
#include "sbfwi_internal.h"

namespace {

struct PendingPair {
  int id;
  hipEvent_t a, b;
};

struct Prof {
  uint32_t mask = 0;
  std::vector<PendingPair> pending;
  std::vector<hipEvent_t> pool;
  double ms[SBFWI_PROF_KERNELS] = {};
  int64_t calls[SBFWI_PROF_KERNELS] = {};
};

Prof g_prof;

// Accumulates the oldest recorded pairs (waiting for them) and returns their
// events to the pool.
int drain(size_t count) {
  count = count < g_prof.pending.size() ? count : g_prof.pending.size();
  for (size_t i = 0; i < count; ++i) {
    auto& p = g_prof.pending[i];
    SBFWI_HIP(hipEventSynchronize(p.b));
    float ms = 0.f;
    SBFWI_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    g_prof.ms[p.id] += ms;
    g_prof.calls[p.id] += 1;
    g_prof.pool.push_back(p.a);
    g_prof.pool.push_back(p.b);
  }
  g_prof.pending.erase(g_prof.pending.begin(), g_prof.pending.begin() + count);
  return SBFWI_OK;
}

// pairs kept in flight before the oldest half is drained (bounds the event pool;
// the newest half stays queued, so the device never runs dry)
constexpr size_t kMaxPending = 8192;

hipEvent_t take() {
  if (!g_prof.pool.empty()) {
    hipEvent_t e = g_prof.pool.back();
    g_prof.pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

}  // namespace

static int g_suspended = 0;

void sbfwi_prof_suspend(int on) { g_suspended = on; }

ProfScope::ProfScope(int id, hipStream_t s) : id_(id), s_(s) {
  if (g_suspended || !(g_prof.mask & (1u << id))) return;
  a_ = take();
  if (a_ && hipEventRecord((hipEvent_t)a_, s) != hipSuccess) a_ = nullptr;
}

ProfScope::~ProfScope() {
  if (!a_) return;
  hipEvent_t b = take();
  if (!b) return;
  if (hipEventRecord(b, s_) != hipSuccess) return;
  g_prof.pending.push_back({id_, (hipEvent_t)a_, b});
  if (g_prof.pending.size() > kMaxPending) drain(kMaxPending / 2);
}

extern "C" int sbfwi_profile(uint32_t kernel_mask) {
  g_prof.mask = kernel_mask;
  return SBFWI_OK;
}

// Destroys every event of the pool and of the pending pairs (their times are
// discarded) and switches timing off.
int sbfwi_prof_release() {
  int rc = SBFWI_OK;
  g_prof.mask = 0;
  for (auto& p : g_prof.pending) {
    g_prof.pool.push_back(p.a);
    g_prof.pool.push_back(p.b);
  }
  g_prof.pending.clear();
  for (hipEvent_t e : g_prof.pool)
    if (hipEventDestroy(e) != hipSuccess) rc = sbfwi_fail(SBFWI_EHIP, "hipEventDestroy failed");
  g_prof.pool.clear();
  return rc;
}

extern "C" int sbfwi_profile_read(double* out, int reset) {
  if (!out) return sbfwi_fail(SBFWI_EINVAL, "NULL argument");
  SBFWI_CHECK(drain(g_prof.pending.size()));
  for (int k = 0; k < SBFWI_PROF_KERNELS; ++k) {
    out[2 * k] = (double)g_prof.calls[k];
    out[2 * k + 1] = g_prof.ms[k];
    if (reset) {
      g_prof.calls[k] = 0;
      g_prof.ms[k] = 0.0;
    }
  }
  return SBFWI_OK;
}
