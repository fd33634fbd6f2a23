// Optional per-kernel timing: when enabled, every kernel launch of the
// library is bracketed by two hipEvents recorded on the launch stream.
// rfd_profile_read synchronises the device and folds the finished pairs into
// per-kernel totals.
#include <atomic>
#include <mutex>
#include <vector>

#include "rfd_internal.h"

namespace rfd {
namespace {

struct Pending {
  int id;
  hipEvent_t a, b;
};

struct Profiler {
  std::mutex mu;
  bool on = false;
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double total_ms[kNumKernelIds] = {};
  int64_t count[kNumKernelIds] = {};

  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};

Profiler& prof() {
  static Profiler p;
  return p;
}

}  // namespace

static std::atomic<int> g_capturing{0};
void set_capturing(bool on) { g_capturing.fetch_add(on ? 1 : -1); }

ProfileScope::ProfileScope(int id, hipStream_t st) : id_(id), st_(st) {
  if (g_capturing.load() > 0) return;
  Profiler& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  if (!p.on) return;
  a_ = p.get();
  b_ = p.get();
  if (a_ && b_ && hipEventRecord(a_, st_) == hipSuccess) active_ = true;
}

ProfileScope::~ProfileScope() {
  if (!active_) return;
  Profiler& p = prof();
  std::lock_guard<std::mutex> g(p.mu);
  if (hipEventRecord(b_, st_) == hipSuccess) p.pending.push_back(Pending{id_, a_, b_});
}

const char* kernel_name(int id) {
  static const char* names[kNumKernelIds] = {"k_bta_gram", "k_bta", "k_reduce", "k_phi1", "k_gcore", "k_expand",
                                             "k_phi1_batch", "k_bta_batch", "k_expand_batch",
                                             "k_phi1_apply"};
  return (id >= 0 && id < kNumKernelIds) ? names[id] : "?";
}

}  // namespace rfd

extern "C" {

void rfd_profile_enable(int on) {
  rfd::Profiler& p = rfd::prof();
  std::lock_guard<std::mutex> g(p.mu);
  p.on = on != 0;
}

int32_t rfd_profile_read(double* total_ms, int64_t* counts, int32_t n, int32_t reset) {
  rfd::Profiler& p = rfd::prof();
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(p.mu);
  for (const auto& q : p.pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
      p.total_ms[q.id] += ms;
      p.count[q.id] += 1;
    }
    p.pool.push_back(q.a);
    p.pool.push_back(q.b);
  }
  p.pending.clear();
  const int k = n < rfd::kNumKernelIds ? n : rfd::kNumKernelIds;
  for (int i = 0; i < k; ++i) {
    if (total_ms) total_ms[i] = p.total_ms[i];
    if (counts) counts[i] = p.count[i];
  }
  if (reset) {
    for (int i = 0; i < rfd::kNumKernelIds; ++i) {
      p.total_ms[i] = 0.0;
      p.count[i] = 0;
    }
  }
  return rfd::kNumKernelIds;
}

const char* rfd_profile_kernel_name(int32_t id) { return rfd::kernel_name(id); }

void rfd_library_release(void) {
  rfd::Profiler& p = rfd::prof();
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(p.mu);
  for (const auto& q : p.pending) {
    p.pool.push_back(q.a);
    p.pool.push_back(q.b);
  }
  p.pending.clear();
  for (hipEvent_t e : p.pool) (void)hipEventDestroy(e);
  p.pool.clear();
  p.on = false;
  rfd::release_spectrum_records();
}

}  // extern "C"
