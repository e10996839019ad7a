// Per-kernel event timing for the benchmark: when enabled for a kernel name,
// every launch of that kernel is bracketed by a pair of HIP events recorded on
// the launch stream, together with the launch's algorithmic bytes and flops.
// dd_kernel_timer_read synchronises the recorded events and reports totals.
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>

#include "ktimer.h"

namespace {

struct Rec {
  hipEvent_t a, b;
  double bytes, flops;
};

struct Timers {
  std::mutex mu;
  std::map<std::string, std::vector<Rec>> recs;
  std::vector<hipEvent_t> pool;
  bool all = false;
  std::map<std::string, bool> on;
  std::atomic<bool> any{false};   // some kernel is being timed (read without the lock)
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e;
    (void)hipEventCreate(&e);
    return e;
  }
};

Timers& T() {
  static Timers t;
  return t;
}

thread_local hipEvent_t t_start = nullptr;
thread_local bool t_suspended = false;
thread_local double t_model_bytes = 0.0, t_model_flops = 0.0;

}  // namespace

void ktimer_suspend(bool on) { t_suspended = on; }

void ktimer_account(double bytes, double flops) {
  t_model_bytes += bytes;
  t_model_flops += flops;
}
void ktimer_model(double* bytes, double* flops) {
  *bytes = t_model_bytes;
  *flops = t_model_flops;
}
void ktimer_model_set(double bytes, double flops) {
  t_model_bytes = bytes;
  t_model_flops = flops;
}

bool ktimer_enabled(const char* tag) {
  if (t_suspended) return false;   // launches being captured into a graph are not timed
  Timers& t = T();
  if (!t.any.load(std::memory_order_acquire)) return false;
  std::lock_guard<std::mutex> g(t.mu);
  return t.all || t.on.count(tag);
}

void ktimer_begin(const char* tag, hipStream_t st) {
  Timers& t = T();
  std::lock_guard<std::mutex> g(t.mu);
  t_start = t.get();
  (void)hipEventRecord(t_start, st);
}

void ktimer_end(const char* tag, hipStream_t st, double bytes, double flops) {
  Timers& t = T();
  std::lock_guard<std::mutex> g(t.mu);
  hipEvent_t e = t.get();
  (void)hipEventRecord(e, st);
  t.recs[tag].push_back(Rec{t_start, e, bytes, flops});
}

extern "C" {

// Enable timing for a kernel name ("*" = every instrumented kernel); NULL disables all and clears.
dd_status dd_kernel_timer_enable(const char* name) {
  Timers& t = T();
  std::lock_guard<std::mutex> g(t.mu);
  if (!name) {
    t.all = false;
    t.on.clear();
    for (auto& kv : t.recs)
      for (auto& r : kv.second) {
        t.pool.push_back(r.a);
        t.pool.push_back(r.b);
      }
    t.recs.clear();
    t.any.store(false, std::memory_order_release);
    return DD_OK;
  }
  if (std::strcmp(name, "*") == 0) t.all = true;
  else t.on[name] = true;
  t.any.store(true, std::memory_order_release);
  return DD_OK;
}

// Totals for one kernel name since it was enabled: summed event time (ms),
// launches, algorithmic bytes and flops.  Synchronises the recorded events.
dd_status dd_kernel_timer_read(const char* name, double* total_ms, int64_t* launches, double* bytes, double* flops) {
  Timers& t = T();
  std::lock_guard<std::mutex> g(t.mu);
  double ms = 0.0, by = 0.0, fl = 0.0;
  int64_t n = 0;
  auto it = t.recs.find(name ? name : "");
  if (it != t.recs.end())
    for (auto& r : it->second) {
      if (hipEventSynchronize(r.b) != hipSuccess) return DD_EDEVICE;
      float e = 0.0f;
      if (hipEventElapsedTime(&e, r.a, r.b) != hipSuccess) return DD_EDEVICE;
      ms += e;
      by += r.bytes;
      fl += r.flops;
      ++n;
    }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = n;
  if (bytes) *bytes = by;
  if (flops) *flops = fl;
  return DD_OK;
}

// Names of the kernels with records, separated by ';' (buffer of `cap` bytes).
dd_status dd_kernel_timer_names(char* buf, size_t cap) {
  Timers& t = T();
  std::lock_guard<std::mutex> g(t.mu);
  std::string s;
  for (auto& kv : t.recs) {
    if (!s.empty()) s += ";";
    s += kv.first;
  }
  if (!buf || cap == 0) return DD_EINVAL;
  std::strncpy(buf, s.c_str(), cap - 1);
  buf[cap - 1] = 0;
  return DD_OK;
}

}  // extern "C"
