// Kernel timing with HIP events: each profiled launch is bracketed by two
// events on its own stream; sched_profile_read synchronises on the stop
// events and sums the elapsed times per kernel name.
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "prof.h"

namespace {
struct Pending {
  std::string name;
  hipEvent_t start, stop;
};
struct Acc {
  double ms = 0.0;
  int64_t launches = 0;
};
std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<hipEvent_t> g_pool;
std::vector<Pending> g_pending;
std::map<std::string, hipEvent_t> g_open;  // name -> start event of an open bracket
std::map<std::string, Acc> g_acc;

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

void drain_locked() {
  for (auto &p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.stop) == hipSuccess &&
        hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      Acc &a = g_acc[p.name];
      a.ms += ms;
      a.launches += 1;
    }
    g_pool.push_back(p.start);
    g_pool.push_back(p.stop);
  }
  g_pending.clear();
}
}  // namespace

namespace schedk {
bool prof_on() { return g_on.load(std::memory_order_relaxed); }

void prof_begin(const char *name, hipStream_t s) {
  if (!prof_on()) return;
  std::lock_guard<std::mutex> g(g_mu);
  hipEvent_t e = take_event();
  if (!e) return;
  (void)hipEventRecord(e, s);
  g_open[name] = e;
}

void prof_end(const char *name, hipStream_t s) {
  if (!prof_on()) return;
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_open.find(name);
  if (it == g_open.end()) return;
  hipEvent_t e = take_event();
  if (!e) return;
  (void)hipEventRecord(e, s);
  g_pending.push_back({name, it->second, e});
  g_open.erase(it);
  if (g_pending.size() > 4096) drain_locked();
}
}  // namespace schedk

extern "C" int sched_profile(int32_t enable) {
  if (enable < 0 || enable > 2) return SCHED_E_INVALID;
  std::lock_guard<std::mutex> g(g_mu);
  drain_locked();
  if (enable == 1) g_acc.clear();
  g_on.store(enable != 0);
  return SCHED_OK;
}

extern "C" int sched_profile_read(const char *kernel, double *total_ms, int64_t *launches) {
  if (!kernel || !total_ms || !launches) return SCHED_E_INVALID;
  std::lock_guard<std::mutex> g(g_mu);
  drain_locked();
  auto it = g_acc.find(kernel);
  *total_ms = it == g_acc.end() ? 0.0 : it->second.ms;
  *launches = it == g_acc.end() ? 0 : it->second.launches;
  return SCHED_OK;
}
