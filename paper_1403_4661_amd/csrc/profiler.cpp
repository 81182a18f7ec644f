// Event-pair timing of named kernel launches (osht_plan_set_profiling).

#include <cstring>

#include "common.hpp"

namespace osht {

hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  OSHT_HIP(hipEventCreate(&e));
  return e;
}

Profiler::Stat& Profiler::stat(const char* name) {
  for (auto& kv : stats)
    if (kv.first == name) return kv.second;
  stats.emplace_back(name, Stat{});
  return stats.back().second;
}

void Profiler::flush(Stat& s) {
  for (auto& pr : s.pending) {
    OSHT_HIP(hipEventSynchronize(pr.second));
    float ms = 0.f;
    OSHT_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
    s.ms += ms;
    s.count += 1;
    pool.push_back(pr.first);
    pool.push_back(pr.second);
  }
  s.pending.clear();
}

void Profiler::reset() {
  for (auto& kv : stats) {
    for (auto& pr : kv.second.pending) {
      (void)hipEventSynchronize(pr.second);
      pool.push_back(pr.first);
      pool.push_back(pr.second);
    }
  }
  stats.clear();
}

Profiler::~Profiler() {
  reset();
  for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

}  // namespace osht
