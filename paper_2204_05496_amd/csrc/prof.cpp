// prof.cpp -- opt-in per-kernel timing with HIP events recorded on the stream
// each kernel is launched on (lrhe_prof_* in include/lrhe.h).
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lrhe_internal.h"

namespace lrhe {
namespace {
struct Rec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::map<std::string, std::pair<uint64_t, double>> g_sum;   // name -> (launches, ms)

hipEvent_t take() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}
void drain_locked() {
  for (auto& r : g_recs) {
    float ms = 0;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& s = g_sum[r.name];
      s.first += 1;
      s.second += ms;
    }
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
}
}  // namespace

ProfScope::ProfScope(hipStream_t s, const char* name) : s_(s), name_(name) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return;
  a_ = take();
  b_ = take();
  (void)hipEventRecord((hipEvent_t)a_, s_);
}
ProfScope::~ProfScope() {
  if (!a_) return;
  std::lock_guard<std::mutex> lk(g_mu);
  (void)hipEventRecord((hipEvent_t)b_, s_);
  g_recs.push_back({name_, (hipEvent_t)a_, (hipEvent_t)b_});
  if (g_recs.size() > 4096) drain_locked();
}
}  // namespace lrhe

extern "C" void lrhe_prof_enable(int on) {
  std::lock_guard<std::mutex> lk(lrhe::g_mu);
  lrhe::g_on = on != 0;
}
extern "C" void lrhe_prof_reset(void) {
  std::lock_guard<std::mutex> lk(lrhe::g_mu);
  lrhe::drain_locked();
  lrhe::g_sum.clear();
}
extern "C" int lrhe_prof_get(const char* kernel, uint64_t* launches, double* total_ms) {
  std::lock_guard<std::mutex> lk(lrhe::g_mu);
  lrhe::drain_locked();
  auto it = lrhe::g_sum.find(kernel ? kernel : "");
  if (launches) *launches = it == lrhe::g_sum.end() ? 0 : it->second.first;
  if (total_ms) *total_ms = it == lrhe::g_sum.end() ? 0.0 : it->second.second;
  return LRHE_OK;
}
