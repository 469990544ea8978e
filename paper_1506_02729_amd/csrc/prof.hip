// Optional per-kernel timing with HIP events recorded on the launch stream.
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "frsd_internal.h"

namespace frsd {

namespace {
struct Rec {
  std::string name;
  hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

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

bool prof_on() { return g_on; }

ProfScope::ProfScope(const char *name, hipStream_t s) : name_(name), s_(s) {
  if (!g_on) return;
  std::lock_guard<std::mutex> lk(g_mu);
  a_ = take_event();
  b_ = take_event();
  if (a_ && b_) hipEventRecord(a_, s_);
}

ProfScope::~ProfScope() {
  if (!a_ || !b_) return;
  hipEventRecord(b_, s_);
  std::lock_guard<std::mutex> lk(g_mu);
  g_recs.push_back({name_, a_, b_});
}

}  // namespace frsd

using namespace frsd;

extern "C" int frsd_profile(int enable) {
  clear_error();
  std::lock_guard<std::mutex> lk(g_mu);
  g_on = enable != 0;
  return FRSD_OK;
}

extern "C" int frsd_profile_report(char *buf, size_t len) {
  clear_error();
  if (!buf || len == 0) return fail(FRSD_EINVAL, "null buffer");
  std::lock_guard<std::mutex> lk(g_mu);
  std::map<std::string, std::pair<long, double>> agg;
  int rc = FRSD_OK;
  for (auto &r : g_recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      rc = fail(FRSD_EHIP, "event timing failed");
    auto &e = agg[r.name];
    e.first += 1;
    e.second += ms;
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
  std::string out;
  for (auto &kv : agg)
    out += kv.first + " " + std::to_string(kv.second.first) + " " + std::to_string(kv.second.second) + "\n";
  const size_t n = out.size() < len - 1 ? out.size() : len - 1;
  out.copy(buf, n);
  buf[n] = '\0';
  return rc;
}
