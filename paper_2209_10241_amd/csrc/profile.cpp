// Per-kernel timing with HIP events, for observability: while enabled, the
// counting calls bracket each kernel launch with events on the launch stream;
// hm_profile_read waits for the recorded events and reports, per kernel, the
// number of launches and the summed duration.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "hm_internal.h"

namespace hm {
namespace {

struct Pending {
  std::string name;
  hipEvent_t start, stop;
};

struct Totals {
  uint64_t launches = 0;
  double ms = 0.0;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Pending> g_pending;
std::map<std::string, Totals> g_totals;

int drain_locked() {
  for (auto& p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.stop) != hipSuccess || hipEventElapsedTime(&ms, p.start, p.stop) != hipSuccess) {
      set_error("profiling event failed");
      return HM_EDEVICE;
    }
    Totals& t = g_totals[p.name];
    t.launches += 1;
    t.ms += ms;
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  g_pending.clear();
  return HM_OK;
}

}  // namespace

thread_local int g_capturing = 0;

bool profiling() { return g_on && !g_capturing; }
void capture_begin() { ++g_capturing; }
void capture_end() { --g_capturing; }

ProfileScope::ProfileScope(const char* name, hipStream_t st) : name_(name), st_(st) {
  if (!profiling()) return;
  if (hipEventCreate(&start_) != hipSuccess || hipEventCreate(&stop_) != hipSuccess) return;
  if (hipEventRecord(start_, st_) != hipSuccess) return;
  active_ = true;
}

ProfileScope::~ProfileScope() {
  if (!active_) return;
  if (hipEventRecord(stop_, st_) != hipSuccess) return;
  std::lock_guard<std::mutex> lock(g_mu);
  g_pending.push_back(Pending{name_, start_, stop_});
}

}  // namespace hm

extern "C" {

int hm_profile_enable(int on) {
  try {
    std::lock_guard<std::mutex> lock(hm::g_mu);
    hm::g_on = on != 0;
    return HM_OK;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_profile_reset(void) {
  try {
    std::lock_guard<std::mutex> lock(hm::g_mu);
    int rc = hm::drain_locked();
    hm::g_totals.clear();
    return rc;
  } catch (...) {
    return hm::api_failure();
  }
}

int hm_profile_read(int max_entries, char* names, uint64_t* launches, double* total_ms) {
  try {
    std::lock_guard<std::mutex> lock(hm::g_mu);
    HM_TRY(hm::drain_locked());
    int n = 0;
    for (const auto& kv : hm::g_totals) {
      if (n >= max_entries) break;
      if (names) {
        std::strncpy(names + size_t(n) * 64, kv.first.c_str(), 63);
        names[size_t(n) * 64 + 63] = '\0';
      }
      if (launches) launches[n] = kv.second.launches;
      if (total_ms) total_ms[n] = kv.second.ms;
      ++n;
    }
    return n;
  } catch (...) {
    return hm::api_failure();
  }
}

}  // extern "C"
