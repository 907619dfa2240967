// Opt-in per-kernel timing: two events per launch on the launch's stream,
// summed per kernel name when collected.  Off by default; costs nothing then.

#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

#include "internal.h"

namespace umbir {
namespace {

struct Pending {
  const char* name;
  hipEvent_t start, stop;
};

struct Totals {
  long long launches = 0;
  double ms = 0.0;
};

std::atomic<bool> g_on{false};
std::atomic<bool> g_filtered{false};
std::mutex g_mu;
std::vector<std::string> g_select;  // kernel names timed while g_filtered
std::vector<long long> g_seen;      // launches of each selected kernel so far
int g_every = 1;                    // while g_filtered: time every g_every-th launch
std::vector<Pending> g_pending;
std::map<std::string, Totals> g_totals;

}  // namespace

bool prof_on(const char* name) {
  if (!g_on.load(std::memory_order_relaxed)) return false;
  if (!g_filtered.load(std::memory_order_relaxed)) return true;
  std::lock_guard<std::mutex> lk(g_mu);
  for (size_t k = 0; k < g_select.size(); ++k)
    if (g_select[k] == name) return g_seen[k]++ % g_every == 0;
  return false;
}

hipEvent_t prof_start(hipStream_t s) {
  // launches recorded into a graph are not timed (the events would be captured too)
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return nullptr;
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  if (hipEventRecord(e, s) != hipSuccess) {
    (void)hipEventDestroy(e);
    return nullptr;
  }
  return e;
}

void prof_stop(const char* name, hipStream_t s, hipEvent_t start) {
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess || hipEventRecord(e, s) != hipSuccess) {
    if (e) (void)hipEventDestroy(e);
    (void)hipEventDestroy(start);
    return;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  g_pending.push_back({name, start, e});
}

}  // namespace umbir

using namespace umbir;

extern "C" {

void umbir_profile_enable(int on) { g_on.store(on != 0); }

void umbir_profile_select(const char* names) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_select.clear();
  if (names) {
    std::string cur;
    for (const char* p = names;; ++p) {
      if (*p == ',' || *p == '\0') {
        if (!cur.empty()) g_select.push_back(cur);
        cur.clear();
        if (*p == '\0') break;
      } else if (*p != ' ') {
        cur += *p;
      }
    }
  }
  g_seen.assign(g_select.size(), 0);
  g_filtered.store(!g_select.empty());
}

void umbir_profile_stride(int every) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_every = every > 1 ? every : 1;
  g_seen.assign(g_select.size(), 0);
}

int umbir_profile_collect(umbir_kernel_time* out, int max_entries, int* n_out) {
  if (max_entries < 0 || (max_entries > 0 && !out)) return fail(UMBIR_EINVAL, "bad output buffer");
  std::lock_guard<std::mutex> lk(g_mu);
  int st = UMBIR_OK;
  for (const Pending& p : g_pending) {
    float ms = 0.0f;
    hipError_t e = hipEventSynchronize(p.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.start, p.stop);
    if (e != hipSuccess && st == UMBIR_OK) st = check_hip(e, "umbir_profile_collect");
    Totals& t = g_totals[p.name];
    t.launches += 1;
    t.ms += ms;
    (void)hipEventDestroy(p.start);
    (void)hipEventDestroy(p.stop);
  }
  g_pending.clear();
  int n = 0;
  for (const auto& kv : g_totals) {
    if (n < max_entries) {
      std::memset(&out[n], 0, sizeof(umbir_kernel_time));
      std::strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
      out[n].launches = kv.second.launches;
      out[n].total_ms = kv.second.ms;
    }
    ++n;
  }
  if (n_out) *n_out = n;
  g_totals.clear();
  return st;
}

}  // extern "C"
