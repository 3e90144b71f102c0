// Per-launch timing behind pq_profile_*: while enabled, every launch the
// library makes inside a ProfScope is bracketed by two hipEvents recorded on
// the caller's stream (not while that stream is being captured into a graph).
// A scope may cover several back-to-back launches of one kernel (the sweeps
// of the Jacobi): one event pair then brackets all of them, so that short
// launches are not stretched by events between them, and the scope counts
// as that many launches.  Events come from a pool that grows on demand and is
// reused after a reset.
#include <cstring>
#include <mutex>
#include <vector>

#include "internal.hpp"

namespace pq {
namespace {

struct Rec {
  const char* name;
  hipEvent_t a, b;
  int count;  // launches the bracket covers
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

thread_local int t_mute = 0;

ProfMute::ProfMute() { ++t_mute; }
ProfMute::~ProfMute() { --t_mute; }

ProfScope::ProfScope(const char* name, hipStream_t s, int launches) : name_(name), s_(s), count_(launches) {
  if (t_mute > 0) return;
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_on) return;
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;  // no events inside a captured graph
  if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) return;
  a_ = take_event();
  if (a_) hipEventRecord(a_, s_);
}

ProfScope::~ProfScope() {
  if (!a_) return;
  std::lock_guard<std::mutex> g(g_mu);
  hipEvent_t b = take_event();
  if (!b) {
    g_pool.push_back(a_);
    return;
  }
  hipEventRecord(b, s_);
  g_recs.push_back({name_, a_, b, count_});
}

void prof_enable(bool on) {
  std::lock_guard<std::mutex> g(g_mu);
  g_on = on;
}

void prof_reset() {
  std::lock_guard<std::mutex> g(g_mu);
  for (Rec& r : g_recs) {
    g_pool.push_back(r.a);
    g_pool.push_back(r.b);
  }
  g_recs.clear();
}

hipError_t prof_query(const char* name, double* total_ms, int* launches) {
  std::lock_guard<std::mutex> g(g_mu);
  double tot = 0.0;
  int n = 0;
  for (const Rec& r : g_recs) {
    if (std::strcmp(r.name, name) != 0) continue;
    hipError_t e = hipEventSynchronize(r.b);
    if (e != hipSuccess) return e;
    float ms = 0.f;
    e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess) return e;
    tot += ms;
    n += r.count;
  }
  *total_ms = tot;
  *launches = n;
  return hipSuccess;
}

bool prof_names(char* buf, size_t len) {
  std::lock_guard<std::mutex> g(g_mu);
  std::vector<const char*> seen;
  for (const Rec& r : g_recs) {
    bool dup = false;
    for (const char* q : seen) dup |= std::strcmp(q, r.name) == 0;
    if (!dup) seen.push_back(r.name);
  }
  size_t pos = 0;
  buf[0] = 0;
  for (const char* q : seen) {
    const size_t l = std::strlen(q);
    if (pos + l + 2 > len) return false;
    if (pos) buf[pos++] = ',';
    std::memcpy(buf + pos, q, l);
    pos += l;
    buf[pos] = 0;
  }
  return true;
}

}  // namespace pq
