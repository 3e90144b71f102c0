// Launch-configuration autotuner: a process-wide table from a launch-shape key
// (kernel family, precision, sizes) to the index of the fastest candidate
// configuration.  While tuning is switched on, a launch site whose key has
// no entry times every candidate on the caller's stream (one warm-up launch,
// then three timed launches between hipEvents; this synchronises) and records
// the fastest (with PQ_TUNE_TRACE set in the environment each candidate's
// time is printed to stderr).  Otherwise, and always while the stream is
// being captured into a graph, the recorded choice or the site's default is
// used without any synchronisation.  The table can be saved to and loaded
// from a text file of "key choice" lines.
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>

#include "internal.hpp"

namespace pq {
namespace {

std::mutex g_mu;
bool g_on = false;
std::map<std::string, int>& table() {
  static std::map<std::string, int> t;
  return t;
}

}  // namespace

void tune_enable(bool on) {
  std::lock_guard<std::mutex> g(g_mu);
  g_on = on;
}

int tune_entries() {
  std::lock_guard<std::mutex> g(g_mu);
  return (int)table().size();
}

bool tune_save(const char* path) {
  std::lock_guard<std::mutex> g(g_mu);
  std::ofstream f(path);
  if (!f) return false;
  for (const auto& kv : table()) f << kv.first << ' ' << kv.second << '\n';
  return (bool)f;
}

bool tune_load(const char* path) {
  std::ifstream f(path);
  if (!f) return false;
  std::lock_guard<std::mutex> g(g_mu);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string key;
    int v;
    if (is >> key >> v) table()[key] = v;
  }
  return true;
}

hipError_t tuned_launch(const std::string& key, int ncand, int dflt, hipStream_t s,
                        const std::function<hipError_t(int)>& launch) {
  int choice = -1;
  bool tune = false;
  {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = table().find(key);
    if (it != table().end() && it->second >= 0 && it->second < ncand) choice = it->second;
    else tune = g_on && ncand > 1;
  }
  if (tune) {  // timing synchronises: never while the stream is being captured into a graph
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess || st != hipStreamCaptureStatusNone) tune = false;
  }
  if (choice < 0 && tune) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    float best = 0.f;
    for (int c = 0; c < ncand && err == hipSuccess; ++c) {
      if ((err = launch(c)) != hipSuccess) break;
      if ((err = hipEventRecord(e0, s)) != hipSuccess) break;
      for (int r = 0; r < 3 && err == hipSuccess; ++r) err = launch(c);
      if (err != hipSuccess) break;
      if ((err = hipEventRecord(e1, s)) != hipSuccess) break;
      if ((err = hipEventSynchronize(e1)) != hipSuccess) break;
      float ms = 0.f;
      if ((err = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
      if (std::getenv("PQ_TUNE_TRACE")) std::fprintf(stderr, "[pq tune] %s cand %d: %.2f us\n", key.c_str(), c, ms * 1000.f / 3);
      if (choice < 0 || ms < best) {
        best = ms;
        choice = c;
      }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (err != hipSuccess) return err;
    std::lock_guard<std::mutex> g(g_mu);
    table()[key] = choice;
  }
  if (choice < 0) choice = dflt;
  return launch(choice);
}

}  // namespace pq
