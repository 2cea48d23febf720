// Kernel timers: event pairs per named launch, summed on read.
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "profile.hpp"

namespace yr {

namespace {
struct Pair {
  hipEvent_t a, b;
  int name;
};
std::mutex g_mu;
bool g_on = false;
std::vector<std::string> g_select;  // names timed while on (empty: all)
std::vector<std::string> g_names;
std::vector<Pair> g_pairs;   // recorded, not yet resolved
std::vector<Pair> g_free;    // reusable events
std::map<std::string, std::pair<long long, double>> g_acc;  // name -> (launches, ms)

int name_id(const char* n) {
  for (size_t i = 0; i < g_names.size(); ++i)
    if (g_names[i] == n) return (int)i;
  g_names.emplace_back(n);
  return (int)g_names.size() - 1;
}

void resolve_locked() {
  for (auto& p : g_pairs) {
    float ms = 0;
    if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      auto& acc = g_acc[g_names[p.name]];
      acc.first += 1;
      acc.second += ms;
    }
    g_free.push_back(p);
  }
  g_pairs.clear();
}
}  // namespace

bool prof_on() { return g_on; }

int prof_begin(const char* name, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_on) return -1;
  if (!g_select.empty()) {
    bool hit = false;
    for (const auto& n : g_select) hit = hit || n == name;
    if (!hit) return -1;
  }
  if (g_pairs.size() >= 16384) resolve_locked();
  Pair p;
  if (!g_free.empty()) {
    p = g_free.back();
    g_free.pop_back();
  } else {
    if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) return -1;
  }
  p.name = name_id(name);
  (void)hipEventRecord(p.a, s);
  g_pairs.push_back(p);
  return (int)g_pairs.size() - 1;
}

void prof_end(int slot, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (slot < 0 || slot >= (int)g_pairs.size()) return;
  (void)hipEventRecord(g_pairs[slot].b, s);
}

}  // namespace yr

using namespace yr;

extern "C" {

int yr_profile_enable(int on) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!on) resolve_locked();
  g_on = on != 0;
  return YR_OK;
}

int yr_profile_select(const char* names) {
  std::lock_guard<std::mutex> lk(g_mu);
  g_select.clear();
  if (!names) return YR_OK;
  std::string all(names), cur;
  for (char c : all + ",") {
    if (c == ',') {
      if (!cur.empty()) g_select.push_back(cur);
      cur.clear();
    } else {
      cur += c;
    }
  }
  return YR_OK;
}

int yr_profile_reset(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  resolve_locked();
  g_acc.clear();
  return YR_OK;
}

int yr_profile_read(const char* name, int64_t* launches, double* ms) {
  YR_REQUIRE(name && launches && ms, YR_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(g_mu);
  resolve_locked();
  auto it = g_acc.find(name);
  *launches = it == g_acc.end() ? 0 : it->second.first;
  *ms = it == g_acc.end() ? 0.0 : it->second.second;
  return YR_OK;
}

}  // extern "C"
