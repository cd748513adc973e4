// Per-kernel event timing behind tpc_profile_enable / tpc_profile_read.
#include <string.h>

#include <map>
#include <string>
#include <vector>

#include "tpc_internal.h"

namespace {

constexpr int kPool = 16384;  // event pairs

struct Rec {
  const char* name;
  hipEvent_t a, b;
};

bool g_on = false;
std::vector<hipEvent_t> g_ev;
std::vector<Rec> g_rec;
int g_next = 0;

}  // namespace

namespace tpcca {

int prof_begin(hipStream_t s, const char* name)
{
  if (!g_on || g_next + 2 > (int)g_ev.size()) return -1;
  Rec r{name, g_ev[g_next], g_ev[g_next + 1]};
  g_next += 2;
  if (hipEventRecord(r.a, s) != hipSuccess) return -1;
  g_rec.push_back(r);
  return (int)g_rec.size() - 1;
}

void prof_end(hipStream_t s, int slot)
{
  if (slot >= 0) (void)hipEventRecord(g_rec[slot].b, s);
}

}  // namespace tpcca

extern "C" {

tpc_status tpc_profile_enable(int32_t on)
{
  if (on && !g_on) {
    g_ev.assign(2 * kPool, nullptr);
    for (size_t i = 0; i < g_ev.size(); i++)
      if (hipEventCreate(&g_ev[i]) != hipSuccess) {
        // leave the timer off, holding no events
        for (size_t j = 0; j < i; j++) (void)hipEventDestroy(g_ev[j]);
        g_ev.clear();
        return TPC_ERR_HIP;
      }
    g_rec.clear();
    g_next = 0;
    g_on = true;
  } else if (!on && g_on) {
    (void)hipDeviceSynchronize();
    for (auto& e : g_ev) (void)hipEventDestroy(e);
    g_ev.clear();
    g_rec.clear();
    g_next = 0;
    g_on = false;
  }
  return TPC_OK;
}

int32_t tpc_profile_read(tpc_kernel_time* out, int32_t max_entries)
{
  if (!out || max_entries < 0) return TPC_ERR_INVALID;
  std::map<std::string, std::pair<double, int64_t>> acc;
  for (const Rec& r : g_rec) {
    if (hipEventSynchronize(r.b) != hipSuccess) return TPC_ERR_HIP;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return TPC_ERR_HIP;
    auto& v = acc[r.name];
    v.first += ms;
    v.second += 1;
  }
  g_rec.clear();
  g_next = 0;
  int32_t n = 0;
  for (const auto& kv : acc) {
    if (n >= max_entries) break;
    memset(out[n].name, 0, sizeof(out[n].name));
    strncpy(out[n].name, kv.first.c_str(), sizeof(out[n].name) - 1);
    out[n].total_ms = kv.second.first;
    out[n].launches = kv.second.second;
    n++;
  }
  return n;
}

}  // extern "C"
