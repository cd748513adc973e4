// Drives the C ABI's host code (built with the stand-in launchers of
// stub_launchers.cpp) under AddressSanitizer and UndefinedBehaviorSanitizer:
// size queries over a range of sizes, valid calls whose carved workspaces
// the stand-ins check, and invalid calls that must be rejected.  Exit code 0
// and no sanitizer report = pass.  Test infrastructure only.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "tpcca.h"

namespace stub {
extern const char* g_ws;
extern size_t g_ws_bytes;
extern int g_calls;
}  // namespace stub

static int g_fail = 0;
#define EXPECT(cond)                                                   \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "%s:%d: expectation failed: %s\n", __FILE__,      \
              __LINE__, #cond);                                        \
      g_fail++;                                                        \
    }                                                                  \
  } while (0)

static tpc_geometry geom()
{
  tpc_geometry g;
  memset(&g, 0, sizeof(g));
  g.n_rows = TPC_N_ROWS;
  for (int r = 0; r < TPC_N_ROWS; r++) g.row_x[r] = (float)(85.0 + r * 162.0 / 151.0);
  g.bz_tesla = 0.5f;
  g.tan_half_sector = 0.17632698f;
  g.sigma_y2 = 0.01f;
  g.sigma_z2 = 0.0225f;
  return g;
}

// stand-in device pointer: never dereferenced by the host code
static void* fake(uintptr_t v) { return reinterpret_cast<void*>(v); }

static void grid_and_track(int32_t n_inst, const std::vector<int64_t>& off, float occ,
                           int64_t cap_tl)
{
  tpc_geometry g = geom();
  tpc_params p;
  tpc_default_params(&p);
  p.grid_occupancy = occ;
  const int64_t n = off[n_inst];
  const size_t gws = tpc_grid_workspace_bytes(&p, n_inst, n);
  const size_t tws = tpc_track_workspace_bytes(n_inst, n, cap_tl);
  std::vector<char> ws(gws > tws ? gws : tws);
  tpc_clusters in = {(const float*)fake(0x1000), (const float*)fake(0x1000),
                     (const float*)fake(0x1000), (const uint16_t*)fake(0x1000), nullptr};
  tpc_grid grid = {(int32_t*)fake(0x2000), (int32_t*)fake(0x2000), (tpc_row_meta*)fake(0x2000),
                   (int32_t*)fake(0x2000), (int32_t*)fake(0x2000), (float*)fake(0x2000),
                   tpc_grid_bin_capacity(&p, n_inst, n)};
  stub::g_ws = ws.data();
  stub::g_ws_bytes = gws;
  const int before = stub::g_calls;
  EXPECT(tpc_grid_build(&g, &p, n_inst, off.data(), (const int64_t*)fake(0x3000), in, &grid,
                        (tpc_result*)fake(0x4000), ws.data(), gws, nullptr) == TPC_OK);
  EXPECT(tpc_grid_build(&g, &p, n_inst, off.data(), (const int64_t*)fake(0x3000), in, &grid,
                        (tpc_result*)fake(0x4000), ws.data(), gws - 1, nullptr) ==
         TPC_ERR_WORKSPACE);
  tpc_tracks out = {(float*)fake(0x5000), (float*)fake(0x5000), (float*)fake(0x5000),
                    (int32_t*)fake(0x5000), (float*)fake(0x5000), (int32_t*)fake(0x5000),
                    (int32_t*)fake(0x5000), (int32_t*)fake(0x5000), 100, 1000};
  stub::g_ws_bytes = tws;
  for (int det = 0; det < 2; det++) {
    p.flags = det ? TPC_FLAG_DETERMINISTIC : 0u;
    EXPECT(tpc_sector_track(&g, &p, n_inst, off.data(), (const int64_t*)fake(0x3000), in, &grid,
                            &out, (tpc_result*)fake(0x4000), ws.data(), tws, cap_tl,
                            nullptr) == TPC_OK);
  }
  // optional per-hit data: 16-byte aligned or rejected
  out.hit_data = (float*)fake(0x6000);
  EXPECT(tpc_sector_track(&g, &p, n_inst, off.data(), (const int64_t*)fake(0x3000), in, &grid,
                          &out, (tpc_result*)fake(0x4000), ws.data(), tws, cap_tl,
                          nullptr) == TPC_OK);
  out.hit_data = (float*)fake(0x6008);
  EXPECT(tpc_sector_track(&g, &p, n_inst, off.data(), (const int64_t*)fake(0x3000), in, &grid,
                          &out, (tpc_result*)fake(0x4000), ws.data(), tws, cap_tl,
                          nullptr) == TPC_ERR_INVALID);
  out.hit_data = nullptr;
  EXPECT(tpc_sector_track(&g, &p, n_inst, off.data(), (const int64_t*)fake(0x3000), in, &grid,
                          &out, (tpc_result*)fake(0x4000), ws.data(), tws - 1, cap_tl,
                          nullptr) == TPC_ERR_WORKSPACE);
  EXPECT(stub::g_calls == before + 4);
  tpc_track_ws_layout lay;
  EXPECT(tpc_track_workspace_layout(n_inst, n, cap_tl, &lay) == TPC_OK);
  EXPECT(lay.total == (int64_t)tws);
}

static void invalid_calls()
{
  tpc_geometry g = geom();
  tpc_params p;
  tpc_default_params(&p);
  std::vector<int64_t> off = {0, 100};
  std::vector<char> ws(1 << 20);
  tpc_clusters in = {(const float*)fake(0x1000), (const float*)fake(0x1000),
                     (const float*)fake(0x1000), (const uint16_t*)fake(0x1000), nullptr};
  tpc_grid grid = {(int32_t*)fake(0x2000), (int32_t*)fake(0x2000), (tpc_row_meta*)fake(0x2000),
                   (int32_t*)fake(0x2000), (int32_t*)fake(0x2000), (float*)fake(0x2000), 1000};
  auto gb = [&](const tpc_geometry* gg, const tpc_params* pp, int32_t ni, const int64_t* o) {
    return tpc_grid_build(gg, pp, ni, o, (const int64_t*)fake(0x3000), in, &grid,
                          (tpc_result*)fake(0x4000), ws.data(), ws.size(), nullptr);
  };
  EXPECT(gb(nullptr, &p, 1, off.data()) == TPC_ERR_INVALID);
  EXPECT(gb(&g, nullptr, 1, off.data()) == TPC_ERR_INVALID);
  EXPECT(gb(&g, &p, 0, off.data()) == TPC_ERR_INVALID);
  tpc_params q = p;
  q.flags = 2u;
  EXPECT(gb(&g, &q, 1, off.data()) == TPC_ERR_INVALID);
  q = p;
  q.grid_occupancy = NAN;
  EXPECT(gb(&g, &q, 1, off.data()) == TPC_ERR_INVALID);
  q = p;
  q.snp_max = 1.5f;
  EXPECT(gb(&g, &q, 1, off.data()) == TPC_ERR_INVALID);
  tpc_geometry h = g;
  h.row_x[50] = NAN;
  EXPECT(gb(&h, &p, 1, off.data()) == TPC_ERR_INVALID);
  h = g;
  h.sigma_y2 = -1.0f;
  EXPECT(gb(&h, &p, 1, off.data()) == TPC_ERR_INVALID);
  std::vector<int64_t> big(17);
  for (int i = 0; i <= 16; i++) big[i] = (int64_t)i * ((1 << 24) - 1);
  q = p;
  q.grid_occupancy = 0.25f;
  EXPECT(gb(&g, &q, 16, big.data()) == TPC_ERR_INVALID);
  std::vector<int64_t> neg = {0, 10, 5};
  EXPECT(gb(&g, &p, 2, neg.data()) == TPC_ERR_INVALID);
  // refit
  tpc_refit_tracks trk = {(const int32_t*)fake(0x6000), (const int32_t*)fake(0x6000),
                          (const uint8_t*)fake(0x6000), (const float*)fake(0x6000), 10, 100};
  const float* dmap = (const float*)fake(0x7000);
  float* f = (float*)fake(0x8000);
  int32_t* st = (int32_t*)fake(0x8000);
  EXPECT(tpc_refit(&g, &p, 1000, in, trk, dmap, nullptr, f, st, f, nullptr) == TPC_OK);
  EXPECT(tpc_refit(&g, &p, (int64_t)1 << 31, in, trk, dmap, nullptr, f, st, f, nullptr) == TPC_ERR_INVALID);
  EXPECT(tpc_refit(&g, &p, 1000, in, trk, nullptr, nullptr, f, st, f, nullptr) == TPC_ERR_INVALID);
  q = p;
  q.flags = 4u;
  EXPECT(tpc_refit(&g, &q, 1000, in, trk, dmap, nullptr, f, st, f, nullptr) == TPC_ERR_INVALID);
  // field map and material: the z binning of a given field map is checked
  tpc_material mat = {(const float*)fake(0x7100), 0, (const float*)fake(0x7200), nullptr};
  EXPECT(tpc_refit(&g, &p, 1000, in, trk, dmap, &mat, f, st, f, nullptr) == TPC_ERR_INVALID);
  mat.nzb = 65537;
  EXPECT(tpc_refit(&g, &p, 1000, in, trk, dmap, &mat, f, st, f, nullptr) == TPC_ERR_INVALID);
  mat.nzb = 25;
  EXPECT(tpc_refit(&g, &p, 1000, in, trk, dmap, &mat, f, st, f, nullptr) == TPC_OK);
  mat.bz = nullptr;
  mat.nzb = 0;  // ignored without a field map
  EXPECT(tpc_refit(&g, &p, 1000, in, trk, dmap, &mat, f, st, f, nullptr) == TPC_OK);
  std::vector<char> rws(tpc_refit_workspace_bytes());
  stub::g_ws = rws.data();
  stub::g_ws_bytes = rws.size();
  EXPECT(tpc_refit_backward(&g, &p, 1000, in, trk, dmap, nullptr, f, st, f, f, f, f, f, rws.data(),
                            rws.size(), nullptr) == TPC_OK);
  EXPECT(tpc_refit_backward(&g, &p, 1000, in, trk, dmap, nullptr, f, st, f, f, f, f, f, rws.data(),
                            rws.size() - 1, nullptr) == TPC_ERR_WORKSPACE);
  EXPECT(tpc_refit_backward_noalloc(&g, &p, 1000, in, trk, dmap, nullptr, f, st, f, f, f, f, f,
                                    nullptr) == TPC_OK);
  EXPECT(tpc_refit_backward_noalloc(&g, &q, 1000, in, trk, dmap, nullptr, f, st, f, f, f, f, f,
                                    nullptr) == TPC_ERR_INVALID);
  EXPECT(tpc_refit_backward_noalloc(&g, &p, 1000, in, trk, dmap, nullptr, f, st, f, nullptr, f, f, f,
                                    nullptr) == TPC_ERR_INVALID);
  // cluster transformation
  tpc_transform_geometry tg;
  memset(&tg, 0, sizeof(tg));
  tg.nu = tg.nv = tg.nw = 2;
  tpc_raw_clusters raw = {(const uint8_t*)fake(0x9000), (const uint16_t*)fake(0x9000),
                          (const float*)fake(0x9000), (const float*)fake(0x9000)};
  const float* cm = (const float*)fake(0xA000);
  uint16_t* ro = (uint16_t*)fake(0xB000);
  EXPECT(tpc_cluster_transform(&tg, 1u, 1000, raw, dmap, cm, f, f, f, ro, nullptr) == TPC_OK);
  EXPECT(tpc_cluster_transform(&tg, 1u, 0, raw, nullptr, nullptr, nullptr, nullptr, nullptr,
                               nullptr, nullptr) == TPC_OK);
  EXPECT(tpc_cluster_transform(nullptr, 1u, 1000, raw, dmap, cm, f, f, f, ro, nullptr) ==
         TPC_ERR_INVALID);
  EXPECT(tpc_cluster_transform(&tg, 2u, 1000, raw, dmap, cm, f, f, f, ro, nullptr) ==
         TPC_ERR_INVALID);
  EXPECT(tpc_cluster_transform(&tg, 1u, -1, raw, dmap, cm, f, f, f, ro, nullptr) ==
         TPC_ERR_INVALID);
  EXPECT(tpc_cluster_transform(&tg, 1u, 1000, raw, dmap, cm, f, nullptr, f, ro, nullptr) ==
         TPC_ERR_INVALID);
  EXPECT(tpc_cluster_transform(&tg, 1u, 1000, raw, dmap, (const float*)fake(0xA004), f, f, f, ro,
                               nullptr) == TPC_ERR_INVALID);
  tg.nw = 1;
  EXPECT(tpc_cluster_transform(&tg, 1u, 1000, raw, dmap, cm, f, f, f, ro, nullptr) ==
         TPC_ERR_INVALID);
  // merging
  tpc_merge_params mp;
  tpc_default_merge_params(&mp);
  EXPECT(mp.cos_d > 0.93f && mp.cos_d < 0.94f && mp.sin_a[0] > 0.17f && mp.sin_a[0] < 0.18f);
  tpc_tracks seg = {(float*)fake(0xC000), (float*)fake(0xC000), (float*)fake(0xC000),
                    (int32_t*)fake(0xC000), (float*)fake(0xC000), (int32_t*)fake(0xC000),
                    (int32_t*)fake(0xC000), (int32_t*)fake(0xC000), 500, 20000};
  tpc_merged mo;
  memset(&mo, 0, sizeof(mo));
  mo.param = mo.cov = mo.chi2 = mo.x_ref = (float*)fake(0xD000);
  mo.ndf = mo.status = mo.sector = mo.hit_off = mo.hit_clu = mo.seg_off = mo.seg = mo.next =
      (int32_t*)fake(0xD000);
  mo.counts = (int64_t*)fake(0xD000);
  mo.cap_tracks = 500;
  mo.cap_hits = 20000;
  std::vector<char> mws(tpc_merge_workspace_bytes(500, 20000));
  EXPECT(tpc_merge_workspace_bytes(500, -1) == 0 && tpc_merge_workspace_bytes(-1, 20000) == 0);
  stub::g_ws = mws.data();
  stub::g_ws_bytes = mws.size();
  const int64_t* io = (const int64_t*)fake(0xE000);
  const tpc_result* rs = (const tpc_result*)fake(0xE000);
  EXPECT(tpc_merge_tracks(&g, &p, &mp, 36, io, in, &seg, rs, &mo, mws.data(), mws.size(),
                          nullptr) == TPC_OK);
  EXPECT(tpc_merge_tracks(&g, &p, &mp, 35, io, in, &seg, rs, &mo, mws.data(), mws.size(),
                          nullptr) == TPC_ERR_INVALID);
  EXPECT(tpc_merge_tracks(&g, &p, &mp, 36, io, in, &seg, rs, &mo, mws.data(), mws.size() - 1,
                          nullptr) == TPC_ERR_WORKSPACE);
  // optional per-hit data of the segments: 16-byte aligned or rejected
  seg.hit_data = (float*)fake(0xF000);
  EXPECT(tpc_merge_tracks(&g, &p, &mp, 36, io, in, &seg, rs, &mo, mws.data(), mws.size(),
                          nullptr) == TPC_OK);
  seg.hit_data = (float*)fake(0xF004);
  EXPECT(tpc_merge_tracks(&g, &p, &mp, 36, io, in, &seg, rs, &mo, mws.data(), mws.size(),
                          nullptr) == TPC_ERR_INVALID);
  seg.hit_data = nullptr;
  mo.cap_hits = 19999;
  EXPECT(tpc_merge_tracks(&g, &p, &mp, 36, io, in, &seg, rs, &mo, mws.data(), mws.size(),
                          nullptr) == TPC_ERR_INVALID);
  for (int s = 1; s >= -5; s--) EXPECT(tpc_status_string((tpc_status)s) != nullptr);
  EXPECT(tpc_standard_configuration(&g, &p) == 1);
  EXPECT(tpc_standard_configuration(nullptr, &p) == TPC_ERR_INVALID);
}

int main()
{
  // sizes: empty, one instance, many small instances, ragged, one at the
  // per-instance limit; default and explicit tracklet capacities
  grid_and_track(1, {0, 0}, 2.0f, 0);
  grid_and_track(1, {0, 7}, 2.0f, 0);
  grid_and_track(3, {0, 1000, 1000, 25000}, 0.5f, 0);
  grid_and_track(2, {0, 5000, 9000}, 1.0f, 17);
  std::vector<int64_t> many(401);
  for (int i = 0; i <= 400; i++) many[i] = (int64_t)i * 37 + (i * i) % 11;
  grid_and_track(400, many, 2.0f, 0);
  grid_and_track(1, {0, (1 << 24) - 1}, 2.0f, 0);
  invalid_calls();
  for (int64_t n : {0LL, 1LL, 1000LL, 123457LL, 20000000LL}) {
    tpc_params p;
    tpc_default_params(&p);
    EXPECT(tpc_grid_bin_capacity(&p, 36, n) >= 5 * n / 2);
    EXPECT(tpc_track_workspace_bytes(36, n, 0) > 0);
  }
  if (g_fail) {
    fprintf(stderr, "%d expectation(s) failed\n", g_fail);
    return 1;
  }
  printf("abi harness ok (%d launcher calls)\n", stub::g_calls);
  return 0;
}
