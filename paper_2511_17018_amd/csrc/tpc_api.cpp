// Host side of the C ABI declared in include/tpcca.h: argument validation,
// workspace carving, derived constants, dispatch to the deterministic or
// production build of the kernels.  Allocates nothing.
#include <math.h>
#include <string.h>

#include "tpc_defaults.h"
#include "tpc_internal.h"

using namespace tpcca;

extern "C" int64_t tpc_grid_bin_capacity(const tpc_params* params, int32_t n_inst,
                                         int64_t n_clusters);

namespace {

constexpr int64_t kAlign = 256;
constexpr int64_t kScanTile = 2048;  // items per block of the scan kernels
constexpr int64_t kMaxInstClusters = (int64_t)1 << 24;
constexpr uint32_t kKnownFlags =
    TPC_FLAG_DETERMINISTIC | TPC_FLAG_GENERIC | TPC_FLAG_COUNT_CANDIDATES;

int64_t align_up(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Carve {
  int64_t off = 0;
  int64_t take(int64_t bytes)
  {
    int64_t o = off;
    off = align_up(off + (bytes > 0 ? bytes : 0));
    return o;
  }
};

int64_t default_cap(int32_t n_inst, int64_t n) { return n / 3 + n_inst; }

struct GridWs {
  int64_t cseg, seg_cnt, seg_mm, inst_bad, nb1, fill, seg_pos, seg_cursor, tmp_perm, tmp_yz;
  int64_t scan_tmp, scan_len, total;
};

GridWs grid_ws(const tpc_params* p, int32_t n_inst, int64_t n)
{
  const int64_t n_seg = (int64_t)n_inst * kRows;
  const int64_t bin_cap = tpc_grid_bin_capacity(p, n_inst, n);
  GridWs w;
  Carve c;
  w.cseg = c.take(4 * n);
  w.seg_cnt = c.take(4 * n_seg);
  w.seg_mm = c.take(16 * n_seg);
  w.inst_bad = c.take(4 * (int64_t)n_inst);
  w.nb1 = c.take(4 * n_seg);
  w.fill = c.take(4 * bin_cap);
  w.seg_pos = c.take(4 * n_seg);
  w.seg_cursor = c.take(4 * n_seg);
  w.tmp_perm = c.take(4 * n);
  w.tmp_yz = c.take(8 * n);
  const int64_t big = bin_cap > n_seg ? bin_cap : n_seg;
  w.scan_len = big / kScanTile + 2;
  w.scan_tmp = c.take(8 * w.scan_len);
  w.total = c.off;
  return w;
}

struct TrackWs {
  tpc_track_ws_layout pub;
  int64_t tl_own, tsv, tl_first, chunk_off, tl_key, tl_owned, own_t, tl_rec, start_flag,
      counters, scan_len;
};

TrackWs track_ws(int32_t n_inst, int64_t n, int64_t cap)
{
  if (cap <= 0) cap = default_cap(n_inst, n);
  TrackWs w;
  Carve c;
  w.pub.up = c.take(4 * n);
  w.pub.dn = c.take(4 * n);
  w.pub.up2 = c.take(4 * n);
  w.pub.dn2 = c.take(4 * n);
  w.pub.start = c.take(4 * cap);
  w.pub.tl_par = c.take(4 * 5 * cap);
  w.pub.tl_cov = c.take(4 * 15 * cap);
  w.pub.tl_chi2 = c.take(4 * cap);
  w.pub.tl_nhit = c.take(4 * cap);
  w.pub.tl_rmin = c.take(4 * cap);
  w.pub.tl_rmax = c.take(4 * cap);
  w.pub.tl_status = c.take(4 * cap);
  w.pub.tl_hit = c.take(4 * (int64_t)kRows * cap);
  w.pub.tl_ncand = c.take(4 * cap);
  w.pub.owner = c.take(8 * n);
  w.tl_own = c.take(4 * cap);
  w.tsv = c.take(8 * cap);
  w.tl_first = c.take(8 * ((int64_t)n_inst + 1));
  w.chunk_off = c.take(8 * ((int64_t)n_inst + 1));
  w.tl_key = c.take(8 * cap);
  w.tl_owned = c.take((int64_t)kRows * cap);
  w.own_t = c.take(4 * n);
  w.tl_rec = c.take(32 * cap);
  w.start_flag = c.take((n + kScanTile - 1) / kScanTile * kScanTile);
  w.counters = c.take(8 * 8);
  const int64_t big = n > cap ? n : cap;
  w.scan_len = big / kScanTile + 2;
  w.pub.scratch = c.take(8 * w.scan_len);
  w.pub.total = c.off;
  w.pub.cap_tracklets = cap;
  return w;
}

tpc_status check_common(const tpc_geometry* g, const tpc_params* p, int32_t n_inst,
                        const int64_t* off_h, const int64_t* off_d, const tpc_clusters& in,
                        int64_t* n_out)
{
  if (!g || !p || !off_h || !off_d || n_inst < 1) return TPC_ERR_INVALID;
  if (g->n_rows != kRows) return TPC_ERR_INVALID;
  for (int r = 0; r + 1 < kRows; r++)
    if (!(g->row_x[r + 1] > g->row_x[r])) return TPC_ERR_INVALID;
  if (!(g->sigma_y2 > 0) || !(g->sigma_z2 > 0) || !(g->tan_half_sector > 0)) return TPC_ERR_INVALID;
  if (off_h[0] != 0) return TPC_ERR_INVALID;
  for (int32_t i = 0; i < n_inst; i++) {
    int64_t sz = off_h[i + 1] - off_h[i];
    if (sz < 0 || sz >= kMaxInstClusters) return TPC_ERR_INVALID;
  }
  const int64_t n = off_h[n_inst];
  if (n >= ((int64_t)1 << 31) - 1) return TPC_ERR_INVALID;
  if (n > 0 && (!in.y || !in.z || !in.row)) return TPC_ERR_INVALID;
  if (p->flags & ~kKnownFlags) return TPC_ERR_INVALID;
  // bin bases and offsets are 32-bit: the table the size query asks for
  // must fit
  if (tpc_grid_bin_capacity(p, n_inst, n) > (int64_t)INT32_MAX) return TPC_ERR_INVALID;
  if (p->min_chain < 3 || p->tc_max_miss < 1 || p->min_track_hits < 1 ||
      p->min_tracklet_hits < 0 || !(p->grid_occupancy > 0) || !(p->snp_max > 0) ||
      !(p->snp_max < 1) || !(p->search_margin >= 0) ||
      (p->tl_chunk != 0 && p->tl_chunk != 64 && p->tl_chunk != 128 && p->tl_chunk != 256))
    return TPC_ERR_INVALID;
  *n_out = n;
  return TPC_OK;
}

Consts make_consts(const tpc_geometry* g, const tpc_params* p)
{
  Consts k;
  memcpy(k.row_x, g->row_x, sizeof(k.row_x));
  k.tan_half = g->tan_half_sector;
  // derived once in binary64 and rounded (the CPU reference does the same)
  k.kB = (float)(-0.299792458e-2 * (double)g->bz_tesla);
  k.bz = g->bz_tesla;
  k.vy = g->sigma_y2;
  k.vz = g->sigma_z2;
  k.ivy = (float)(1.0 / (1.5 * (double)g->sigma_y2));
  k.ivz = (float)(1.0 / (1.5 * (double)g->sigma_z2));
  k.nf_win_y = p->nf_win_y;
  k.nf_win_z = p->nf_win_z;
  k.nf_chi2_max = p->nf_chi2_max;
  k.tc_chi2_pick = p->tc_chi2_pick;
  k.snp_max = p->snp_max;
  k.grid_occupancy = p->grid_occupancy;
  k.edge_margin = p->edge_margin;
  k.search_margin = p->search_margin;
  k.y_valid_margin = p->y_valid_margin;
  k.min_chain = p->min_chain;
  k.tc_max_miss = p->tc_max_miss;
  k.min_tracklet_hits = p->min_tracklet_hits;
  k.min_track_hits = p->min_track_hits;
  k.tl_chunk = p->tl_chunk > 0 ? p->tl_chunk : 256;
  return k;
}

// A call's constants equal the standard configuration's bit for bit (the
// performance-only fields aside): the kernels instantiated for it may run.
bool is_standard(const Consts& k)
{
  Consts a = k;
  a.grid_occupancy = kStdConsts.grid_occupancy;
  a.tl_chunk = kStdConsts.tl_chunk;
  return memcmp(&a, &kStdConsts, sizeof(Consts)) == 0;
}

template <class T>
T* at(void* base, int64_t off)
{
  return reinterpret_cast<T*>(static_cast<char*>(base) + off);
}

}  // namespace

extern "C" {

void tpc_default_params(tpc_params* p)
{
  if (!p) return;
  p->nf_win_y = 3.0f;
  p->nf_win_z = 3.5f;
  p->nf_chi2_max = 13.8f;
  p->tc_chi2_pick = 13.8f;
  p->snp_max = 0.99f;
  p->grid_occupancy = 2.0f;
  p->edge_margin = 1.0f;
  p->search_margin = 0.01f;
  p->y_valid_margin = 2.0f;
  p->min_chain = 3;
  p->tc_max_miss = 10;
  p->min_tracklet_hits = 10;
  p->min_track_hits = 10;
  p->flags = 0;
  p->tl_chunk = 0;
}

int32_t tpc_standard_configuration(const tpc_geometry* geom, const tpc_params* params)
{
  if (!geom || !params) return TPC_ERR_INVALID;
  if (geom->n_rows != kRows) return 0;
  return !(params->flags & TPC_FLAG_GENERIC) && is_standard(make_consts(geom, params)) ? 1 : 0;
}

const char* tpc_status_string(tpc_status s)
{
  switch (s) {
    case TPC_OK: return "ok";
    case TPC_ERR_INVALID: return "invalid argument";
    case TPC_ERR_UNSUPPORTED: return "unsupported mode";
    case TPC_ERR_HIP: return "HIP runtime error";
    case TPC_ERR_WORKSPACE: return "workspace too small";
  }
  return "unknown status";
}

int64_t tpc_grid_bin_capacity(const tpc_params* params, int32_t n_inst, int64_t n_clusters)
{
  // A row of n clusters has nb = max(1, floor(n / occupancy)) and a bin width w
  // with dy*dz/w^2 <= nb, dy/w <= nb, dz/w <= nb, so with one step of rounding
  // in each ceil: ny*nz <= (dy/w + 2)(dz/w + 2) <= 5 nb + 4; plus a sentinel.
  const double occ = params && params->grid_occupancy > 0 ? params->grid_occupancy : 2.0;
  const int64_t rows = (int64_t)kRows * (n_inst > 0 ? n_inst : 0);
  return (int64_t)ceil(5.0 * (double)n_clusters / occ) + 10 * rows + 16;
}

size_t tpc_grid_workspace_bytes(const tpc_params* params, int32_t n_inst, int64_t n_clusters)
{
  if (n_inst < 1 || n_clusters < 0) return 0;
  return (size_t)grid_ws(params, n_inst, n_clusters).total;
}

size_t tpc_track_workspace_bytes(int32_t n_inst, int64_t n_clusters, int64_t cap_tracklets)
{
  if (n_inst < 1 || n_clusters < 0) return 0;
  return (size_t)track_ws(n_inst, n_clusters, cap_tracklets).pub.total;
}

tpc_status tpc_track_workspace_layout(int32_t n_inst, int64_t n_clusters, int64_t cap_tracklets,
                                      tpc_track_ws_layout* out)
{
  if (!out || n_inst < 1 || n_clusters < 0) return TPC_ERR_INVALID;
  *out = track_ws(n_inst, n_clusters, cap_tracklets).pub;
  return TPC_OK;
}

tpc_status tpc_grid_build(const tpc_geometry* geom, const tpc_params* params, int32_t n_inst,
                          const int64_t* inst_off_host, const int64_t* inst_off_dev,
                          tpc_clusters in, const tpc_grid* grid, tpc_result* result_dev,
                          void* ws_dev, size_t ws_bytes, void* stream)
{
  int64_t n = 0;
  tpc_status st = check_common(geom, params, n_inst, inst_off_host, inst_off_dev, in, &n);
  if (st != TPC_OK) return st;
  if (!grid || !result_dev || !ws_dev) return TPC_ERR_INVALID;
  if (n > 0 && (!grid->sseg || !grid->perm || !grid->yz)) return TPC_ERR_INVALID;
  if (reinterpret_cast<uintptr_t>(grid->yz) % 8) return TPC_ERR_INVALID;
  if (!grid->row_off || !grid->meta || !grid->bin_off || grid->bin_cap < 1) return TPC_ERR_INVALID;
  const GridWs w = grid_ws(params, n_inst, n);
  if ((int64_t)ws_bytes < w.total) return TPC_ERR_WORKSPACE;
  GridBufs b;
  b.x = in.x;
  b.y = in.y;
  b.z = in.z;
  b.row = in.row;
  b.inst_off = inst_off_dev;
  b.n_inst = n_inst;
  b.n = n;
  b.sseg = grid->sseg;
  b.row_off = grid->row_off;
  b.meta = grid->meta;
  b.bin_off = grid->bin_off;
  b.perm = grid->perm;
  b.yz = reinterpret_cast<float2*>(grid->yz);
  // the workspace's fill counters and scan partials are sized for this capacity
  const int64_t ws_cap = tpc_grid_bin_capacity(params, n_inst, n);
  b.bin_cap = grid->bin_cap < ws_cap ? grid->bin_cap : ws_cap;
  b.res = result_dev;
  b.cseg = at<int32_t>(ws_dev, w.cseg);
  b.seg_cnt = at<int32_t>(ws_dev, w.seg_cnt);
  b.seg_mm = at<uint32_t>(ws_dev, w.seg_mm);
  b.inst_bad = at<int32_t>(ws_dev, w.inst_bad);
  b.nb1 = at<int32_t>(ws_dev, w.nb1);
  b.fill = at<int32_t>(ws_dev, w.fill);
  b.seg_pos = at<int32_t>(ws_dev, w.seg_pos);
  b.seg_cursor = at<int32_t>(ws_dev, w.seg_cursor);
  b.tmp_perm = at<int32_t>(ws_dev, w.tmp_perm);
  b.tmp_yz = at<float2>(ws_dev, w.tmp_yz);
  b.scan_tmp = at<int64_t>(ws_dev, w.scan_tmp);
  b.scan_tmp_len = w.scan_len;
  const Consts k = make_consts(geom, params);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = (params->flags & TPC_FLAG_DETERMINISTIC) ? det::grid_build(k, b, s)
                                                           : prod::grid_build(k, b, s);
  return e == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

tpc_status tpc_sector_track(const tpc_geometry* geom, const tpc_params* params, int32_t n_inst,
                            const int64_t* inst_off_host, const int64_t* inst_off_dev,
                            tpc_clusters in, const tpc_grid* grid, const tpc_tracks* out,
                            tpc_result* result_dev, void* ws_dev, size_t ws_bytes,
                            int64_t cap_tracklets, void* stream)
{
  int64_t n = 0;
  tpc_status st = check_common(geom, params, n_inst, inst_off_host, inst_off_dev, in, &n);
  if (st != TPC_OK) return st;
  if (!grid || !out || !result_dev || !ws_dev) return TPC_ERR_INVALID;
  if (n > 0 && (!grid->sseg || !grid->perm || !grid->yz || !out->clu2trk))
    return TPC_ERR_INVALID;
  if (!grid->row_off || !grid->meta || !grid->bin_off) return TPC_ERR_INVALID;
  if (out->cap_tracks < 0 || out->cap_hits < 0 || !out->hit_off) return TPC_ERR_INVALID;
  if (out->cap_tracks > 0 && (!out->param || !out->cov || !out->chi2 || !out->ndf || !out->x_ref))
    return TPC_ERR_INVALID;
  if (out->cap_hits > 0 && !out->hit_clu) return TPC_ERR_INVALID;
  if (out->hit_data && reinterpret_cast<uintptr_t>(out->hit_data) % 16) return TPC_ERR_INVALID;
  if (out->cap_tracks >= ((int64_t)1 << 31) || out->cap_hits >= ((int64_t)1 << 31))
    return TPC_ERR_INVALID;
  const TrackWs w = track_ws(n_inst, n, cap_tracklets);
  if ((int64_t)ws_bytes < w.pub.total) return TPC_ERR_WORKSPACE;
  TrackBufs b;
  b.inst_off = inst_off_dev;
  b.n_inst = n_inst;
  b.n = n;
  b.sseg = grid->sseg;
  b.row_off = grid->row_off;
  b.meta = grid->meta;
  b.bin_off = grid->bin_off;
  b.perm = grid->perm;
  if (reinterpret_cast<uintptr_t>(grid->yz) % 8) return TPC_ERR_INVALID;
  b.yz = reinterpret_cast<const float2*>(grid->yz);
  b.up = at<int32_t>(ws_dev, w.pub.up);
  b.dn = at<int32_t>(ws_dev, w.pub.dn);
  b.up2 = at<int32_t>(ws_dev, w.pub.up2);
  b.dn2 = at<int32_t>(ws_dev, w.pub.dn2);
  b.start = at<int32_t>(ws_dev, w.pub.start);
  b.cap = w.pub.cap_tracklets;
  b.tl_par = at<float>(ws_dev, w.pub.tl_par);
  b.tl_cov = at<float>(ws_dev, w.pub.tl_cov);
  b.tl_chi2 = at<float>(ws_dev, w.pub.tl_chi2);
  b.tl_nhit = at<int32_t>(ws_dev, w.pub.tl_nhit);
  b.tl_rmin = at<int32_t>(ws_dev, w.pub.tl_rmin);
  b.tl_rmax = at<int32_t>(ws_dev, w.pub.tl_rmax);
  b.tl_status = at<int32_t>(ws_dev, w.pub.tl_status);
  b.tl_hit = at<int32_t>(ws_dev, w.pub.tl_hit);
  b.tl_ncand = at<int32_t>(ws_dev, w.pub.tl_ncand);
  b.owner = at<unsigned long long>(ws_dev, w.pub.owner);
  b.tl_own = at<int32_t>(ws_dev, w.tl_own);
  b.tsv = at<int64_t>(ws_dev, w.tsv);
  b.tl_first = at<int64_t>(ws_dev, w.tl_first);
  b.chunk_off = at<int64_t>(ws_dev, w.chunk_off);
  b.tl_key = at<unsigned long long>(ws_dev, w.tl_key);
  b.tl_owned = at<uint8_t>(ws_dev, w.tl_owned);
  b.own_t = at<int32_t>(ws_dev, w.own_t);
  b.tl_rec = at<int4>(ws_dev, w.tl_rec);
  b.start_flag = at<unsigned long long>(ws_dev, w.start_flag);
  b.counters = at<int64_t>(ws_dev, w.counters);
  b.scan_tmp = at<int64_t>(ws_dev, w.pub.scratch);
  b.scan_tmp_len = w.scan_len;
  b.count_candidates = (params->flags & TPC_FLAG_COUNT_CANDIDATES) != 0;
  b.out = *out;
  b.res = result_dev;
  const Consts k = make_consts(geom, params);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const bool std_cfg = !(params->flags & TPC_FLAG_GENERIC) && is_standard(k);
  hipError_t e = (params->flags & TPC_FLAG_DETERMINISTIC) ? det::sector_track(k, b, std_cfg, s)
                                                           : prod::sector_track(k, b, std_cfg, s);
  return e == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

size_t tpc_refit_workspace_bytes(void) { return bwd::refit_scratch_bytes(); }

static tpc_status refit_check(const tpc_geometry* g, const tpc_params* p, int64_t n_clusters,
                              const tpc_clusters& in, const tpc_refit_tracks& trk,
                              const float* dmap)
{
  if (!g || !p || g->n_rows != kRows || n_clusters < 0 || trk.n_tracks < 0 || trk.n_hits < 0)
    return TPC_ERR_INVALID;
  // cluster indices are 32-bit
  if (n_clusters >= ((int64_t)1 << 31) || (p->flags & ~kKnownFlags)) return TPC_ERR_INVALID;
  if (!dmap || !(p->snp_max > 0) || !(p->snp_max < 1)) return TPC_ERR_INVALID;
  if (trk.n_tracks > 0 && (!trk.hit_off || !trk.seed)) return TPC_ERR_INVALID;
  if (trk.n_hits > 0 && (!trk.hit_clu || !trk.sector || !in.x || !in.y || !in.z || !in.row))
    return TPC_ERR_INVALID;
  return TPC_OK;
}

// the field map's z binning must give at least one bin
static bool material_ok(const tpc_material* m)
{
  return !m || !m->bz || (m->nzb >= 1 && m->nzb <= 65536);
}

static void set_material(RefitBufs& b, const tpc_material* m)
{
  if (!m) return;
  b.bz = m->bz;
  b.nzb = m->bz ? m->nzb : 0;
  b.ix0 = m->ix0;
  b.eloss = m->eloss;
}

static RefitBufs refit_bufs(int64_t n_clusters, const tpc_clusters& in, const tpc_refit_tracks& trk,
                            const float* dmap)
{
  RefitBufs b;
  memset(&b, 0, sizeof(b));
  b.x = in.x;
  b.y = in.y;
  b.z = in.z;
  b.row = in.row;
  b.sector = trk.sector;
  b.hit_off = trk.hit_off;
  b.hit_clu = trk.hit_clu;
  b.seed = trk.seed;
  b.dmap = dmap;
  b.n_tracks = trk.n_tracks;
  b.n_clusters = n_clusters;
  return b;
}

tpc_status tpc_refit(const tpc_geometry* geom, const tpc_params* params, int64_t n_clusters,
                     tpc_clusters in, tpc_refit_tracks trk, const float* dist_map_dev,
                     const tpc_material* mat, float* chi2_dev, int32_t* status_dev,
                     float* ckpt_dev, void* stream)
{
  tpc_status st = refit_check(geom, params, n_clusters, in, trk, dist_map_dev);
  if (st != TPC_OK) return st;
  if (!material_ok(mat)) return TPC_ERR_INVALID;
  if (trk.n_tracks > 0 && (!chi2_dev || !status_dev)) return TPC_ERR_INVALID;
  if (trk.n_hits > 0 && (!ckpt_dev || reinterpret_cast<uintptr_t>(ckpt_dev) % 16))
    return TPC_ERR_INVALID;
  RefitBufs b = refit_bufs(n_clusters, in, trk, dist_map_dev);
  set_material(b, mat);
  b.chi2 = chi2_dev;
  b.status = status_dev;
  b.ckpt = ckpt_dev;
  const Consts k = make_consts(geom, params);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = (params->flags & TPC_FLAG_DETERMINISTIC) ? det::refit_forward(k, b, s)
                                                           : prod::refit_forward(k, b, s);
  return e == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

static tpc_status refit_backward_check(const tpc_geometry* geom, const tpc_params* params,
                                       int64_t n_clusters, const tpc_clusters& in,
                                       const tpc_refit_tracks& trk, const float* dist_map_dev,
                                       const tpc_material* mat,
                                       const float* ckpt_dev, const int32_t* status_dev,
                                       const float* grad_chi2_dev, const float* grad_map_dev,
                                       const float* grad_x_dev, const float* grad_y_dev,
                                       const float* grad_z_dev)
{
  tpc_status st = refit_check(geom, params, n_clusters, in, trk, dist_map_dev);
  if (st != TPC_OK) return st;
  if (!material_ok(mat)) return TPC_ERR_INVALID;
  if (!grad_map_dev) return TPC_ERR_INVALID;
  if (trk.n_tracks > 0 && (!status_dev || !grad_chi2_dev)) return TPC_ERR_INVALID;
  if (trk.n_hits > 0 && (!ckpt_dev || reinterpret_cast<uintptr_t>(ckpt_dev) % 16))
    return TPC_ERR_INVALID;
  if (n_clusters > 0 && (!grad_x_dev || !grad_y_dev || !grad_z_dev)) return TPC_ERR_INVALID;
  return TPC_OK;
}

tpc_status tpc_refit_backward_noalloc(const tpc_geometry* geom, const tpc_params* params,
                                      int64_t n_clusters, tpc_clusters in, tpc_refit_tracks trk,
                                      const float* dist_map_dev, const tpc_material* mat,
                                      const float* ckpt_dev,
                                      const int32_t* status_dev, const float* grad_chi2_dev,
                                      float* grad_map_dev, float* grad_x_dev, float* grad_y_dev,
                                      float* grad_z_dev, void* stream)
{
  tpc_status st = refit_backward_check(geom, params, n_clusters, in, trk, dist_map_dev, mat,
                                       ckpt_dev,
                                       status_dev, grad_chi2_dev, grad_map_dev, grad_x_dev,
                                       grad_y_dev, grad_z_dev);
  if (st != TPC_OK) return st;
  RefitBufs b = refit_bufs(n_clusters, in, trk, dist_map_dev);
  set_material(b, mat);
  b.ckpt = const_cast<float*>(ckpt_dev);
  b.status = const_cast<int32_t*>(status_dev);
  b.grad_chi2 = grad_chi2_dev;
  b.grad_map = grad_map_dev;
  b.gx = grad_x_dev;
  b.gy = grad_y_dev;
  b.gz = grad_z_dev;
  const Consts k = make_consts(geom, params);
  hipError_t e = bwd::refit_backward_noalloc(k, b, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

tpc_status tpc_refit_backward(const tpc_geometry* geom, const tpc_params* params,
                              int64_t n_clusters, tpc_clusters in, tpc_refit_tracks trk,
                              const float* dist_map_dev, const tpc_material* mat,
                              const float* ckpt_dev,
                              const int32_t* status_dev, const float* grad_chi2_dev,
                              float* grad_map_dev, float* grad_x_dev, float* grad_y_dev,
                              float* grad_z_dev, void* ws_dev, size_t ws_bytes, void* stream)
{
  tpc_status st = refit_backward_check(geom, params, n_clusters, in, trk, dist_map_dev, mat,
                                       ckpt_dev,
                                       status_dev, grad_chi2_dev, grad_map_dev, grad_x_dev,
                                       grad_y_dev, grad_z_dev);
  if (st != TPC_OK) return st;
  if (!ws_dev) return TPC_ERR_INVALID;
  if (ws_bytes < tpc_refit_workspace_bytes()) return TPC_ERR_WORKSPACE;
  if (reinterpret_cast<uintptr_t>(ws_dev) % 8) return TPC_ERR_INVALID;
  RefitBufs b = refit_bufs(n_clusters, in, trk, dist_map_dev);
  set_material(b, mat);
  b.ckpt = const_cast<float*>(ckpt_dev);
  b.status = const_cast<int32_t*>(status_dev);
  b.grad_chi2 = grad_chi2_dev;
  b.grad_map = grad_map_dev;
  b.gx = grad_x_dev;
  b.gy = grad_y_dev;
  b.gz = grad_z_dev;
  b.acc = static_cast<long long*>(ws_dev);
  b.flags = reinterpret_cast<int*>(static_cast<char*>(ws_dev) + 8 * kRows * kPhi);
  const Consts k = make_consts(geom, params);
  hipError_t e = bwd::refit_backward(k, b, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

void tpc_default_merge_params(tpc_merge_params* m)
{
  if (!m) return;
  m->max_dz = 20.0f;
  m->max_dist = 40.0f;
  m->chi2_max = 30.0f;
  const double deg = 3.14159265358979323846 / 180.0;
  for (int k = 0; k < kPhi; k++) {
    const double a = (20.0 * (k + 0.5)) * deg;
    m->cos_a[k] = (float)cos(a);
    m->sin_a[k] = (float)sin(a);
  }
  m->cos_d = (float)cos(20.0 * deg);
  m->sin_d = (float)sin(20.0 * deg);
}

namespace {
struct MergeWs {
  int64_t n_seg, seg_inst, seg_pos, out_ok, out_p, out_c, out_x, seg_key, bkt_cur, bkt_off,
      bkt_order, bkt_pos, bkt_tq, hit_md, succ, pred_key, has_pred, chain_head, it_ns, it_nh, ch_part,
      total;
};

MergeWs merge_ws(int64_t cap, int64_t cap_hits)
{
  MergeWs w;
  Carve c;
  w.n_seg = c.take(8);
  w.seg_inst = c.take(4 * cap);
  w.seg_pos = c.take(24 * cap);
  w.out_ok = c.take(4 * cap);
  w.out_p = c.take(20 * cap);
  w.out_c = c.take(60 * cap);
  w.out_x = c.take(4 * cap);
  w.seg_key = c.take(4 * 2 * cap);
  w.bkt_cur = c.take(4 * 2 * kMergeBuckets);
  w.bkt_off = c.take(4 * 2 * (kMergeBuckets + 1));
  w.bkt_order = c.take(4 * 2 * cap);
  w.bkt_pos = c.take(16 * 2 * cap);
  w.bkt_tq = c.take(16 * 2 * cap);
  w.hit_md = c.take(16 * cap_hits);
  w.succ = c.take(4 * cap);
  w.pred_key = c.take(8 * cap);
  w.has_pred = c.take(4 * cap);
  w.chain_head = c.take(4 * cap);
  w.it_ns = c.take(4 * 2 * cap);
  w.it_nh = c.take(4 * 2 * cap);
  w.ch_part = c.take(8 * 3 * ((2 * cap + kBlock - 1) / kBlock + 1));
  w.total = c.off;
  return w;
}
}  // namespace

size_t tpc_merge_workspace_bytes(int64_t cap_segments, int64_t cap_hits)
{
  if (cap_segments < 0 || cap_hits < 0) return 0;
  return (size_t)merge_ws(cap_segments, cap_hits).total;
}

tpc_status tpc_merge_tracks(const tpc_geometry* geom, const tpc_params* params,
                            const tpc_merge_params* mp, int32_t n_inst,
                            const int64_t* inst_off_dev, tpc_clusters in,
                            const tpc_tracks* seg, const tpc_result* seg_result_dev,
                            const tpc_merged* out, void* ws_dev, size_t ws_bytes, void* stream)
{
  if (!geom || !params || !mp || !seg || !out || !inst_off_dev || !seg_result_dev || !ws_dev)
    return TPC_ERR_INVALID;
  if (geom->n_rows != kRows || n_inst != 2 * kPhi || (params->flags & ~kKnownFlags))
    return TPC_ERR_INVALID;
  if (!(geom->sigma_y2 > 0) || !(geom->sigma_z2 > 0)) return TPC_ERR_INVALID;
  const int64_t cap = seg->cap_tracks;
  if (cap < 0 || cap >= ((int64_t)1 << 31) || seg->cap_hits < 0 ||
      seg->cap_hits >= ((int64_t)1 << 31))
    return TPC_ERR_INVALID;
  if (cap > 0 && (!seg->param || !seg->cov || !seg->x_ref || !seg->hit_off || !seg->hit_clu ||
                  !in.y || !in.z || !in.row))
    return TPC_ERR_INVALID;
  if (out->cap_tracks < cap || out->cap_hits < seg->cap_hits) return TPC_ERR_INVALID;
  if (seg->hit_data && reinterpret_cast<uintptr_t>(seg->hit_data) % 16) return TPC_ERR_INVALID;
  if (cap > 0 && (!out->param || !out->cov || !out->chi2 || !out->ndf || !out->status ||
                  !out->sector || !out->x_ref || !out->hit_off || !out->hit_clu ||
                  !out->seg_off || !out->seg || !out->next || !out->counts))
    return TPC_ERR_INVALID;
  const MergeWs w = merge_ws(cap, seg->cap_hits);
  if ((int64_t)ws_bytes < w.total) return TPC_ERR_WORKSPACE;
  MergeBufs b;
  b.y = in.y;
  b.z = in.z;
  b.row = in.row;
  b.inst_off = inst_off_dev;
  b.seg = *seg;
  b.res = seg_result_dev;
  b.cap_seg = cap;
  b.mp = *mp;
  b.out = *out;
  b.n_seg = at<int64_t>(ws_dev, w.n_seg);
  b.seg_inst = at<int32_t>(ws_dev, w.seg_inst);
  b.seg_pos = at<float>(ws_dev, w.seg_pos);
  b.out_ok = at<int32_t>(ws_dev, w.out_ok);
  b.out_p = at<float>(ws_dev, w.out_p);
  b.out_c = at<float>(ws_dev, w.out_c);
  b.out_x = at<float>(ws_dev, w.out_x);
  b.seg_key = at<int32_t>(ws_dev, w.seg_key);
  b.bkt_cur = at<int32_t>(ws_dev, w.bkt_cur);
  b.bkt_off = at<int32_t>(ws_dev, w.bkt_off);
  b.bkt_order = at<int32_t>(ws_dev, w.bkt_order);
  b.bkt_pos = at<float4>(ws_dev, w.bkt_pos);
  b.bkt_tq = at<float4>(ws_dev, w.bkt_tq);
  b.hit_md = at<float4>(ws_dev, w.hit_md);
  b.succ = at<int32_t>(ws_dev, w.succ);
  b.pred_key = at<unsigned long long>(ws_dev, w.pred_key);
  b.has_pred = at<int32_t>(ws_dev, w.has_pred);
  b.chain_head = at<int32_t>(ws_dev, w.chain_head);
  b.it_ns = at<int32_t>(ws_dev, w.it_ns);
  b.it_nh = at<int32_t>(ws_dev, w.it_nh);
  b.ch_part = at<int64_t>(ws_dev, w.ch_part);
  const Consts k = make_consts(geom, params);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = (params->flags & TPC_FLAG_DETERMINISTIC) ? det::merge_tracks(k, b, s)
                                                           : prod::merge_tracks(k, b, s);
  return e == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

tpc_status tpc_cluster_transform(const tpc_transform_geometry* tg, uint32_t flags,
                                 int64_t n_clusters, tpc_raw_clusters in,
                                 const float* dist_map_dev, const float* corr_map_dev,
                                 float* x_dev, float* y_dev, float* z_dev, uint16_t* row_dev,
                                 void* stream)
{
  if (!tg || n_clusters < 0 || (flags & ~kKnownFlags)) return TPC_ERR_INVALID;
  if (corr_map_dev && (tg->nu < 2 || tg->nv < 2 || tg->nw < 2)) return TPC_ERR_INVALID;
  if (n_clusters > 0 && (!in.sector || !in.row || !in.pad || !in.time || !x_dev || !y_dev ||
                         !z_dev || !row_dev))
    return TPC_ERR_INVALID;
  if (corr_map_dev && reinterpret_cast<uintptr_t>(corr_map_dev) % 16) return TPC_ERR_INVALID;
  TransformConsts k;
  memcpy(k.row_x, tg->row_x, sizeof(k.row_x));
  memcpy(k.pad_w, tg->pad_w, sizeof(k.pad_w));
  memcpy(k.pad_c, tg->pad_c, sizeof(k.pad_c));
  k.tbin = tg->tbin_us;
  k.vdrift = tg->vdrift_cm_us;
  k.zlen = tg->zlen_cm;
  k.t0 = tg->t0_us;
  k.nu = tg->nu;
  k.nv = tg->nv;
  k.nw = tg->nw;
  k.u0 = tg->u0;
  k.iu = tg->iu;
  k.v0 = tg->v0;
  k.iv = tg->iv;
  k.w0 = tg->w0;
  k.iw = tg->iw;
  TransformBufs b;
  b.sector = in.sector;
  b.row = in.row;
  b.pad = in.pad;
  b.time = in.time;
  b.dmap = dist_map_dev;
  b.rmap = reinterpret_cast<const float4*>(corr_map_dev);
  b.x = x_dev;
  b.y = y_dev;
  b.z = z_dev;
  b.row_out = row_dev;
  b.n = n_clusters;
  auto al = [](const void* p, uintptr_t a) { return reinterpret_cast<uintptr_t>(p) % a == 0; };
  b.aligned = al(in.sector, 4) && al(in.row, 8) && al(in.pad, 16) && al(in.time, 16) &&
              al(x_dev, 16) && al(y_dev, 16) && al(z_dev, 16) && al(row_dev, 8);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = (flags & TPC_FLAG_DETERMINISTIC) ? det::cluster_transform(k, b, s)
                                                   : prod::cluster_transform(k, b, s);
  return e == hipSuccess ? TPC_OK : TPC_ERR_HIP;
}

}  // extern "C"
