// Host-only stand-ins for the kernel launchers of libtpcca, for running the
// C ABI's host code (tpc_api.cpp: validation, workspace carving, constant
// derivation) under AddressSanitizer and UndefinedBehaviorSanitizer without
// a GPU.  Each stand-in checks that every workspace array the host code
// carved lies inside the workspace the caller passed, touches the first and
// last byte of each (so an out-of-range carve is an ASan error), and
// returns success.  Test infrastructure only.
#include <stdio.h>
#include <stdlib.h>

#include "tpc_internal.h"

namespace stub {
const char* g_ws = nullptr;
size_t g_ws_bytes = 0;
int g_calls = 0;

void in_ws(const void* p, int64_t bytes, const char* what)
{
  if (bytes <= 0) return;
  const char* c = static_cast<const char*>(p);
  if (!g_ws || c < g_ws || c + bytes > g_ws + g_ws_bytes) {
    fprintf(stderr, "workspace array %s [%p, +%lld) outside [%p, +%zu)\n", what, p,
            (long long)bytes, (const void*)g_ws, g_ws_bytes);
    abort();
  }
  volatile char a = c[0];
  volatile char b = c[bytes - 1];
  (void)a;
  (void)b;
}
}  // namespace stub

namespace tpcca {

static hipError_t grid_stub(const Consts& k, const GridBufs& b)
{
  using stub::in_ws;
  const int64_t n = b.n, seg = (int64_t)b.n_inst * kRows;
  if (!(k.grid_occupancy > 0) || k.tl_chunk < 64) abort();
  in_ws(b.cseg, 4 * n, "cseg");
  in_ws(b.seg_cnt, 4 * seg, "seg_cnt");
  in_ws(b.seg_mm, 16 * seg, "seg_mm");
  in_ws(b.inst_bad, 4 * b.n_inst, "inst_bad");
  in_ws(b.nb1, 4 * seg, "nb1");
  in_ws(b.fill, 4 * b.bin_cap, "fill");
  in_ws(b.seg_pos, 4 * seg, "seg_pos");
  in_ws(b.seg_cursor, 4 * seg, "seg_cursor");
  in_ws(b.tmp_perm, 4 * n, "tmp_perm");
  in_ws(b.tmp_yz, 8 * n, "tmp_yz");
  in_ws(b.scan_tmp, 8 * b.scan_tmp_len, "scan_tmp");
  stub::g_calls++;
  return hipSuccess;
}

static hipError_t track_stub(const TrackBufs& b)
{
  using stub::in_ws;
  const int64_t n = b.n, cap = b.cap;
  in_ws(b.up, 4 * n, "up");
  in_ws(b.dn, 4 * n, "dn");
  in_ws(b.up2, 4 * n, "up2");
  in_ws(b.dn2, 4 * n, "dn2");
  in_ws(b.start, 4 * cap, "start");
  in_ws(b.tl_par, 20 * cap, "tl_par");
  in_ws(b.tl_cov, 60 * cap, "tl_cov");
  in_ws(b.tl_chi2, 4 * cap, "tl_chi2");
  in_ws(b.tl_hit, 4 * (int64_t)kRows * cap, "tl_hit");
  in_ws(b.tl_ncand, 4 * cap, "tl_ncand");
  in_ws(b.owner, 8 * n, "owner");
  in_ws(b.tl_own, 4 * cap, "tl_own");
  in_ws(b.tsv, 8 * cap, "tsv");
  in_ws(b.tl_first, 8 * (b.n_inst + 1), "tl_first");
  in_ws(b.chunk_off, 8 * (b.n_inst + 1), "chunk_off");
  in_ws(b.tl_key, 8 * cap, "tl_key");
  in_ws(b.tl_owned, (int64_t)kRows * cap, "tl_owned");
  in_ws(b.own_t, 4 * n, "own_t");
  in_ws(b.tl_rec, 32 * cap, "tl_rec");
  in_ws(b.start_flag, n, "start_flag");
  in_ws(b.counters, 64, "counters");
  in_ws(b.scan_tmp, 8 * b.scan_tmp_len, "scan_tmp");
  stub::g_calls++;
  return hipSuccess;
}

static hipError_t refit_stub(const RefitBufs& b)
{
  if (b.n_tracks < 0 || b.n_clusters < 0 || (b.bz && b.nzb < 1)) abort();
  stub::g_calls++;
  return hipSuccess;
}

#define STUB_NS(NS)                                                                  \
  namespace NS {                                                                     \
  hipError_t grid_build(const Consts& k, const GridBufs& b, hipStream_t)            \
  {                                                                                  \
    return grid_stub(k, b);                                                          \
  }                                                                                  \
  hipError_t sector_track(const Consts&, const TrackBufs& b, bool, hipStream_t)     \
  {                                                                                  \
    return track_stub(b);                                                            \
  }                                                                                  \
  hipError_t refit_forward(const Consts&, const RefitBufs& b, hipStream_t)          \
  {                                                                                  \
    return refit_stub(b);                                                            \
  }                                                                                  \
  hipError_t merge_tracks(const Consts&, const MergeBufs& b, hipStream_t)           \
  {                                                                                  \
    using stub::in_ws;                                                               \
    const int64_t c = b.cap_seg;                                                     \
    in_ws(b.n_seg, 8, "n_seg");                                                      \
    in_ws(b.seg_pos, 24 * c, "seg_pos");                                             \
    in_ws(b.out_c, 60 * c, "out_c");                                                 \
    in_ws(b.bkt_off, 4 * 2 * (kMergeBuckets + 1), "bkt_off");                       \
    in_ws(b.bkt_order, 4 * 2 * c, "bkt_order");                                      \
    in_ws(b.bkt_pos, 16 * 2 * c, "bkt_pos");                                         \
    in_ws(b.bkt_tq, 16 * 2 * c, "bkt_tq");                                           \
    in_ws(b.hit_md, 16 * b.seg.cap_hits, "hit_md");                                 \
    in_ws(b.chain_head, 4 * c, "chain_head");                                        \
    in_ws(b.ch_part, 8 * 3 * ((2 * c + 255) / 256), "ch_part");                      \
    stub::g_calls++;                                                                 \
    return hipSuccess;                                                               \
  }                                                                                  \
  hipError_t cluster_transform(const TransformConsts& k, const TransformBufs& b,    \
                               hipStream_t)                                          \
  {                                                                                  \
    if (b.n < 0 || (b.rmap && (k.nu < 2 || k.nv < 2 || k.nw < 2))) abort();          \
    stub::g_calls++;                                                                 \
    return hipSuccess;                                                               \
  }                                                                                  \
  }
STUB_NS(det)
STUB_NS(prod)

namespace bwd {
hipError_t refit_backward(const Consts&, const RefitBufs& b, hipStream_t)
{
  stub::in_ws(b.acc, 8 * kRows * kPhi + 4, "acc");
  return refit_stub(b);
}
hipError_t refit_backward_noalloc(const Consts&, RefitBufs b, hipStream_t) { return refit_stub(b); }
size_t refit_scratch_bytes() { return 8 * kRows * kPhi + 256; }
}  // namespace bwd

}  // namespace tpcca
