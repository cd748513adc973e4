// Internal interface between the C-ABI host code (tpc_api.cpp) and the two
// builds of the kernels (tpc_kernels.hip compiled into namespaces det and
// prod with different floating-point flags).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tpcca.h"

namespace tpcca {

constexpr int kRows = TPC_N_ROWS;
constexpr int kBlock = 256;

// Constants every kernel may need, passed by value in the kernel arguments.
struct Consts {
  float row_x[kRows];
  float tan_half;
  float kB;            // curvature per unit q/pT: (float)(-0.299792458e-2 * B)
  float bz;            // field [T] (the binary64 reverse pass derives its own kB)
  float vy, vz;        // cluster variances
  float ivy, ivz;      // (float)(1 / (1.5 * variance)) of the neighbour score
  float nf_win_y, nf_win_z, nf_chi2_max;
  float tc_chi2_pick, snp_max;
  float grid_occupancy, edge_margin, search_margin, y_valid_margin;
  int32_t min_chain, tc_max_miss, min_tracklet_hits, min_track_hits;
  int32_t tl_chunk;    // tracklets per workgroup of the tracklet kernel (64, 128, 256)
};

// Device buffers of one call.
struct GridBufs {
  const float *x, *y, *z;
  const uint16_t* row;
  const int64_t* inst_off;
  int32_t n_inst;
  int64_t n;
  // outputs
  int32_t* sseg;
  int32_t* row_off;
  tpc_row_meta* meta;
  int32_t* bin_off;
  int32_t* perm;
  float2* yz;
  int64_t bin_cap;
  tpc_result* res;
  // workspace
  int32_t* cseg;       // [n] segment of each input cluster, -1 invalid
  int32_t* seg_cnt;    // [n_seg]
  uint32_t* seg_mm;    // [4][n_seg] ordered-float min y, max y, min z, max z
  int32_t* inst_bad;   // [n_inst]
  int32_t* nb1;        // [n_seg] bins + 1 per segment, then their exclusive scan
  int32_t* fill;       // [bin_cap] bin counters of segments with too many bins for LDS
  int32_t* seg_pos;    // [n_seg] segment lengths, then the segments' first positions
  int32_t* seg_cursor; // [n_seg] partition cursors
  int32_t* tmp_perm;   // [n] clusters partitioned by segment: input index
  float2* tmp_yz;      // [n] and (y, z)
  int64_t* scan_tmp;   // scan partials
  int64_t scan_tmp_len;
};

struct TrackBufs {
  const int64_t* inst_off;
  int32_t n_inst;
  int64_t n;
  // grid (inputs)
  const int32_t* sseg;
  const int32_t* row_off;
  const tpc_row_meta* meta;
  const int32_t* bin_off;
  const int32_t* perm;
  const float2* yz;
  // workspace
  int32_t *up, *dn, *up2, *dn2;
  int32_t* start;
  unsigned long long* start_flag;  // [scan tiles * kBlock] start flags, one byte each
  int64_t cap;         // tracklet capacity
  float* tl_par;       // [5][cap]
  float* tl_cov;       // [15][cap]
  float* tl_chi2;
  int32_t *tl_nhit, *tl_rmin, *tl_rmax, *tl_status;
  int32_t* tl_hit;     // [152][cap]: hit slot of row r of tracklet t at r * cap + t
  int32_t* tl_ncand;   // [cap] candidates evaluated by the extension searches
  unsigned long long* owner;  // [n]
  unsigned long long* tl_key;  // [cap] selection key, 0 for rejected tracklets
  uint8_t* tl_owned;   // [152][cap] 1 where the tracklet owns its hit on the row
  int32_t* own_t;      // [n] tracklet owning each position, -1 if none
  int4* tl_rec;        // [cap][2] track record: (track, first hit, owned-row mask
                       // words 0-1), (mask words 2-4, unused); track -1 if none
  int32_t* tl_own;     // [cap] owned hits of accepted tracklets, 0 otherwise
  int64_t* tsv;        // [cap] packed (track flag << 32 | owned hits), then its scan
  int64_t* scan_tmp;
  int64_t scan_tmp_len;
  int64_t* tl_first;   // [n_inst + 1] first tracklet of each instance
  int64_t* chunk_off;  // [n_inst + 1] first tracklet chunk of each instance
  int64_t* counters;   // [8] device counters
  bool count_candidates;  // instrumented tracklet kernel (tl_ncand)
  // outputs
  tpc_tracks out;
  tpc_result* res;
};

// Buffers of the refit (a8) and its reverse pass (a9).
struct RefitBufs {
  const float *x, *y, *z;
  const uint16_t* row;
  const uint8_t* sector;
  const int32_t *hit_off, *hit_clu;
  const float* seed;      // [n_tracks][5]
  const float* dmap;      // [152][18]
  int64_t n_tracks, n_clusters;
  float* chi2;            // [n_tracks]
  int32_t* status;        // [n_tracks]
  float* ckpt;            // [n_hits][20]
  const float* grad_chi2; // [n_tracks]
  float* grad_map;        // [152*18]
  float *gx, *gy, *gz;    // [n_clusters]
  long long* acc;         // [152*18] fixed-point map-gradient accumulators
  int* flags;             // [1] accumulator overflow flag
  // field map and material (any may be null: the uniform field of Consts,
  // no scattering, no energy loss)
  const float* bz;        // [152][nzb] field [T] per row and z bin
  int32_t nzb;            // z bins over [-250, 250] cm
  const float* ix0;       // [152] inverse radiation length [1/cm]
  const float* eloss;     // [152] mean energy loss at minimum ionisation [GeV/cm]
};

constexpr int kPhi = 18;

// Constants of the cluster transformation (f3), by value in the kernel
// arguments.
struct TransformConsts {
  float row_x[kRows], pad_w[kRows], pad_c[kRows];
  float tbin, vdrift, zlen, t0;
  int32_t nu, nv, nw;
  float u0, iu, v0, iv, w0, iw;
};

struct TransformBufs {
  const uint8_t* sector;
  const uint16_t* row;
  const float *pad, *time;
  const float* dmap;    // [152][18] or null
  const float4* rmap;   // [36][nu][nv][nw] nodes (dx, dy, dz, unused) or null
  float *x, *y, *z;
  uint16_t* row_out;
  int64_t n;
  bool aligned;         // every array allows the four-cluster vector accesses
};

// Buffers of sector-track merging and the global refit (f1).
// Pair-search buckets of the merging step: 36 instances x 1024 z bins of
// 16 cm from -8192 cm (clusters of collisions later in a time frame sit up
// to the frame's drift length away from the detector's +-250 cm; beyond
// +-8192 cm the end bins take them).
constexpr int kMergeZBins = 1024;
constexpr float kMergeZ0 = -8192.0f, kMergeZInv = 1.0f / 16.0f;
constexpr int kMergeBuckets = 36 * kMergeZBins;

struct MergeBufs {
  const float *y, *z;
  const uint16_t* row;
  const int64_t* inst_off;   // [37]
  tpc_tracks seg;            // the tracker's tracks (param, cov, x_ref, hit lists)
  const tpc_result* res;     // their counts
  int64_t cap_seg;
  tpc_merge_params mp;
  tpc_merged out;
  // workspace
  int64_t* n_seg;            // [1] segments of this call
  int32_t* seg_inst;         // [cap] instance of each segment
  float* seg_pos;            // [cap][6] global x, y, z of the first and the last hit
  int32_t* out_ok;           // [cap] outer state valid
  float *out_p, *out_c, *out_x;  // [cap][5], [cap][15], [cap] (x: also where a failed pass stopped)
  // pair-search buckets: two keys per segment, (instance, z bin) of its
  // first hit (key 0) and of its last hit (key 1)
  int32_t* seg_key;          // [2][cap] bucket of each segment
  int32_t* bkt_cur;          // [2][kMergeBuckets] counts, then scatter cursors
  int32_t* bkt_off;          // [2][kMergeBuckets + 1] first position of each bucket
  int32_t* bkt_order;        // [2][cap] segments in bucket order
  float4* bkt_pos;           // [2][cap] their end of key w: x, y, z, outer state valid (1/0)
  float4* bkt_tq;            // [2][cap] tgl, q/pt and their variances: key 0 of the inner
                             // (tracker's) state, key 1 of the outer state
  float4* hit_md;            // [seg.cap_hits] the tracker's hit data in merged order
  int32_t* succ;             // [cap] best successor
  unsigned long long* pred_key;  // [cap] best predecessor: min of (chi2 bits << 32 | segment)
  int32_t* has_pred;         // [cap] a kept link ends here
  int32_t* chain_head;       // [cap] first segment of each chain
  int32_t *it_ns, *it_nh;    // [2 cap] chain-start items: segment and hit counts
  int64_t* ch_part;          // [3][ceil(2 cap / kBlock)] workgroup sums, then offsets
};

// Kernel timing hooks (tpc_profile_*): no-ops unless profiling is enabled.
int prof_begin(hipStream_t s, const char* name);
void prof_end(hipStream_t s, int slot);

// Scan partials needed for an array of n items.
int64_t scan_partials(int64_t n);

#define TPCCA_DECLARE_LAUNCHERS(NS)                                                  \
  namespace NS {                                                                     \
  hipError_t grid_build(const Consts& k, const GridBufs& b, hipStream_t s);         \
  hipError_t sector_track(const Consts& k, const TrackBufs& b, bool standard,       \
                          hipStream_t s);                                            \
  hipError_t refit_forward(const Consts& k, const RefitBufs& b, hipStream_t s);     \
  hipError_t cluster_transform(const TransformConsts& k, const TransformBufs& b,    \
                               hipStream_t s);                                       \
  hipError_t merge_tracks(const Consts& k, const MergeBufs& b, hipStream_t s);      \
  }

namespace bwd {
hipError_t refit_backward(const Consts& k, const RefitBufs& b, hipStream_t s);
// the same on the library's static per-device scratch (b.acc, b.flags unused)
hipError_t refit_backward_noalloc(const Consts& k, RefitBufs b, hipStream_t s);
size_t refit_scratch_bytes();
}

TPCCA_DECLARE_LAUNCHERS(det)
TPCCA_DECLARE_LAUNCHERS(prod)

}  // namespace tpcca
