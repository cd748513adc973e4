/*
 * tpcca.h -- C ABI of the MI355X TPC sector tracker (libtpcca.so).
 *
 * Problem (Rohr, "Improvements of the GPU Processing Framework for ALICE"):
 * online TPC processing finds tracks in the clusters of each TPC sector and
 * assigns clusters to tracks (Sec. 1; the cluster-to-track association is the
 * quantity compared in Sec. 2).  The library runs the hot path of that step on
 * one gfx950 GPU: cluster grid (a1), neighbour finding (a2) and cleaning (a3),
 * start hits (a4), tracklet construction with a Kalman helix fit in the
 * solenoid field (a5) and tracklet selection (a6), in a deterministic mode
 * whose output is bit-identical to the CPU reference and a production mode
 * (Sec. 2: deterministic processing mode).
 *
 * Conventions for every entry point:
 *   - Pointers named *_dev and every array inside the tpc_clusters, tpc_grid,
 *     tpc_tracks and tpc_result structs are DEVICE pointers owned by the
 *     caller; pointers named *_host and the tpc_geometry / tpc_params structs
 *     are host memory, read during the call only.
 *   - Calls enqueue work on `stream` (a hipStream_t, NULL = default stream)
 *     and return before it completes; nothing is allocated or freed.
 *   - Argument errors are returned synchronously (nothing is enqueued then);
 *     data-dependent conditions (invalid clusters, output capacity) are
 *     reported in the device-resident tpc_result, readable after the stream
 *     has completed.
 *   - One workspace may serve one call at a time; calls with distinct
 *     workspaces and outputs may run concurrently.  No C++ exception crosses
 *     the ABI.
 *
 * Data layout:
 *   clusters   SoA over all instances; instance i owns input indices
 *              [inst_off[i], inst_off[i+1]); inst_off[0] = 0 and each
 *              instance holds fewer than 2^24 clusters.
 *   positions  the grid orders the valid clusters of instance i by
 *              (row, bin, input index) into positions
 *              [inst_off[i], inst_off[i] + n_valid_i); the remaining positions
 *              of the instance are padding (sseg = perm = -1, y = z = 0).
 *              Links and tracklet hits are positions; track hit lists and
 *              clu2trk use input indices.
 */
#ifndef TPCCA_H
#define TPCCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TPC_N_ROWS 152

typedef enum {
  TPC_OK = 0,
  TPC_ERR_INVALID = -1,     /* bad argument (null pointer, size, layout)  */
  TPC_ERR_UNSUPPORTED = -2, /* mode not built into this library           */
  TPC_ERR_HIP = -3,         /* a HIP runtime call failed                  */
  TPC_ERR_WORKSPACE = -4    /* workspace smaller than the size query said */
} tpc_status;

/* params->flags: any other bit set is rejected with TPC_ERR_INVALID.  (Every
 * call only enqueues work on its stream, so any call can be captured into a
 * HIP graph as it is; no flag asks for that.) */
enum {
  TPC_FLAG_DETERMINISTIC = 1u, /* contraction-free code object + ordering kernels (Sec. 2) */
  TPC_FLAG_GENERIC = 8u,       /* never use the kernels compiled for the standard
                                  configuration (results are the same; for measuring) */
  TPC_FLAG_COUNT_CANDIDATES = 16u /* tpc_sector_track: an instrumented tracklet kernel
                                  counts, per tracklet, the clusters inside its search
                                  windows into the workspace's tl_ncand (results are the
                                  same; slower; for byte counts) */
};

/* Detector description (host, by pointer).  n_rows must be 152; row_x are
 * the pad-row plane positions [cm] along the sector axis, ascending;
 * bz_tesla the solenoid field; tan_half_sector = tan(10 deg); sigma_y2,
 * sigma_z2 the cluster position variances [cm^2]. */
typedef struct {
  int32_t n_rows;
  float row_x[TPC_N_ROWS];
  float bz_tesla;
  float tan_half_sector;
  float sigma_y2, sigma_z2;
} tpc_geometry;

/* Algorithm parameters (host); tpc_default_params() fills the defaults:
 * neighbour windows 3.0 / 3.5 cm and score cut 13.8, tracklet chi2 cut 13.8,
 * |snp| < 0.99, grid occupancy 2, sector-edge margin 1 cm, window margin
 * 0.01 cm, cluster validity margin 2 cm, chains >= 3 hits, 10 consecutive
 * misses, >= 10 hits per tracklet and per track, flags 0, and the
 * performance-only tl_chunk = 0 (tracklets per workgroup of the tracklet
 * kernel: 64, 128 or 256; 0 selects 256).  Results do not depend on
 * grid_occupancy (the bin size) or tl_chunk. */
typedef struct {
  float nf_win_y, nf_win_z, nf_chi2_max;
  float tc_chi2_pick, snp_max;
  float grid_occupancy;
  float edge_margin, search_margin;
  float y_valid_margin;
  int32_t min_chain, tc_max_miss, min_tracklet_hits, min_track_hits;
  uint32_t flags;
  int32_t tl_chunk;
} tpc_params;

/* Clusters: device SoA, n_clusters entries each (charge is carried, unused). */
typedef struct {
  const float *x, *y, *z;
  const uint16_t *row, *charge;
} tpc_clusters;

/* Geometry of one (instance,row) grid: ny x nz bins, bin = iz*ny + iy,
 * bin_off entries [bin_base, bin_base + ny*nz] (last = row end);
 * count = valid clusters; iy = trunc((y - y0) * iwy) clamped to [0, ny-1]. */
typedef struct {
  int32_t ny, nz, bin_base, count;
  float y0, z0, iwy, iwz;
} tpc_row_meta;

/* Grid output of tpc_grid_build (device arrays, caller-allocated):
 *   sseg    [n_clusters]            instance*152 + row of each position, -1 = padding
 *   row_off [n_inst*153]            first position of each (instance,row); entry 152 = end
 *   meta    [n_inst*152]
 *   bin_off [bin_cap]               bin_cap >= tpc_grid_bin_capacity(params, ...)
 *   perm    [n_clusters]            input index of each position, -1 = padding
 *   yz      [2*n_clusters]          cluster (y, z) pairs in position order, 8-byte
 *                                   aligned                                          */
typedef struct {
  int32_t* sseg;
  int32_t* row_off;
  tpc_row_meta* meta;
  int32_t* bin_off;
  int32_t* perm;
  float* yz;
  int64_t bin_cap;
} tpc_grid;

/* Tracks (device arrays, caller-allocated): parameters (y, z, snp, tgl, qpt)
 * and lower-triangular covariance at plane x_ref (innermost hit of the fit);
 * chi2 and ndf of the fit; hit lists in CSR form (hit_off[cap_tracks+1],
 * hit_clu[cap_hits], input indices, ascending row); clu2trk[n_clusters]
 * = track index or -1.  Deterministic mode emits tracks in tracklet order;
 * production mode in any order.  If capacity is short the longest prefix
 * that fits is written and tpc_result says what was needed.
 * hit_data (optional, NULL to skip): per hit slot of hit_clu, four floats
 * -- the x of the hit's row plane, its y and z, and the phi sector k of its
 * instance (i mod 18, as a float) -- written by tpc_sector_track beside the
 * hit list, 16-byte aligned.  tpc_merge_tracks reads its segments' hits
 * from there when it is not NULL (contiguously instead of through the
 * cluster arrays); the values are the same, so is the result. */
typedef struct {
  float* param;    /* [cap_tracks][5]  */
  float* cov;      /* [cap_tracks][15] */
  float* chi2;     /* [cap_tracks]     */
  int32_t* ndf;    /* [cap_tracks]     */
  float* x_ref;    /* [cap_tracks]     */
  int32_t* hit_off;
  int32_t* hit_clu;
  int32_t* clu2trk;
  int64_t cap_tracks, cap_hits;
  float* hit_data; /* [cap_hits][4] or NULL */
} tpc_tracks;

/* Device-resident status word, written by the calls.  overflow bits:
 * 1 bin table, 2 tracklets, 4 tracks, 8 track hits. */
typedef struct {
  int64_t n_valid, n_bad, n_bins;
  int64_t n_start, n_tracklets_kept;
  int64_t n_tracks, n_hits;
  int64_t need_tracklets, need_tracks, need_hits;
  int32_t overflow, reserved;
} tpc_result;

/* Byte offsets of the intermediate arrays inside the tracking workspace
 * (for inspection and testing; the tracker owns them during a call):
 *   up, dn, up2, dn2   i32[n_clusters]  raw and cleaned links (positions, -1 none)
 *   start              i32[cap_tracklets] start hits in list order
 *   tl_par             f32[5][cap_tracklets]   tl_cov f32[15][cap_tracklets]
 *   tl_chi2            f32[cap_tracklets]      tl_nhit, tl_rmin, tl_rmax, tl_status i32
 *   tl_hit             i32[152][cap_tracklets] (row-major by row: slot of row r of
 *                      tracklet t at r * cap_tracklets + t; -1 outside rmin..rmax)
 *   tl_ncand           i32[cap_tracklets] with TPC_FLAG_COUNT_CANDIDATES: clusters
 *                      inside the extension searches' window boxes (the candidates
 *                      any search must examine, whatever the bin size); otherwise
 *                      not written
 *   owner              u64[n_clusters]  selection keys per position          */
typedef struct {
  int64_t up, dn, up2, dn2, start;
  int64_t tl_par, tl_cov, tl_chi2, tl_nhit, tl_rmin, tl_rmax, tl_status, tl_hit, tl_ncand;
  int64_t owner;
  int64_t scratch;
  int64_t total;
  int64_t cap_tracklets;
} tpc_track_ws_layout;

void tpc_default_params(tpc_params* p);
const char* tpc_status_string(tpc_status s);

/* 1 if tpc_sector_track would run the kernels compiled for the standard
 * configuration (the synthetic detector description -- 152 planes at
 * 85 + r*162/151 cm, B = 0.5 T, tan(10 deg), sigma^2 = 0.01 / 0.0225 cm^2 --
 * with the default parameters, grid_occupancy and tl_chunk aside, and
 * TPC_FLAG_GENERIC clear), 0 if it would run the generic ones, TPC_ERR_INVALID
 * for a null argument.  Both give the same results; the compile-time
 * constants are the analogue of the paper's run-time compilation (Sec. 5). */
int32_t tpc_standard_configuration(const tpc_geometry* geom, const tpc_params* params);

/* Size queries (no device work).  cap_tracklets <= 0 selects the proven
 * bound n_clusters/3 + n_inst (every start hit heads a disjoint chain of at
 * least three clusters). */
int64_t tpc_grid_bin_capacity(const tpc_params* params, int32_t n_inst, int64_t n_clusters);
size_t tpc_grid_workspace_bytes(const tpc_params* params, int32_t n_inst, int64_t n_clusters);
size_t tpc_track_workspace_bytes(int32_t n_inst, int64_t n_clusters, int64_t cap_tracklets);
tpc_status tpc_track_workspace_layout(int32_t n_inst, int64_t n_clusters, int64_t cap_tracklets,
                                      tpc_track_ws_layout* out);

/* a1: build the per (instance,row) grid of the valid clusters, ordered by
 * (row, bin, input index): the total-order sort that Sec. 2 requires of the
 * deterministic mode.  The grid is a search structure of the tracker only
 * (the paper does not describe the tracker's data structures): results of
 * tpc_sector_track do not depend on its bin size.  Invalid clusters (row >= 152,
 * |y| beyond the sector plus margin, |z| > 1e5, NaN) are counted in
 * result->n_bad and left out.  Writes result fields n_valid, n_bad, n_bins
 * (overflow bit 1 if bin_cap is too small; the grid is then unusable).
 * inst_off_host and inst_off_dev hold the same n_inst+1 offsets.
 * Errors: TPC_ERR_INVALID (null pointer, n_rows != 152, bad offsets,
 * instance >= 2^24 clusters, a bin table that tpc_grid_bin_capacity sizes
 * above 2^31 - 1 entries -- bin offsets are 32-bit --, unknown flags),
 * TPC_ERR_WORKSPACE, TPC_ERR_HIP. */
tpc_status tpc_grid_build(const tpc_geometry* geom, const tpc_params* params, int32_t n_inst,
                          const int64_t* inst_off_host, const int64_t* inst_off_dev,
                          tpc_clusters in, const tpc_grid* grid, tpc_result* result_dev,
                          void* ws_dev, size_t ws_bytes, void* stream);

/* a2..a6: TPC sector tracking -- finding the tracks in the clusters of
 * each instance (one TPC sector of one collision or time frame) and
 * assigning clusters to tracks, the online step whose cluster-to-track
 * association Sec. 2 compares between CPU and GPU -- on a grid built by
 * tpc_grid_build with the same arguments: neighbour finding and cleaning,
 * start hits, tracklet construction with a Kalman helix fit in the solenoid
 * field (the track propagation of Sec. 4), tracklet selection.  Writes the
 * tracks (tpc_tracks) and the remaining result fields.
 * TPC_FLAG_DETERMINISTIC in params->flags selects the deterministic code
 * object and ordering kernels, whose output equals the binary32 CPU
 * reference bit for bit (Sec. 2: deterministic processing mode); without it
 * clusters may be assigned differently in rare ties of rounding (Sec. 2
 * quotes far below 0.001 % of clusters).  cap_tracklets <= 0 selects the
 * default capacity (tpc_track_workspace_bytes); more start hits than the
 * capacity set overflow bit 2 and the tracklets beyond it are dropped.
 * Errors: TPC_ERR_INVALID (as tpc_grid_build; also null output arrays,
 * capacities >= 2^31, hit_data not 16-byte aligned), TPC_ERR_WORKSPACE,
 * TPC_ERR_HIP. */
tpc_status tpc_sector_track(const tpc_geometry* geom, const tpc_params* params, int32_t n_inst,
                            const int64_t* inst_off_host, const int64_t* inst_off_dev,
                            tpc_clusters in, const tpc_grid* grid, const tpc_tracks* out,
                            tpc_result* result_dev, void* ws_dev, size_t ws_bytes,
                            int64_t cap_tracklets, void* stream);

/* Found tracks for the refit (device arrays, caller-owned):
 *   hit_off [n_tracks+1]   CSR offsets into hit_clu (hit_off[0] = 0)
 *   hit_clu [n_hits]       cluster index of each hit, ascending row within a track
 *   sector  [n_clusters]   phi-sector 0..17 of each cluster (selects the map column)
 *   seed    [n_tracks][5]  (y, z, snp, tgl, qpt); the filter starts from the first
 *                          hit's (y, z) and the seed's (snp, tgl, qpt), which are
 *                          constants of the fit (not differentiated)            */
typedef struct {
  const int32_t* hit_off;
  const int32_t* hit_clu;
  const uint8_t* sector;
  const float* seed;
  int64_t n_tracks, n_hits;
} tpc_refit_tracks;

#define TPC_N_PHI 18

/* f2: solenoid field map and material budget of the refit (Sec. 4 lists the
 * field map and the material budget map among the components of the track
 * propagation that TPC tracking shares; the formulas are this library's).
 * A host struct of caller-owned device arrays; the struct pointer, and each
 * array pointer in it, may be NULL:
 *   bz     [152][nzb]  field [T] of a step, taken at the destination hit: its
 *                      row and the z bin of its measured z (bins of 500/nzb cm
 *                      from z = -250 cm, clamped to the first and last bin);
 *                      NULL: the geometry's uniform bz_tesla
 *   nzb                z bins, 1..65536 when bz is given
 *   ix0    [152]       inverse radiation length [1/cm] of the gas at each row:
 *                      after each step's propagation, multiple-scattering noise
 *                      on (snp, tgl, q/pt) from the Highland width without its
 *                      logarithm, theta^2 = 0.0136^2 * t / (beta p)^2 with t the
 *                      traversed thickness in radiation lengths (pion mass);
 *                      NULL or entries <= 0: no scattering
 *   eloss  [152]       mean energy loss at minimum ionisation [GeV/cm]: dE/dx =
 *                      eloss / beta^2 changes q/pt by the factor
 *                      1 + E dE / p^2 along the step (outward steps lose
 *                      energy), and the covariance row of q/pt by the same
 *                      factor; NULL or entries <= 0: no energy loss
 * The field cell is piecewise constant and carries no gradient; the material
 * terms are differentiated like the rest of the filter. */
typedef struct {
  const float* bz;
  int32_t nzb;
  const float* ix0;
  const float* eloss;
} tpc_material;

/* a8: Kalman refit of found tracks under a per-row radial distortion map.
 * Each hit is measured on the plane X = x + dist_map[row][sector % 18]; the
 * filter of the tracker (propagation, Jacobian, update) runs from the first
 * hit outwards; chi2[t] is the sum of the update chi2 values, status[t] = 1
 * (and chi2 = 0) if the propagation failed (|snp| reaching snp_max).  The
 * state after every update (and the start state at the first hit) is
 * checkpointed, 20 floats per hit: (y, z, snp, tgl, qpt, lower-triangular
 * covariance), in five 16-byte parts of four floats.  ckpt holds n_hits * 20
 * floats (16-byte aligned), grouped by 64 consecutive tracks: the group of
 * tracks 64g .. 64g+63 fills floats [20 hit_off[64g], 20 hit_off[64g+64])
 * (the last group ends at n_hits), by hit number j (0 = a track's first
 * hit).  With L_k the group's track lengths, the a_j = #{k : L_k > j}
 * tracks that have a hit j store it from float4 5 E_j on, E_j =
 * hit_off[64g] + sum_k min(L_k, j): part q of track t at float4
 *   5 E_j + q a_j + #{k < t : L_k > j}
 * (so that the 64 lanes running a group store and load one contiguous run
 * per part and step).
 * With TPC_FLAG_DETERMINISTIC chi2 and every checkpoint equal the binary32
 * CPU reference bit for bit.  This refit is the
 * differentiable extension of the tracking step; the paper's shared track
 * propagation with field and material maps (Sec. 4) is its context.  With
 * mat (NULL: uniform field, no material), each step uses the field of its
 * destination hit's cell and is followed by the material's scattering noise
 * and energy loss, before that hit's update (see tpc_material).
 * A hit must name a cluster in [0, n_clusters) whose row is below 152 (the
 * map has no plane for other rows): a track with any other hit is not
 * refitted (status 2, chi2 0; 2 takes precedence over 1).  Checkpoints of
 * tracks with status != 0 are unspecified.
 * Errors: TPC_ERR_INVALID (null pointers, n_tracks < 0, n_clusters >= 2^31,
 * n_rows != 152, unknown flags, mat->bz given with nzb outside 1..65536). */
tpc_status tpc_refit(const tpc_geometry* geom, const tpc_params* params, int64_t n_clusters,
                     tpc_clusters in, tpc_refit_tracks trk, const float* dist_map_dev,
                     const tpc_material* mat, float* chi2_dev, int32_t* status_dev,
                     float* ckpt_dev, void* stream);

/* a9: gradient of L = sum_t grad_chi2[t] * chi2[t] with respect to the map
 * (grad_map[152][18]) and the cluster coordinates (grad_x, grad_y, grad_z,
 * [n_clusters]; clusters on no refitted track get 0).  The paper names the
 * offline-only TPC distortion corrections (Sec. 6) and the shared track
 * propagation (Sec. 4) but no gradient: this reverse-mode derivative of the
 * refit's chi2 is the differentiable extension, for fitting such a
 * correction map.  All outputs are overwritten.  Uses the forward call's
 * ckpt and status (same inputs, mat included); tracks with status != 0
 * contribute nothing.
 * Precondition: each cluster is a hit of at most one refitted track (as in
 * the tracker's output, where clu2trk names one track per cluster).  The
 * cluster gradients are stored, not added, so a cluster on several tracks
 * gets the gradient of one of its hits, which one is unspecified; the map
 * gradient stays the full sum over all hits.
 * Every step is rebuilt from the previous checkpoint and differentiated in
 * reverse.  The map sums are exact 64-bit fixed-point sums (scale 2^24), so
 * the gradient is identical from run to run.  ws_dev must hold
 * tpc_refit_workspace_bytes() bytes (accumulators and an overflow flag that
 * is set, and the sum clamped, if a hit's |dL/dX| exceeds 2^37). */
size_t tpc_refit_workspace_bytes(void);
tpc_status tpc_refit_backward(const tpc_geometry* geom, const tpc_params* params,
                              int64_t n_clusters, tpc_clusters in, tpc_refit_tracks trk,
                              const float* dist_map_dev, const tpc_material* mat,
                              const float* ckpt_dev,
                              const int32_t* status_dev, const float* grad_chi2_dev,
                              float* grad_map_dev, float* grad_x_dev, float* grad_y_dev,
                              float* grad_z_dev, void* ws_dev, size_t ws_bytes, void* stream);

/* Allocation-free variant of tpc_refit_backward, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid hipMalloc): the same kernels, with
 * the map-gradient accumulators and the overflow flag (the workspace of
 * tpc_refit_backward, tpc_refit_workspace_bytes() bytes) in a static array
 * of the library that each GPU holds once, for the whole process.  Its size
 * does not depend on the inputs, so no input is too large for it.  Every
 * call on a GPU shares that GPU's array, which each call clears itself
 * before use (with a kernel, no memset): calls that overlap on one GPU race
 * and must not be issued on concurrent streams.  Arguments, outputs and
 * errors as tpc_refit_backward; nothing is allocated, not even on the first
 * call on a device (which looks the array's address up once). */
tpc_status tpc_refit_backward_noalloc(const tpc_geometry* geom, const tpc_params* params,
                                      int64_t n_clusters, tpc_clusters in, tpc_refit_tracks trk,
                                      const float* dist_map_dev, const tpc_material* mat,
                                      const float* ckpt_dev,
                                      const int32_t* status_dev, const float* grad_chi2_dev,
                                      float* grad_map_dev, float* grad_x_dev, float* grad_y_dev,
                                      float* grad_z_dev, void* stream);

/* f3: cluster coordinate transformation with corrections -- the step before
 * tpc_grid_build.  Online TPC processing transforms the clusters' readout
 * coordinates into space points, and the paper's offline-only corrections
 * amend that transformation (Sec. 6: they cost about 20 % of the online
 * time by making the code more complicated); the formulas are this
 * library's (readings R31-R34 of the design notes):
 *   raw cluster  sector s (0..35 = phi-sector k + 18 side, side 1 = C at
 *                negative z), row r, pad and time (continuous pad and
 *                time-bin coordinates);
 *   nominal      x = row_x[r], y = (pad - pad_c[r]) * pad_w[r],
 *                drift d = (time * tbin_us - t0_us) * vdrift,
 *                z = zlen - d on side A, -(zlen - d) on side C;
 *   corrections  x += dist_map[r][k] (the radial map that tpc_refit fits;
 *                NULL: none), then a residual correction (dx, dy, dz)
 *                added to (x, y, z), interpolated trilinearly in
 *                (u = r, v = y / x, w = d) on a regular grid per sector s
 *                (corr_map [36][nu][nv][nw] nodes of four floats dx, dy, dz,
 *                unused; NULL: none): node i of an axis sits at
 *                q0 + i / iq, the cell is clamp(floor((q - q0) iq), 0, n - 2)
 *                and the fraction is clamped to [0, 1] (boundary values
 *                continue outside the grid); three rounds of
 *                lerp(a, b, t) = a + (b - a) t, along w, then v, then u.
 * A raw cluster with s >= 36 or r >= 152 gets row_out 0xFFFF (and x = y =
 * z = 0); non-finite pad or time give non-finite y or z.  tpc_grid_build
 * counts both as invalid.  The outputs are the tracker's x, y, z, row
 * arrays in the input order.  With TPC_FLAG_DETERMINISTIC the outputs equal
 * the binary32 CPU reference bit for bit.
 * Errors: TPC_ERR_INVALID (null pointers, n < 0, a grid axis with fewer
 * than 2 nodes, unknown flags), TPC_ERR_HIP. */
typedef struct {
  float row_x[TPC_N_ROWS];  /* pad-row planes [cm] */
  float pad_w[TPC_N_ROWS];  /* pad width [cm] */
  float pad_c[TPC_N_ROWS];  /* centre pad coordinate of the row */
  float tbin_us, vdrift_cm_us, zlen_cm, t0_us;
  int32_t nu, nv, nw;       /* residual-map nodes per axis */
  float u0, iu, v0, iv, w0, iw;  /* first node and inverse spacing per axis */
} tpc_transform_geometry;

typedef struct {
  const uint8_t* sector;
  const uint16_t* row;
  const float *pad, *time;
} tpc_raw_clusters;

tpc_status tpc_cluster_transform(const tpc_transform_geometry* tg, uint32_t flags,
                                 int64_t n_clusters, tpc_raw_clusters in,
                                 const float* dist_map_dev, const float* corr_map_dev,
                                 float* x_dev, float* y_dev, float* z_dev, uint16_t* row_dev,
                                 void* stream);

/* f1: sector-track merging and global refit.  The paper counts track
 * propagation in the magnetic field among the components TPC tracking
 * shares (Sec. 4) and judges the output by the cluster-to-track association
 * (Sec. 2); how the segments that one particle leaves in several sectors are
 * joined is this library's reading (R35-R41 of the design notes):
 *   - the instances are the 36 TPC sectors, i = k + 18 side (n_inst = 36);
 *     the segments are the tracks of tpc_sector_track;
 *   - each segment's outer state comes from an outward Kalman filter over
 *     its own hits (seeded at its first hit with its snp, tgl, q/pt);
 *   - segment A's outer state is compared with the inner state (the
 *     tracker's parameters at x_ref) of every segment B of sector k +- 1 on
 *     the same side or of sector k on the other side whose first hit lies
 *     within max_dz in z and max_dist in the transverse plane of A's last
 *     hit: A's state is rotated into B's frame (cos_d, sin_d: one sector's
 *     angle) and propagated to B's reference plane, and the chi2 of the
 *     five-parameter difference under the summed covariance (an LDL^T
 *     solve) must be <= chi2_max;
 *   - a link A -> B is kept iff B is A's best successor and A is B's best
 *     predecessor (minimum of (chi2, segment index)); chains follow the links
 *     from the segments without a predecessor, in the order of their first
 *     segment (then, for link cycles, from their lowest segment);
 *   - each chain is one merged track: its segments' hits in chain order,
 *     refitted by an outward filter (rotating at every change of sector)
 *     and an inward filter started from the outward end state with its
 *     covariance inflated a hundredfold; the inward state at the first hit
 *     is the output (frame of the first segment's sector), with the inward
 *     chi2 and ndf = 2 hits - 5; status 1 if a propagation or rotation
 *     failed (|snp| reaching 0.99, or the track turning back).
 * Every segment belongs to exactly one merged track.  The segment count and
 * hit count are read from seg_result_dev (n_tracks, n_hits), so the call can
 * follow tpc_sector_track on the same stream without a host round trip;
 * seg->cap_tracks and cap_hits bound them.  With TPC_FLAG_DETERMINISTIC the
 * outputs equal the binary32 CPU reference bit for bit.
 * Errors: TPC_ERR_INVALID (null pointers, n_inst != 36, capacities below
 * the segment arrays', unknown flags, seg->hit_data not 16-byte aligned),
 * TPC_ERR_WORKSPACE, TPC_ERR_HIP. */
typedef struct {
  float max_dz, max_dist, chi2_max;
  float cos_a[TPC_N_PHI], sin_a[TPC_N_PHI];  /* sector axis k at (k + 1/2) 20 deg */
  float cos_d, sin_d;                        /* the 20 deg between two sectors */
} tpc_merge_params;

/* Merged tracks (device arrays, caller-allocated, cap_tracks >= the
 * segment capacity, cap_hits >= the segments' hit capacity):
 *   param [cap][5], cov [cap][15], chi2, ndf, status, sector (phi sector of
 *   the output frame), x_ref (plane of the first hit);
 *   hit_off [cap + 1], hit_clu [cap_hits]   merged hit lists (input indices)
 *   seg_off [cap + 1], seg [cap]            the segments of each track
 *   next [cap]                              each segment's kept link (-1 none)
 *   counts [2] (int64)                      merged tracks, merged hits      */
typedef struct {
  float* param;
  float* cov;
  float* chi2;
  int32_t* ndf;
  int32_t* status;
  int32_t* sector;
  float* x_ref;
  int32_t* hit_off;
  int32_t* hit_clu;
  int32_t* seg_off;
  int32_t* seg;
  int32_t* next;
  int64_t* counts;
  int64_t cap_tracks, cap_hits;
} tpc_merged;

void tpc_default_merge_params(tpc_merge_params* m);
/* Workspace of tpc_merge_tracks for cap_segments = seg->cap_tracks and
 * cap_hits = seg->cap_hits (0 if either is negative). */
size_t tpc_merge_workspace_bytes(int64_t cap_segments, int64_t cap_hits);
tpc_status tpc_merge_tracks(const tpc_geometry* geom, const tpc_params* params,
                            const tpc_merge_params* mp, int32_t n_inst,
                            const int64_t* inst_off_dev, tpc_clusters in,
                            const tpc_tracks* seg, const tpc_result* seg_result_dev,
                            const tpc_merged* out, void* ws_dev, size_t ws_bytes, void* stream);

/* Optional per-kernel timing for benchmarks.  tpc_profile_enable(1) creates
 * a pool of HIP events (host call, once); afterwards every kernel the library
 * enqueues is bracketed by two events recorded on the stream it is launched
 * on, until the pool is used up.  tpc_profile_read synchronises those events
 * and returns per kernel name the summed elapsed time and launch count since
 * the previous read (at most max_entries rows; returns the number written, or
 * a negative tpc_status).  tpc_profile_enable(0) stops recording and frees
 * the pool.  Not thread-safe; profiling adds two event records per launch. */
typedef struct {
  char name[48];
  double total_ms;
  int64_t launches;
} tpc_kernel_time;

tpc_status tpc_profile_enable(int32_t on);
int32_t tpc_profile_read(tpc_kernel_time* out, int32_t max_entries);

#ifdef __cplusplus
}
#endif
#endif
