/*
 * CPU oracle of the TPC sector tracker -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, single-threaded C implementation of the tracking chain written
 * from the algorithm readings (grid binning, neighbour finding and cleaning,
 * start hits, tracklet construction with an extended Kalman helix fit,
 * tracklet selection, Kalman refit and its adjoint).  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never does.  It shares no code with the GPU path.
 *
 * The same source is compiled twice: with `real` = float (suffix _f32, the
 * bit-exact reference for the deterministic GPU mode, built without FP
 * contraction as the paper's deterministic mode requires: Sec. 2, the
 * compile-time list) and with `real` = double (suffix _f64, the accuracy
 * reference).
 *
 * Conventions (both builds):
 *   - clusters are SoA arrays over all instances; instance i owns input
 *     indices [inst_off[i], inst_off[i+1]);
 *   - the grid sorts the valid clusters of each instance by
 *     (row, bin, input index) into positions [inst_off[i], inst_off[i]+n_valid);
 *     positions past n_valid are padding (sseg = perm = -1, ys = zs = 0);
 *   - links, start hits and tracklet hits are global sorted positions;
 *   - track hit lists and clu2trk use input indices.
 */
#ifndef TPC_ORACLE_H
#define TPC_ORACLE_H
#include <stdint.h>

#define ORC_MAX_ROWS 152

typedef struct {
  int32_t n_rows;
  float row_x[ORC_MAX_ROWS];
  float bz;
  float tan_half;
  float sigma_y2, sigma_z2;
} orc_geom;

typedef struct {
  float nf_win_y, nf_win_z, nf_chi2_max;
  float tc_chi2_pick, snp_max;
  float grid_occupancy;
  float edge_margin, search_margin;
  float y_valid_margin;
  int32_t min_chain, tc_max_miss, min_tracklet_hits, min_track_hits;
} orc_params;

/* field map and material of the refit (readings R42-R44; any pointer may
 * be NULL: uniform field of the geometry, no material) */
typedef struct {
  const float* bz;     /* [152][nzb] solenoid field [T] per row and z bin */
  int32_t nzb;         /* z bins over [-250, 250] cm */
  const float* ix0;    /* [152] inverse radiation length [1/cm] per row */
  const float* eloss;  /* [152] mean energy loss at minimum ionisation [GeV/cm] per row */
} orc_material;

#endif
