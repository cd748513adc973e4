// The standard configuration as kernel constants: the detector description
// of the synthetic events (152 planes from 85 to 247 cm, B = 0.5 T,
// sigma_y^2 = 0.01, sigma_z^2 = 0.0225 cm^2, 20-degree sectors) and the
// default algorithm parameters, derived exactly as the launcher derives
// them from a tpc_geometry and tpc_params.  Kernels instantiated for it read
// these at compile time (the compile-time analogue of the paper's run-time
// compilation, Sec. 5: settings become constants the compiler folds); the
// launcher selects them only when a call's constants equal these bit for
// bit.
#pragma once
#include "tpc_internal.h"

namespace tpcca {

constexpr float kStdTanHalf = 0x1.691e1ep-3f;  // binary32 tan(10 degrees)

constexpr Consts standard_consts()
{
  Consts k{};
  for (int r = 0; r < kRows; r++) k.row_x[r] = (float)(85.0 + r * (162.0 / 151.0));
  k.tan_half = kStdTanHalf;
  k.kB = (float)(-0.299792458e-2 * 0.5);
  k.bz = 0.5f;
  k.vy = 0.01f;
  k.vz = 0.0225f;
  k.ivy = (float)(1.0 / (1.5 * (double)0.01f));
  k.ivz = (float)(1.0 / (1.5 * (double)0.0225f));
  k.nf_win_y = 3.0f;
  k.nf_win_z = 3.5f;
  k.nf_chi2_max = 13.8f;
  k.tc_chi2_pick = 13.8f;
  k.snp_max = 0.99f;
  k.grid_occupancy = 0.0f;  // performance-only: not part of the comparison
  k.edge_margin = 1.0f;
  k.search_margin = 0.01f;
  k.y_valid_margin = 2.0f;
  k.min_chain = 3;
  k.tc_max_miss = 10;
  k.min_tracklet_hits = 10;
  k.min_track_hits = 10;
  k.tl_chunk = 0;           // performance-only: not part of the comparison
  return k;
}

constexpr Consts kStdConsts = standard_consts();

}  // namespace tpcca
