/*
 * Oracle of the cluster coordinate transformation (f3) -- TEST
 * INFRASTRUCTURE ONLY (loaded by the tests and the benchmark's CPU-baseline
 * leg, never by the product library; shares no code with the GPU path).
 *
 * The paper names the step and its cost, not its formulas: online TPC
 * processing transforms cluster coordinates, and offline-only corrections
 * amended that transformation at a cost of about 20 % of the online time
 * (Sec. 6).  Readings R31-R34 (design notes) define it here:
 *
 *   R31 a raw cluster is (sector 0..35, row 0..151, pad, time): sector
 *       s = k + 18 side, side 1 (C) at negative z; pad and time are
 *       continuous pad and time-bin coordinates.
 *   R32 nominal transform: x = X_r (the row's plane), y = (pad - c_r) w_r
 *       with the row's pad width w_r and centre pad c_r, drift distance
 *       d = (time tbin - t0) v_drift, z = L - d on side A, -(L - d) on C.
 *   R33 corrections, in this order: the radial plane offset
 *       x += D[row][k] (the map the refit fits), then a residual map per
 *       sector instance: (dx, dy, dz) interpolated trilinearly on a regular
 *       grid in (u = row, v = y / x, w = d), added to x, y, z.  Cell index
 *       clamp(floor(f), 0, n - 2), fraction clamp(f - i, 0, 1): outside the
 *       grid the boundary values continue (no extrapolation of slopes).
 *       The interpolation is three rounds of lerp(a, b, t) = a + (b - a) t:
 *       along w, then v, then u.
 *   R34 a raw cluster with sector >= 36 or row >= 152 comes out with row
 *       0xFFFF (the tracker counts it as invalid); non-finite pad or time
 *       give non-finite y or z (likewise invalid for the tracker).
 *
 * Compiled as binary32 (bit-exact reference of the deterministic GPU
 * kernel: every expression in the order written, no contraction) and as
 * binary64 (accuracy reference).
 */
#include <math.h>
#include <stdint.h>

#if defined(ORC_F64)
typedef double real;
#define FLOORR floor
#define TSFX(n) n##_f64
#else
typedef float real;
#define FLOORR floorf
#define TSFX(n) n##_f32
#endif

#define T_ROWS 152
#define T_SECTORS 36
#define T_PHI 18

/* transformation constants, host data (derived from the detector
 * description in binary64 and rounded once) */
typedef struct {
  float row_x[T_ROWS];
  float pad_w[T_ROWS];   /* pad width [cm]   */
  float pad_c[T_ROWS];   /* centre pad index */
  float tbin;            /* time-bin length [us]    */
  float vdrift;          /* drift velocity [cm/us]  */
  float zlen;            /* drift length [cm]       */
  float t0;              /* time offset of the call [us] */
  int32_t nu, nv, nw;    /* residual-map grid nodes per axis (>= 2 each) */
  float u0, iu;          /* u = row: first node and 1 / spacing */
  float v0, iv;          /* v = y / x */
  float w0, iw;          /* w = drift distance */
} orc_tgeom;

/* one axis of the trilinear lookup: cell index and fraction */
static void cell(real q, real q0, real iq, int n, int* i, real* a)
{
  real f = (q - q0) * iq;
  real fl = FLOORR(f);
  int k;
  if (!(fl > 0)) k = 0;                 /* also NaN */
  else if (fl > (real)(n - 2)) k = n - 2;
  else k = (int)fl;
  real t = f - (real)k;
  if (!(t > 0)) t = 0;
  if (t > 1) t = 1;
  *i = k;
  *a = t;
}

static real lerp(real a, real b, real t) { return a + (b - a) * t; }

/* map node (iu, iv, iw) of sector s, component c: float4 nodes (dx, dy, dz, 0) */
static real node(const float* map, const orc_tgeom* T, int s, int iu, int iv, int iw, int c)
{
  int64_t n = (((int64_t)s * T->nu + iu) * T->nv + iv) * T->nw + iw;
  return (real)map[n * 4 + c];
}

/* f3: transform n raw clusters.  dmap [152][18] radial offsets (may be
 * NULL: none), rmap [36][nu][nv][nw][4] residual corrections (may be NULL:
 * none).  Outputs x, y, z and the tracker's row (0xFFFF for R34). */
void TSFX(orc_transform)(const orc_tgeom* T, int64_t n, const uint8_t* sector,
                         const uint16_t* row, const float* pad, const float* time,
                         const float* dmap, const float* rmap, real* x, real* y, real* z,
                         uint16_t* row_out)
{
  for (int64_t c = 0; c < n; c++) {
    const int s = sector[c], r = row[c];
    if (s >= T_SECTORS || r >= T_ROWS) {
      x[c] = 0;
      y[c] = 0;
      z[c] = 0;
      row_out[c] = 0xFFFF;
      continue;
    }
    const int side = s >= T_PHI;
    const int k = s - T_PHI * side;
    /* R32 */
    real xc = (real)T->row_x[r];
    real yc = ((real)pad[c] - (real)T->pad_c[r]) * (real)T->pad_w[r];
    real d = ((real)time[c] * (real)T->tbin - (real)T->t0) * (real)T->vdrift;
    real za = (real)T->zlen - d;
    real zc = side ? -za : za;
    /* R33 (a) */
    if (dmap) xc = xc + (real)dmap[r * T_PHI + k];
    /* R33 (b) */
    if (rmap) {
      int iu, iv, iw;
      real au, av, aw;
      cell((real)r, (real)T->u0, (real)T->iu, T->nu, &iu, &au);
      cell(yc / xc, (real)T->v0, (real)T->iv, T->nv, &iv, &av);
      cell(d, (real)T->w0, (real)T->iw, T->nw, &iw, &aw);
      real corr[3];
      for (int q = 0; q < 3; q++) {
        real e00 = lerp(node(rmap, T, s, iu, iv, iw, q), node(rmap, T, s, iu, iv, iw + 1, q), aw);
        real e01 = lerp(node(rmap, T, s, iu, iv + 1, iw, q),
                        node(rmap, T, s, iu, iv + 1, iw + 1, q), aw);
        real e10 = lerp(node(rmap, T, s, iu + 1, iv, iw, q),
                        node(rmap, T, s, iu + 1, iv, iw + 1, q), aw);
        real e11 = lerp(node(rmap, T, s, iu + 1, iv + 1, iw, q),
                        node(rmap, T, s, iu + 1, iv + 1, iw + 1, q), aw);
        real f0 = lerp(e00, e01, av);
        real f1 = lerp(e10, e11, av);
        corr[q] = lerp(f0, f1, au);
      }
      xc = xc + corr[0];
      yc = yc + corr[1];
      zc = zc + corr[2];
    }
    x[c] = xc;
    y[c] = yc;
    z[c] = zc;
    row_out[c] = (uint16_t)r;
  }
}
