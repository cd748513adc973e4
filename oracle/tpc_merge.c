/*
 * Oracle of sector-track merging and the global refit (f1) -- TEST
 * INFRASTRUCTURE ONLY (loaded by the tests and the benchmark's CPU-baseline
 * leg, never by the product library; shares no code with the GPU path).
 *
 * The paper places track propagation with the magnetic field among the
 * components that TPC tracking shares (Sec. 4) and judges the output by the
 * cluster-to-track association (Sec. 2), but does not describe how the
 * segments that one particle leaves in several sectors are joined.  Readings
 * R35-R41 (design notes) define it here:
 *
 *   R35 instances are the 36 TPC sectors, i = k + 18 side (k the phi
 *       sector, side 1 = C); a segment is a track of the sector tracker
 *       (parameters and covariance at its innermost hit, hit list).
 *   R36 a state moves from the frame of phi sector k to that of k' by the
 *       rotation by the angle between the two sector axes, followed by the
 *       move to the rotated point's plane along the track (first order in
 *       the covariance: the Jacobian below); a rotation fails unless the
 *       track still moves outward in the new frame (cos phi' > 0) with
 *       |snp'| < 0.99.  It is taken at the state's point, or, if that or
 *       the move after it fails, at the target point (m_transport).
 *   R37 segment A's outer state (an outward filter over its own hits, seeded
 *       as the refit does with the segment's snp, tgl, q/pt) is compared
 *       with the inner state of a segment B of a neighbouring sector of the
 *       same side (k +- 1) or of the same sector on the other side: A's
 *       last hit and B's first hit within max_dz in z and max_dist in the
 *       transverse plane, A's outer state rotated into B's frame and
 *       propagated to B's reference plane, chi2 of the 5 parameter
 *       difference with the summed covariance (LDL^T solve) <= chi2_max.
 *   R38 every segment keeps its best successor and its best predecessor
 *       (minimum of (chi2, index)); a link A -> B holds iff each is the
 *       other's best: chains follow the links from segments without a
 *       predecessor, in the order of their first segment.
 *   R39 a merged track's hits are its segments' hit lists in chain order.
 *   R40 global refit: outward Kalman filter over the merged hits (seeded at
 *       the first hit with the first segment's snp, tgl, q/pt and the
 *       tracker's start covariance), rotating at every change of phi
 *       sector, then an inward filter from the outward end state with its
 *       covariance inflated a hundredfold, back to the first hit; its state
 *       there is the output, with the inward chi2 and ndf = 2 hits - 5.
 *       (Restarting the inward pass from the start covariance instead lost
 *       positive definiteness in binary32 on low-pT tracks: the update
 *       subtracts nearly equal numbers when the q/pt variance drops by five
 *       orders of magnitude.)
 *   R41 every segment belongs to exactly one output track; a refit that
 *       fails (propagation or rotation) gives status 1.
 *
 * Compiled as binary32 (bit-exact reference of the deterministic GPU
 * kernels) and binary64.
 */
#include "tpc_oracle.h"

#include <stdlib.h>
#include <string.h>

#include "kalman.h"

#define M_PHI 18
#define M_INST 36
#define INWARD_SCALE 100

typedef struct {
  float max_dz, max_dist, chi2_max;
  float cos_a[M_PHI], sin_a[M_PHI];  /* sector axis directions */
  float cos_d, sin_d;                /* rotation by one sector (20 deg) */
} orc_mparams;

/* R36: rotate state s by (ca, sa) = (cos, sin) of (new axis - old axis); x
 * is the plane of s, *xn receives the new plane.  Returns 0 on failure. */
static int m_rotate(kst* s, real x, real ca, real sa, real kB, real smax, real* xn)
{
  const real one = 1;
  const real snp = s->p[2];
  if (!(FABS(snp) < smax)) return 0;
  const real csp = SQRT((one - snp) * (one + snp));
  const real csn = csp * ca + snp * sa;          /* cos(phi - delta) */
  const real snn = snp * ca - csp * sa;          /* sin(phi - delta) */
  if (!(csn > 0) || !(FABS(snn) < smax)) return 0;
  const real y = s->p[0];
  *xn = x * ca + y * sa;
  s->p[0] = y * ca - x * sa;
  s->p[2] = snn;
  /* first-order Jacobian of (rotate, move to the new plane along the
   * track): rows y, z, snp depend on y; snp on snp */
  const real j00 = ca - sa * (snn / csn);
  const real j10 = -(s->p[3] * (sa / csn));
  const real j20 = -(kB * s->p[4]) * sa;
  const real j22 = csn / csp;
  /* C' = J C J^T with J = I except rows 0, 1, 2:
   * row0 = j00 e0, row1 = e1 + j10 e0, row2 = j20 e0 + j22 e2 */
  real c[5][5];
  for (int i = 0; i < 5; i++)
    for (int j = 0; j < 5; j++) c[i][j] = CC(s, i, j);
  real t[5][5]; /* T = J C */
  for (int j = 0; j < 5; j++) {
    t[0][j] = j00 * c[0][j];
    t[1][j] = c[1][j] + j10 * c[0][j];
    t[2][j] = j20 * c[0][j] + j22 * c[2][j];
    t[3][j] = c[3][j];
    t[4][j] = c[4][j];
  }
  for (int i = 0; i < 5; i++) { /* C' = T J^T, lower triangle */
    real r0 = j00 * t[i][0];
    real r1 = t[i][1] + j10 * t[i][0];
    real r2 = j20 * t[i][0] + j22 * t[i][2];
    real r[5] = {r0, r1, r2, t[i][3], t[i][4]};
    for (int j = 0; j <= i; j++) s->c[ci(i, j)] = r[j];
  }
  return 1;
}

/* chi2 of d^T S^-1 d for symmetric S (lower triangle, ci order) by LDL^T;
 * returns a negative value if S is not positive definite */
static real m_chi2(const real* S, const real* d)
{
  real L[5][5], D[5];
  for (int i = 0; i < 5; i++) {
    for (int j = 0; j < i; j++) {
      real v = S[ci(i, j)];
      for (int k = 0; k < j; k++) v = v - L[i][k] * (L[j][k] * D[k]);
      L[i][j] = v / D[j];
    }
    real v = S[ci(i, i)];
    for (int k = 0; k < i; k++) v = v - L[i][k] * (L[i][k] * D[k]);
    if (!(v > 0)) return -1;
    D[i] = v;
  }
  real w[5], chi2 = 0;
  for (int i = 0; i < 5; i++) {
    real v = d[i];
    for (int k = 0; k < i; k++) v = v - L[i][k] * w[k];
    w[i] = v;
    chi2 = chi2 + (v * v) / D[i];
  }
  return chi2;
}

static int inst_of(const int64_t* inst_off, int n_inst, int64_t c)
{
  int lo = 0, hi = n_inst;
  while (hi - lo > 1) {
    int m = (lo + hi) / 2;
    if (inst_off[m] <= c) lo = m; else hi = m;
  }
  return lo;
}

/* move state s from plane x1 to plane x2 (nothing to do when equal) */
static int m_move(kst* s, real x1, real x2, real kB)
{
  if (x1 == x2) return 1;
  return k_propagate(s, x1, x2, kB, (real)0.99);
}

/* R36: bring state s (plane *x of the current frame) into the frame rotated
 * by (ca, sa) and onto the plane xh there, where the point (xh, yh) lies.
 * The rotation is taken at the state's point; if that fails or the move
 * from there fails (|snp| reaching the limit in one of the frames), it is
 * taken at the target point instead: the state first moves in the current
 * frame to the target point's plane (its coordinate xh ca - yh sa there),
 * then rotates, then moves to xh.  Returns 0 if both fail. */
static int m_transport(kst* s, real* x, real ca, real sa, real xh, real yh, real kB)
{
  kst t = *s;
  real xr;
  if (m_rotate(&t, *x, ca, sa, kB, (real)0.99, &xr) && m_move(&t, xr, xh, kB)) {
    *s = t;
    *x = xh;
    return 1;
  }
  t = *s;
  const real xc = xh * ca - yh * sa;
  if (m_move(&t, *x, xc, kB) && m_rotate(&t, xc, ca, sa, kB, (real)0.99, &xr) &&
      m_move(&t, xr, xh, kB)) {
    *s = t;
    *x = xh;
    return 1;
  }
  return 0;
}

/* R40: filter over the merged hits hits[first], hits[first + dir], ...
 * (count of them), from state s at plane *x in phi-sector frame *k:
 * rotation at a change of sector, propagation to the hit's plane, update.
 * Returns 0 on a failure; chi2 accumulates. */
static int m_pass(const orc_geom* g, const orc_mparams* M, kst* s, real* x, int* k,
                  const int32_t* hits, int64_t first, int64_t count, int dir,
                  const int64_t* inst_off, const uint16_t* row, const float* y, const float* z,
                  real* chi2)
{
  const real kB = (real)(-0.299792458e-2 * (double)g->bz);
  const real vy = (real)g->sigma_y2, vz = (real)g->sigma_z2;
  for (int64_t q = 0; q < count; q++) {
    const int64_t c = hits[first + dir * q];
    const int kk = inst_of(inst_off, M_INST, c) % M_PHI;
    const real xh = (real)g->row_x[row[c]];
    if (kk != *k) {
      const int up = (kk - *k + M_PHI) % M_PHI == 1;   /* the next sector: +20 deg */
      const real sa = up ? (real)M->sin_d : -(real)M->sin_d;
      if (!m_transport(s, x, (real)M->cos_d, sa, xh, (real)y[c], kB)) return 0;
      *k = kk;
    } else {
      if (!m_move(s, *x, xh, kB)) return 0;
      *x = xh;
    }
    *chi2 = *chi2 + k_update(s, (real)y[c], (real)z[c], vy, vz);
  }
  return 1;
}

/* the start state of a filter at cluster c: its (y, z), the seed's snp,
 * tgl, q/pt, the tracker's start covariance */
static void m_seed(const orc_geom* g, kst* s, const float* y, const float* z, int64_t c,
                   const real* p5)
{
  s->p[0] = (real)y[c];
  s->p[1] = (real)z[c];
  s->p[2] = p5[2];
  s->p[3] = p5[3];
  s->p[4] = p5[4];
  k_init_cov(s, (real)g->sigma_y2, (real)g->sigma_z2);
}

/* R37: chi2 of segment A's outer state against segment B's inner state, or
 * -1 if the pair is not a candidate */
static real m_pair(const orc_geom* g, const orc_mparams* M, int64_t A, int64_t B,
                   const int* seg_k, const int* seg_side, const int32_t* hit_off,
                   const int32_t* hit_clu, const uint16_t* row, const float* y, const float* z,
                   const real* par, const real* cov, const float* x_ref, const int* out_ok,
                   const real* out_p, const real* out_c, const real* out_x)
{
  const real kB = (real)(-0.299792458e-2 * (double)g->bz);
  if (!out_ok[A]) return -1;
  const int ka = seg_k[A], kb = seg_k[B];
  const int nb = (kb - ka + M_PHI) % M_PHI;
  const int same_side = seg_side[A] == seg_side[B];
  if (!((same_side && (nb == 1 || nb == M_PHI - 1)) || (!same_side && nb == 0))) return -1;
  /* global positions of A's last and B's first hit */
  const int64_t ca = hit_clu[hit_off[A + 1] - 1], cb = hit_clu[hit_off[B]];
  const real xa = (real)g->row_x[row[ca]], xb = (real)g->row_x[row[cb]];
  const real ga0 = xa * (real)M->cos_a[ka] - (real)y[ca] * (real)M->sin_a[ka];
  const real ga1 = xa * (real)M->sin_a[ka] + (real)y[ca] * (real)M->cos_a[ka];
  const real gb0 = xb * (real)M->cos_a[kb] - (real)y[cb] * (real)M->sin_a[kb];
  const real gb1 = xb * (real)M->sin_a[kb] + (real)y[cb] * (real)M->cos_a[kb];
  const real d0 = ga0 - gb0, d1 = ga1 - gb1;
  if (!(FABS((real)z[ca] - (real)z[cb]) <= (real)M->max_dz)) return -1;
  if (!(d0 * d0 + d1 * d1 <= (real)M->max_dist * (real)M->max_dist)) return -1;
  kst s;
  for (int j = 0; j < 5; j++) s.p[j] = out_p[A * 5 + j];
  for (int j = 0; j < 15; j++) s.c[j] = out_c[A * 15 + j];
  real x = out_x[A];
  if (nb != 0) {
    const real sa = nb == 1 ? (real)M->sin_d : -(real)M->sin_d;
    if (!m_transport(&s, &x, (real)M->cos_d, sa, (real)x_ref[B], par[B * 5 + 0], kB)) return -1;
  } else if (!m_move(&s, x, (real)x_ref[B], kB)) {
    return -1;
  }
  real d[5], S[15];
  for (int j = 0; j < 5; j++) d[j] = s.p[j] - par[B * 5 + j];
  for (int j = 0; j < 15; j++) S[j] = s.c[j] + cov[B * 15 + j];
  real chi2 = m_chi2(S, d);
  if (!(chi2 >= 0) || !(chi2 <= (real)M->chi2_max)) return -1;
  return chi2;
}

/*
 * f1 -- merge the segments of the 36 sector instances and refit the merged
 * tracks.  Inputs: the sector tracker's tracks (par [n][5], cov [n][15] at
 * x_ref, hit lists of input indices), the clusters (y, z, row by input
 * index; inst_off [37]).  Outputs (all caller-allocated):
 *   out_ok/out_p/out_c/out_x [n]  each segment's outer state (R37)
 *   succ, pred [n]                best successor / predecessor (-1 none)
 *   next [n]                      kept link (-1 none)
 *   chain_off [n+1], chain_seg [n] chains in output order
 *   m_hit_off [n+1], m_hit_clu [total hits]  merged hit lists
 *   m_par [n][5], m_cov [n][15], m_chi2 [n], m_ndf [n], m_status [n],
 *   m_k [n] (phi sector of the output frame), m_xref [n]
 * Returns the number of merged tracks.
 */
int64_t SFX(orc_merge)(const orc_geom* g, const orc_mparams* M, int64_t n, const real* par,
                       const real* cov, const float* x_ref, const int32_t* hit_off,
                       const int32_t* hit_clu, const int64_t* inst_off, const uint16_t* row,
                       const float* y, const float* z, int32_t* out_ok, real* out_p, real* out_c,
                       real* out_x, int32_t* succ, int32_t* pred, real* succ_chi2,
                       real* pred_chi2, int32_t* next, int32_t* chain_off, int32_t* chain_seg,
                       int32_t* m_hit_off, int32_t* m_hit_clu, real* m_par, real* m_cov,
                       real* m_chi2, int32_t* m_ndf, int32_t* m_status, int32_t* m_k,
                       float* m_xref)
{
  int* seg_k = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
  int* seg_side = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
  int* ok = (int*)malloc(sizeof(int) * (n > 0 ? n : 1));
  char* seen = (char*)calloc(n > 0 ? n : 1, 1);
  /* segments' sectors and outer states (R35, R37) */
  for (int64_t t = 0; t < n; t++) {
    const int64_t a = hit_off[t], b = hit_off[t + 1];
    const int inst = inst_of(inst_off, M_INST, hit_clu[a]);
    seg_k[t] = inst % M_PHI;
    seg_side[t] = inst / M_PHI;
    kst s;
    m_seed(g, &s, y, z, hit_clu[a], par + t * 5);
    real x = (real)g->row_x[row[hit_clu[a]]];
    int k = seg_k[t];
    real chi2 = 0;
    ok[t] = m_pass(g, M, &s, &x, &k, hit_clu, a + 1, b - a - 1, 1, inst_off, row, y, z, &chi2);
    out_ok[t] = ok[t];
    for (int j = 0; j < 5; j++) out_p[t * 5 + j] = ok[t] ? s.p[j] : 0;
    for (int j = 0; j < 15; j++) out_c[t * 15 + j] = ok[t] ? s.c[j] : 0;
    out_x[t] = ok[t] ? x : 0;
  }
  /* best successor and predecessor over all candidate pairs (R37, R38) */
  for (int64_t t = 0; t < n; t++) {
    succ[t] = pred[t] = -1;
    succ_chi2[t] = pred_chi2[t] = 0;
  }
  for (int64_t A = 0; A < n; A++)
    for (int64_t B = 0; B < n; B++) {
      if (A == B) continue;
      real c2 = m_pair(g, M, A, B, seg_k, seg_side, hit_off, hit_clu, row, y, z, par, cov, x_ref,
                       ok, out_p, out_c, out_x);
      if (c2 < 0) continue;
      if (succ[A] < 0 || c2 < succ_chi2[A]) { succ[A] = (int32_t)B; succ_chi2[A] = c2; }
      if (pred[B] < 0 || c2 < pred_chi2[B]) { pred[B] = (int32_t)A; pred_chi2[B] = c2; }
    }
  int* has_pred = (int*)calloc(n > 0 ? n : 1, sizeof(int));
  for (int64_t A = 0; A < n; A++) {
    next[A] = -1;
    if (succ[A] >= 0 && pred[succ[A]] == A) {
      next[A] = succ[A];
      has_pred[succ[A]] = 1;
    }
  }
  /* chains: from every segment without a kept predecessor, then (cycles)
   * from every segment not reached yet, each in index order (R38, R41) */
  int64_t nc = 0, ns = 0;
  for (int pass = 0; pass < 2; pass++)
    for (int64_t t = 0; t < n; t++) {
      if (seen[t] || (pass == 0 && has_pred[t])) continue;
      chain_off[nc] = (int32_t)ns;
      for (int64_t u = t; u >= 0 && !seen[u]; u = next[u]) {
        seen[u] = 1;
        chain_seg[ns++] = (int32_t)u;
      }
      nc++;
    }
  chain_off[nc] = (int32_t)ns;
  /* merged hit lists (R39) and the global refit (R40) */
  int64_t nh = 0;
  for (int64_t m = 0; m < nc; m++) {
    m_hit_off[m] = (int32_t)nh;
    for (int64_t q = chain_off[m]; q < chain_off[m + 1]; q++) {
      const int64_t t = chain_seg[q];
      for (int64_t h = hit_off[t]; h < hit_off[t + 1]; h++) m_hit_clu[nh++] = hit_clu[h];
    }
  }
  m_hit_off[nc] = (int32_t)nh;
  for (int64_t m = 0; m < nc; m++) {
    const int64_t a = m_hit_off[m], b = m_hit_off[m + 1];
    const int64_t t0 = chain_seg[chain_off[m]];
    kst s;
    m_seed(g, &s, y, z, m_hit_clu[a], par + t0 * 5);
    real x = (real)g->row_x[row[m_hit_clu[a]]];
    int k = seg_k[t0];
    real chi2 = 0;
    int good = m_pass(g, M, &s, &x, &k, m_hit_clu, a + 1, b - a - 1, 1, inst_off, row, y, z,
                      &chi2);
    if (good) {
      /* inward: the outward end state with its covariance inflated by
       * INWARD_SCALE (the outward result only seeds the inward pass); the
       * last hit updates it in place, then back to the first hit */
      for (int j = 0; j < 15; j++) s.c[j] = s.c[j] * (real)INWARD_SCALE;
      chi2 = 0;
      good = m_pass(g, M, &s, &x, &k, m_hit_clu, b - 1, b - a, -1, inst_off, row, y, z, &chi2);
    }
    m_status[m] = good ? 0 : 1;
    for (int j = 0; j < 5; j++) m_par[m * 5 + j] = good ? s.p[j] : 0;
    for (int j = 0; j < 15; j++) m_cov[m * 15 + j] = good ? s.c[j] : 0;
    m_chi2[m] = good ? chi2 : 0;
    m_ndf[m] = (int32_t)(2 * (b - a) - 5);
    m_k[m] = k;
    m_xref[m] = (float)x;
  }
  free(seg_k);
  free(seg_side);
  free(ok);
  free(seen);
  free(has_pred);
  return nc;
}

/* R36 alone (for the pins): rotate state p, c at plane x into the frame of
 * the next (up != 0) or the previous phi sector */
int SFX(orc_rotate)(const orc_geom* g, const orc_mparams* M, real* p, real* c, real x, int up,
                    real* xn)
{
  kst s;
  memcpy(s.p, p, sizeof(s.p));
  memcpy(s.c, c, sizeof(s.c));
  const real kB = (real)(-0.299792458e-2 * (double)g->bz);
  const real sa = up ? (real)M->sin_d : -(real)M->sin_d;
  int ok = m_rotate(&s, x, (real)M->cos_d, sa, kB, (real)0.99, xn);
  memcpy(p, s.p, sizeof(s.p));
  memcpy(c, s.c, sizeof(s.c));
  return ok;
}

/* the LDL^T chi2 alone (for the pins) */
real SFX(orc_chi2_5)(const real* S, const real* d) { return m_chi2(S, d); }
