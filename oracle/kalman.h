/*
 * Kalman-filter core shared by the oracle's tracker and refit sources
 * (oracle-internal; test infrastructure only).  Readings R7 (propagation),
 * R8 (its Jacobian) and R9 (measurement update); see tpc_oracle.c.
 * The includer is compiled with ORC_F64, ORC_C128 or neither (binary32).
 */
#ifndef TPC_ORACLE_KALMAN_H
#define TPC_ORACLE_KALMAN_H
#include <math.h>
#include <string.h>

#if defined(ORC_C128)
/* complex binary64: the complex-step derivative check of the refit */
#include <complex.h>
typedef double _Complex real;
#define SQRT csqrt
#define FABS(x) fabs(creal(x))
#define RE(x) creal(x)
#define SFX(n) n##_c128
#define K_SIXTH (1.0 / 6.0)
#define K_3_40 (3.0 / 40.0)
#define K_3_20 (3.0 / 20.0)
#elif defined(ORC_F64)
typedef double real;
#define SQRT sqrt
#define FABS fabs
#define RE(x) (x)
#define FLOOR floor
#define CEIL ceil
#define SFX(n) n##_f64
#define K_SIXTH (1.0 / 6.0)
#define K_3_40 (3.0 / 40.0)
#define K_3_20 (3.0 / 20.0)
#else
typedef float real;
#define SQRT sqrtf
#define FABS fabsf
#define RE(x) (x)
#define FLOOR floorf
#define CEIL ceilf
#if defined(ORC_F32C)
/* binary32 built with contraction (fused multiply-add): a second rounding
 * realisation of the same formulas, for the production-mode bounds */
#define SFX(n) n##_f32c
#else
#define SFX(n) n##_f32
#endif
/* 1/6, 3/40 and 3/20 rounded to binary32 (exact hex literals) */
#define K_SIXTH 0x1.555556p-3f
#define K_3_40 0x1.333334p-4f
#define K_3_20 0x1.333334p-3f
#endif

/* ------------------------------------------------------------------------ */
/* Kalman filter pieces.  State p = (y, z, snp, tgl, qpt) at plane x; the
 * covariance C is stored as its lower triangle in the order
 * 00,10,11,20,21,22,30,31,32,33,40,41,42,43,44. */
typedef struct {
  real p[5];
  real c[15];
} kst;

static int ci(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }
#define CC(s, i, j) ((s)->c[ci((i), (j))])

/*
 * R7 + R8: move the state from plane x1 to plane x2 along the helix of
 * curvature kB*qpt (sin(phi) is linear in x; dy from the chord; the arc
 * length from the chord via the series of asin(u)/u), then C <- F C F^T with
 * F the exact derivative of these formulas.  Returns 0 (state untouched)
 * if |snp| would reach snp_max.
 */
static int k_propagate_ds(kst* s, real x1, real x2, real kB, real snp_max, real* ds_out);

static int k_propagate(kst* s, real x1, real x2, real kB, real snp_max)
{
  real ds;
  return k_propagate_ds(s, x1, x2, kB, snp_max, &ds);
}

/* the same, also returning the step's signed transverse arc length ds */
static int k_propagate_ds(kst* s, real x1, real x2, real kB, real snp_max, real* ds_out)
{
  const real one = 1;
  real dx = x2 - x1;
  real snp = s->p[2], tgl = s->p[3], qpt = s->p[4];
  real cc = kB * qpt;
  real s2 = snp + cc * dx;
  /* the step is defined only for |sin phi| < 1 at both ends (cos phi real) */
  if (!(FABS(snp) < RE(snp_max)) || !(FABS(s2) < RE(snp_max))) return 0;
  real c1 = SQRT((one - snp) * (one + snp));
  real c2 = SQRT((one - s2) * (one + s2));
  real f = (snp + s2) / (c1 + c2);
  real dy = dx * f;
  real L = SQRT(dx * dx + dy * dy);
  real lc = L * cc;
  real u2 = (lc * lc) * (real)0.25;
  real g = one + u2 * (K_SIXTH + u2 * K_3_40);
  real sg = RE(dx) < 0 ? -one : one;
  real ds = (sg * L) * g;
  *ds_out = ds;
  /* Jacobian entries */
  real h = (one + f * f) * (real)0.5;
  real ic1 = one / c1, ic2 = one / c2;
  real dfs = h * (ic1 + ic2);
  real dfq = (h * (dx * ic2)) * kB;
  real dg = K_SIXTH + u2 * K_3_20;
  real dyl = dy / L;
  real hlc = (real)0.5 * lc;
  real Lg = L * dg;
  real a = dx * dfs;                  /* dy/dsnp */
  real dLs = dyl * a;
  real du2s = hlc * (dLs * cc);
  real d = tgl * (sg * (dLs * g + Lg * du2s)); /* dz/dsnp */
  real b = dx * dfq;                  /* dy/dqpt */
  real dLq = dyl * b;
  real du2q = hlc * (dLq * cc + L * kB);
  real gq = tgl * (sg * (dLq * g + Lg * du2q)); /* dz/dqpt */
  real e = ds;                        /* dz/dtgl */
  real hq = kB * dx;                  /* dsnp/dqpt */
  /* state */
  s->p[0] = s->p[0] + dy;
  s->p[1] = s->p[1] + tgl * ds;
  s->p[2] = s2;
  /* B = F C (rows y, z, snp; rows tgl, qpt are unchanged) */
  real B0[5], B1[5], B2[5];
  for (int j = 0; j < 5; j++) {
    B0[j] = (CC(s, 0, j) + a * CC(s, 2, j)) + b * CC(s, 4, j);
    B1[j] = ((CC(s, 1, j) + d * CC(s, 2, j)) + e * CC(s, 3, j)) + gq * CC(s, 4, j);
    B2[j] = CC(s, 2, j) + hq * CC(s, 4, j);
  }
  real n30 = (CC(s, 3, 0) + a * CC(s, 3, 2)) + b * CC(s, 3, 4);
  real n31 = ((CC(s, 3, 1) + d * CC(s, 3, 2)) + e * CC(s, 3, 3)) + gq * CC(s, 3, 4);
  real n32 = CC(s, 3, 2) + hq * CC(s, 3, 4);
  real n40 = (CC(s, 4, 0) + a * CC(s, 4, 2)) + b * CC(s, 4, 4);
  real n41 = ((CC(s, 4, 1) + d * CC(s, 4, 2)) + e * CC(s, 4, 3)) + gq * CC(s, 4, 4);
  real n42 = CC(s, 4, 2) + hq * CC(s, 4, 4);
  /* C' = B F^T, lower triangle */
  s->c[0] = (B0[0] + a * B0[2]) + b * B0[4];
  s->c[1] = (B1[0] + a * B1[2]) + b * B1[4];
  s->c[2] = ((B1[1] + d * B1[2]) + e * B1[3]) + gq * B1[4];
  s->c[3] = (B2[0] + a * B2[2]) + b * B2[4];
  s->c[4] = ((B2[1] + d * B2[2]) + e * B2[3]) + gq * B2[4];
  s->c[5] = B2[2] + hq * B2[4];
  s->c[6] = n30;
  s->c[7] = n31;
  s->c[8] = n32;
  /* c[9] = C33 unchanged */
  s->c[10] = n40;
  s->c[11] = n41;
  s->c[12] = n42;
  /* c[13] = C43, c[14] = C44 unchanged */
  return 1;
}

/* R9: inverse of the 2x2 innovation covariance S = H C H^T + V */
typedef struct {
  real S00, S11, si00, si01, si11;
} kinn;

static kinn k_innov(const kst* s, real vy, real vz)
{
  kinn q;
  real S00 = s->c[0] + vy, S01 = s->c[1], S11 = s->c[2] + vz;
  real det = S00 * S11 - S01 * S01;
  q.S00 = S00;
  q.S11 = S11;
  q.si00 = S11 / det;
  q.si01 = -(S01 / det);
  q.si11 = S00 / det;
  return q;
}

static real k_chi2(const kinn* q, real r0, real r1)
{
  return r0 * (q->si00 * r0 + q->si01 * r1) + r1 * (q->si01 * r0 + q->si11 * r1);
}

/* R9: measurement update with cluster (my, mz); returns its chi2 */
static real k_update(kst* s, real my, real mz, real vy, real vz)
{
  kinn q = k_innov(s, vy, vz);
  real r0 = my - s->p[0], r1 = mz - s->p[1];
  real chi2 = k_chi2(&q, r0, r1);
  real k0[5], k1[5], hc0[5], hc1[5];
  for (int i = 0; i < 5; i++) {
    k0[i] = CC(s, i, 0) * q.si00 + CC(s, i, 1) * q.si01;
    k1[i] = CC(s, i, 0) * q.si01 + CC(s, i, 1) * q.si11;
    hc0[i] = CC(s, 0, i);
    hc1[i] = CC(s, 1, i);
  }
  for (int i = 0; i < 5; i++) s->p[i] = s->p[i] + (k0[i] * r0 + k1[i] * r1);
  for (int i = 0; i < 5; i++)
    for (int j = 0; j <= i; j++)
      s->c[ci(i, j)] = s->c[ci(i, j)] - (k0[i] * hc0[j] + k1[i] * hc1[j]);
  return chi2;
}

static void k_init_cov(kst* s, real vy, real vz)
{
  for (int k = 0; k < 15; k++) s->c[k] = 0;
  s->c[0] = vy;
  s->c[2] = vz;
  s->c[5] = 1;
  s->c[9] = 1;
  s->c[14] = 100;
}

#endif
