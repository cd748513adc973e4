/*
 * Oracle of the differentiable Kalman refit -- TEST INFRASTRUCTURE ONLY.
 *
 * Readings R21-R27 (design notes): each found track (hits in ascending row
 * order) is refitted with the Kalman filter of R7-R9, the measurement planes
 * being X_k = x_k + D[row_k][sector_k mod 18]; the filter starts at the first
 * hit from its (y, z) and a constant seed (snp, tgl, qpt) with
 * C0 = diag(sy2, sz2, 1, 1, 100).  A propagation failure makes the track
 * contribute zero (status 1).  The state after every update is checkpointed
 * (5 parameters + 15 covariance terms).
 *
 * Compiled three times (see oracle/__init__.py): binary32 (forward, the
 * bit-exact reference of the GPU forward), binary64 (forward and the
 * hand-written reverse pass orc_refit_grad_f64) and complex binary64
 * (orc_refit_loss_c128: complex-step derivatives of the very same forward
 * code, an independent check of the reverse pass).
 */
#include "tpc_oracle.h"

#include <stdlib.h>

#include "kalman.h"

#define NPHI 18

#if defined(ORC_C128)
#define PERT(h) ((h) * I)
#else
#define PERT(h) (h)
#endif

static real kB_val(const orc_geom* g) { return (real)(-0.299792458e-2 * (double)g->bz); }

/* R42: the field of the step into cluster c -- the map's value at c's row
 * and the z bin of c's measured z (bins of 500 cm / nzb from -250 cm,
 * clamped), converted like the geometry's field; piecewise constant, so it
 * carries no derivative */
static int zbin(float z, int nzb)
{
  const double f = floor(((double)z + 250.0) * (double)nzb / 500.0);
  if (!(f >= 0)) return 0;
  if (f > nzb - 1) return nzb - 1;
  return (int)f;
}

static double step_B(const orc_geom* g, const orc_material* M, int64_t c, const float* z,
                     const uint16_t* row)
{
  if (!M || !M->bz) return (double)g->bz;
  return (double)M->bz[(int64_t)row[c] * M->nzb + zbin(z[c], M->nzb)];
}

/* R43, R44: material of the step (after the propagation, on its result):
 * multiple-scattering noise on snp, tgl, q/pt from the Highland width
 * without its logarithm, theta^2 = 0.0136^2 t / (beta p)^2 with t the
 * traversed thickness in radiation lengths; then the mean energy loss
 * dE/dx = K / beta^2 changes q/pt by the factor f = 1 + E dE / p^2 (sign
 * of the step: outward steps lose energy), and the covariance row of q/pt
 * by the same factor.  Pion mass hypothesis. */
#define K_MS 1.8496e-4      /* 0.0136^2 [GeV^2] */
#define M_PION2 0.019479785 /* 0.13957^2 [GeV^2] */

static void mat_apply(kst* s, real ads, real sgn, real ix0, real K)
{
  const real one = 1;
  const real snp = s->p[2], tgl = s->p[3], qpt = s->p[4];
  const real t2 = one + tgl * tgl;
  const real w = (qpt * qpt) / t2;
  const real bg = one + (real)M_PION2 * w;
  const real path = ads * SQRT(t2);
  if (RE(ix0) > 0) {
    const real th2 = ((real)K_MS * (path * ix0)) * (w * bg);
    const real qt = qpt * tgl;
    s->c[5] = s->c[5] + th2 * (((one - snp) * (one + snp)) * t2);
    s->c[9] = s->c[9] + th2 * (t2 * t2);
    s->c[13] = s->c[13] + th2 * (t2 * qt);
    s->c[14] = s->c[14] + th2 * (qt * qt);
  }
  if (RE(K) > 0) {
    const real corr = (SQRT(w * bg) * (K * bg)) * (path * sgn);
    const real f = one + corr;
    s->p[4] = qpt * f;
    for (int j = 0; j < 4; j++) s->c[ci(4, j)] = s->c[ci(4, j)] * f;
    s->c[14] = (s->c[14] * f) * f;
  }
}

/* R21: measurement plane of cluster c (optionally perturbed) */
static real plane_x(const float* x, const uint16_t* row, const uint8_t* sector, const float* dmap,
                    int64_t c)
{
  return (real)x[c] + (real)dmap[(int64_t)row[c] * NPHI + sector[c] % NPHI];
}

/* R22-R24: refit of one track; returns 0 on a propagation failure.
 * pert_* adds a perturbation to one input (finite / complex-step checks):
 * which = 0 x[idx], 1 y[idx], 2 z[idx], 3 map cell idx, -1 none. */
static int refit_one(const orc_geom* g, const orc_params* P, const orc_material* M, int64_t a,
                     int64_t b, const int32_t* hit_clu, const uint8_t* sector, const float* x,
                     const float* y, const float* z, const uint16_t* row, const float* seed5,
                     const float* dmap, real* chi2_out, real* ckpt, int which, int64_t idx,
                     real pert)
{
  const real kB0 = kB_val(g);
  const real vy = (real)g->sigma_y2, vz = (real)g->sigma_z2;
  const real smax = (real)P->snp_max;
#define XK(c) (plane_x(x, row, sector, dmap, (c)) + \
               ((which == 0 && (c) == idx) || \
                (which == 3 && (int64_t)row[(c)] * NPHI + sector[(c)] % NPHI == idx) ? pert : (real)0))
#define YK(c) ((real)y[(c)] + ((which == 1 && (c) == idx) ? pert : (real)0))
#define ZK(c) ((real)z[(c)] + ((which == 2 && (c) == idx) ? pert : (real)0))
  const int64_t c0 = hit_clu[a];
  kst st;
  st.p[0] = YK(c0);
  st.p[1] = ZK(c0);
  st.p[2] = (real)seed5[2];
  st.p[3] = (real)seed5[3];
  st.p[4] = (real)seed5[4];
  k_init_cov(&st, vy, vz);
  if (ckpt) {
    for (int j = 0; j < 5; j++) ckpt[a * 20 + j] = st.p[j];
    for (int j = 0; j < 15; j++) ckpt[a * 20 + 5 + j] = st.c[j];
  }
  real chi2 = 0;
  real xprev = XK(c0);
  for (int64_t k = a + 1; k < b; k++) {
    const int64_t c = hit_clu[k];
    const real xk = XK(c);
    const real kB = (M && M->bz) ? (real)(-0.299792458e-2 * step_B(g, M, c, z, row)) : kB0;
    real ds;
    if (!k_propagate_ds(&st, xprev, xk, kB, smax, &ds)) {
      *chi2_out = 0;
      return 0;
    }
    if (M && (M->ix0 || M->eloss)) {
      const real sgn = RE(xk) - RE(xprev) < 0 ? (real)-1 : (real)1;
      mat_apply(&st, ds * sgn, sgn, M->ix0 ? (real)M->ix0[row[c]] : (real)0,
                M->eloss ? (real)M->eloss[row[c]] : (real)0);
    }
    chi2 += k_update(&st, YK(c), ZK(c), vy, vz);
    if (ckpt) {
      for (int j = 0; j < 5; j++) ckpt[k * 20 + j] = st.p[j];
      for (int j = 0; j < 15; j++) ckpt[k * 20 + 5 + j] = st.c[j];
    }
    xprev = xk;
  }
#undef XK
#undef YK
#undef ZK
  *chi2_out = chi2;
  return 1;
}

/* A track is refitted only if every hit names a cluster in [0, n_clusters)
 * on one of the map's rows (the plane offset D[row][.] exists); otherwise it
 * is rejected as a whole: status 2, chi2 0, no checkpoints, zero gradient. */
static int hits_valid(const orc_geom* g, int64_t a, int64_t b, const int32_t* hit_clu,
                      const uint16_t* row, int64_t n_clusters)
{
  for (int64_t k = a; k < b; k++) {
    const int64_t c = hit_clu[k];
    if (c < 0 || c >= n_clusters || row[c] >= g->n_rows) return 0;
  }
  return 1;
}

/* a8 -- forward refit of n_tracks tracks (CSR hit lists, cluster indices). */
void SFX(orc_refit)(const orc_geom* g, const orc_params* P, const orc_material* M,
                    int64_t n_tracks, const int32_t* hit_off, const int32_t* hit_clu,
                    const uint8_t* sector, const float* x, const float* y, const float* z,
                    const uint16_t* row, int64_t n_clusters, const float* seed, const float* dmap,
                    real* chi2, int32_t* status, real* ckpt)
{
  for (int64_t t = 0; t < n_tracks; t++) {
    const int64_t a = hit_off[t], b = hit_off[t + 1];
    if (b <= a) {
      chi2[t] = 0;
      status[t] = 0;
      continue;
    }
    if (!hits_valid(g, a, b, hit_clu, row, n_clusters)) {
      chi2[t] = 0;
      status[t] = 2;
      continue;
    }
    status[t] = refit_one(g, P, M, a, b, hit_clu, sector, x, y, z, row, seed + 5 * t, dmap, &chi2[t],
                          ckpt, -1, -1, (real)0)
                    ? 0
                    : 1;
  }
}

/* Sum_t w_t chi2_t with one input perturbed by h (binary builds: f(x + h);
 * complex build: Im f(x + i h) / h, the complex-step derivative). */
double SFX(orc_refit_loss)(const orc_geom* g, const orc_params* P, const orc_material* M,
                           int64_t n_tracks,
                           const int32_t* hit_off, const int32_t* hit_clu, const uint8_t* sector,
                           const float* x, const float* y, const float* z, const uint16_t* row,
                           int64_t n_clusters, const float* seed, const float* dmap,
                           const double* w, int which, int64_t idx, double h)
{
  real tot = 0;
  for (int64_t t = 0; t < n_tracks; t++) {
    const int64_t a = hit_off[t], b = hit_off[t + 1];
    if (b <= a || !hits_valid(g, a, b, hit_clu, row, n_clusters)) continue;
    real c2 = 0;
    if (refit_one(g, P, M, a, b, hit_clu, sector, x, y, z, row, seed + 5 * t, dmap, &c2, NULL, which,
                  idx, (real)PERT(h)))
      tot += (real)w[t] * c2;
  }
#if defined(ORC_C128)
  return cimag(tot) / h;
#else
  return (double)tot;
#endif
}

#if defined(ORC_F64)
/* ---------------------------------------------------------------------------
 * a9 -- reverse pass (R25, R26), binary64.  Every step k (hits k-1 -> k) is
 * rebuilt from checkpoint k-1: propagation intermediates (R7/R8), predicted
 * state, update intermediates (R9); then adjoints flow backwards through the
 * update and the propagation.  Covariance adjoints are kept as full
 * symmetric 5x5 matrices X with dL = <X, dC> for symmetric dC.
 */
typedef struct {
  double dx, cc, s2, c1, c2, f, dy, L, lc, u2, g, sg, ds, h, ic1, ic2, dfs, dfq, dg, dyl, hlc, Lg;
  double a, dLs, du2s, T1, d, b, dLq, du2q, T2, gq, e, hq;
} prec;

static void prop_record(const double* p, double dx, double kB, prec* q)
{
  const double snp = p[2], tgl = p[3], qpt = p[4];
  q->dx = dx;
  q->cc = kB * qpt;
  q->s2 = snp + q->cc * dx;
  q->c1 = sqrt((1 - snp) * (1 + snp));
  q->c2 = sqrt((1 - q->s2) * (1 + q->s2));
  q->f = (snp + q->s2) / (q->c1 + q->c2);
  q->dy = dx * q->f;
  q->L = sqrt(dx * dx + q->dy * q->dy);
  q->lc = q->L * q->cc;
  q->u2 = (q->lc * q->lc) * 0.25;
  q->g = 1 + q->u2 * (1.0 / 6.0 + q->u2 * (3.0 / 40.0));
  q->sg = dx < 0 ? -1.0 : 1.0;
  q->ds = (q->sg * q->L) * q->g;
  q->h = (1 + q->f * q->f) * 0.5;
  q->ic1 = 1 / q->c1;
  q->ic2 = 1 / q->c2;
  q->dfs = q->h * (q->ic1 + q->ic2);
  q->dfq = (q->h * (dx * q->ic2)) * kB;
  q->dg = 1.0 / 6.0 + q->u2 * (3.0 / 20.0);
  q->dyl = q->dy / q->L;
  q->hlc = 0.5 * q->lc;
  q->Lg = q->L * q->dg;
  q->a = dx * q->dfs;
  q->dLs = q->dyl * q->a;
  q->du2s = q->hlc * (q->dLs * q->cc);
  q->T1 = q->dLs * q->g + q->Lg * q->du2s;
  q->d = tgl * (q->sg * q->T1);
  q->b = dx * q->dfq;
  q->dLq = q->dyl * q->b;
  q->du2q = q->hlc * (q->dLq * q->cc + q->L * kB);
  q->T2 = q->dLq * q->g + q->Lg * q->du2q;
  q->gq = tgl * (q->sg * q->T2);
  q->e = q->ds;
  q->hq = kB * dx;
}

static void unpack(const double* c15, double C[5][5])
{
  for (int i = 0; i < 5; i++)
    for (int j = 0; j <= i; j++) C[i][j] = C[j][i] = c15[i * (i + 1) / 2 + j];
}

static void fmat(const prec* q, double F[5][5])
{
  memset(F, 0, sizeof(double) * 25);
  for (int i = 0; i < 5; i++) F[i][i] = 1;
  F[0][2] = q->a;
  F[0][4] = q->b;
  F[1][2] = q->d;
  F[1][3] = q->e;
  F[1][4] = q->gq;
  F[2][4] = q->hq;
}

static void mm(double A[5][5], double B[5][5], double R[5][5])
{
  double T[5][5];
  for (int i = 0; i < 5; i++)
    for (int j = 0; j < 5; j++) {
      double s = 0;
      for (int k = 0; k < 5; k++) s += A[i][k] * B[k][j];
      T[i][j] = s;
    }
  memcpy(R, T, sizeof(T));
}

static void mtm(double A[5][5], double B[5][5], double R[5][5]) /* R = A^T B */
{
  double T[5][5];
  for (int i = 0; i < 5; i++)
    for (int j = 0; j < 5; j++) {
      double s = 0;
      for (int k = 0; k < 5; k++) s += A[k][i] * B[k][j];
      T[i][j] = s;
    }
  memcpy(R, T, sizeof(T));
}

/* adjoint of the propagation's scalar chain: pb (in: adjoint of the
 * propagated state, out: adjoint of the state before), Fb = adjoints of the
 * six Jacobian entries; returns the adjoint of dx */
static double prop_backward(const double* p, const prec* q, double kB, double* pb, const double Fb[6],
                            double dsb_extra)
{
  const double tgl = p[3], snp = p[2];
  double yb = pb[0], zb = pb[1], s2b = pb[2], tglb = pb[3], qptb = pb[4];
  double dyb = yb, dsb = zb * tgl + dsb_extra;
  tglb += zb * q->ds;
  double ab = Fb[0], bb = Fb[1], db = Fb[2], eb = Fb[3], gqb = Fb[4], hqb = Fb[5];
  double dxb = 0, ccb = 0, Lb = 0, gb = 0, Lgb = 0, hlcb = 0, lcb = 0, u2b = 0, dylb = 0, hb = 0;
  double ic1b = 0, ic2b = 0, c1b = 0, c2b = 0, fb = 0, snpb = 0, dfsb = 0, dfqb = 0, dgb = 0;
  double dLsb = 0, du2sb = 0, dLqb = 0, du2qb = 0;
  dxb += hqb * kB;                               /* hq = kB*dx */
  dsb += eb;                                     /* e = ds */
  tglb += gqb * q->sg * q->T2;                   /* gq = tgl*sg*T2 */
  double T2b = gqb * tgl * q->sg;
  dLqb += T2b * q->g;                            /* T2 = dLq*g + Lg*du2q */
  gb += T2b * q->dLq;
  Lgb += T2b * q->du2q;
  du2qb += T2b * q->Lg;
  hlcb += du2qb * (q->dLq * q->cc + q->L * kB);  /* du2q = hlc*(dLq*cc + L*kB) */
  dLqb += du2qb * q->hlc * q->cc;
  ccb += du2qb * q->hlc * q->dLq;
  Lb += du2qb * q->hlc * kB;
  dylb += dLqb * q->b;                           /* dLq = dyl*b */
  bb += dLqb * q->dyl;
  dxb += bb * q->dfq;                            /* b = dx*dfq */
  dfqb += bb * q->dx;
  tglb += db * q->sg * q->T1;                    /* d = tgl*sg*T1 */
  double T1b = db * tgl * q->sg;
  dLsb += T1b * q->g;                            /* T1 = dLs*g + Lg*du2s */
  gb += T1b * q->dLs;
  Lgb += T1b * q->du2s;
  du2sb += T1b * q->Lg;
  hlcb += du2sb * q->dLs * q->cc;                /* du2s = hlc*(dLs*cc) */
  dLsb += du2sb * q->hlc * q->cc;
  ccb += du2sb * q->hlc * q->dLs;
  dylb += dLsb * q->a;                           /* dLs = dyl*a */
  ab += dLsb * q->dyl;
  dxb += ab * q->dfs;                            /* a = dx*dfs */
  dfsb += ab * q->dx;
  Lb += Lgb * q->dg;                             /* Lg = L*dg */
  dgb += Lgb * q->L;
  lcb += 0.5 * hlcb;                             /* hlc = 0.5*lc */
  dyb += dylb / q->L;                            /* dyl = dy/L */
  Lb -= dylb * q->dy / (q->L * q->L);
  u2b += dgb * (3.0 / 20.0);                     /* dg = 1/6 + u2*3/20 */
  hb += dfqb * q->dx * q->ic2 * kB;              /* dfq = h*dx*ic2*kB */
  dxb += dfqb * q->h * q->ic2 * kB;
  ic2b += dfqb * q->h * q->dx * kB;
  hb += dfsb * (q->ic1 + q->ic2);                /* dfs = h*(ic1+ic2) */
  ic1b += dfsb * q->h;
  ic2b += dfsb * q->h;
  c1b -= ic1b / (q->c1 * q->c1);                 /* ic1 = 1/c1 */
  c2b -= ic2b / (q->c2 * q->c2);
  fb += hb * q->f;                               /* h = (1+f^2)/2 */
  Lb += dsb * q->sg * q->g;                      /* ds = sg*L*g */
  gb += dsb * q->sg * q->L;
  u2b += gb * (1.0 / 6.0 + 2 * q->u2 * (3.0 / 40.0)); /* g = 1 + u2/6 + 3u2^2/40 */
  lcb += u2b * 0.5 * q->lc;                      /* u2 = lc^2/4 */
  Lb += lcb * q->cc;                             /* lc = L*cc */
  ccb += lcb * q->L;
  dxb += Lb * q->dx / q->L;                      /* L = sqrt(dx^2+dy^2) */
  dyb += Lb * q->dy / q->L;
  dxb += dyb * q->f;                             /* dy = dx*f */
  fb += dyb * q->dx;
  const double den = q->c1 + q->c2;              /* f = (snp+s2)/(c1+c2) */
  const double numb = fb / den, denb = -fb * q->f / den;
  snpb += numb;
  s2b += numb;
  c1b += denb;
  c2b += denb;
  s2b += c2b * (-q->s2 / q->c2);                 /* c2 = sqrt(1-s2^2) */
  snpb += c1b * (-snp / q->c1);                  /* c1 = sqrt(1-snp^2) */
  snpb += s2b;                                   /* s2 = snp + cc*dx */
  ccb += s2b * q->dx;
  dxb += s2b * q->cc;
  qptb += ccb * kB;                              /* cc = kB*qpt */
  pb[0] = yb;
  pb[1] = zb;
  pb[2] = snpb;
  pb[3] = tglb;
  pb[4] = qptb;
  return dxb;
}

/* adjoint of the R9 update; C is the predicted covariance, p the predicted
 * state; pb, Xb in/out (adjoints of the updated state), chib the weight of
 * this chi2; writes mb (adjoint of the measurement) */
static void update_backward(const double* p, double C[5][5], double my, double mz, double vy,
                            double vz, double chib, double* pb, double Xb[5][5], double* mb)
{
  const double S00 = C[0][0] + vy, S01 = C[0][1], S11 = C[1][1] + vz;
  const double det = S00 * S11 - S01 * S01;
  const double Si[2][2] = {{S11 / det, -S01 / det}, {-S01 / det, S00 / det}};
  const double r[2] = {my - p[0], mz - p[1]};
  double U[5][2], K[5][2];
  for (int i = 0; i < 5; i++) {
    U[i][0] = C[i][0];
    U[i][1] = C[i][1];
    for (int a = 0; a < 2; a++) K[i][a] = U[i][0] * Si[0][a] + U[i][1] * Si[1][a];
  }
  const double w[2] = {Si[0][0] * r[0] + Si[0][1] * r[1], Si[1][0] * r[0] + Si[1][1] * r[1]};
  double Ub[5][2] = {{0}}, Sib[2][2] = {{0}}, rb[2] = {0, 0};
  /* C_out = C - U Si U^T */
  for (int i = 0; i < 5; i++)
    for (int a = 0; a < 2; a++) {
      double s = 0;
      for (int j = 0; j < 5; j++) s += Xb[i][j] * K[j][a];
      Ub[i][a] += -2 * s;
    }
  for (int a = 0; a < 2; a++)
    for (int bq = 0; bq < 2; bq++) {
      double s = 0;
      for (int i = 0; i < 5; i++)
        for (int j = 0; j < 5; j++) s += U[i][a] * Xb[i][j] * U[j][bq];
      Sib[a][bq] -= s;
    }
  /* p_out = p + U Si r */
  double Utp[2] = {0, 0};
  for (int i = 0; i < 5; i++)
    for (int a = 0; a < 2; a++) {
      Ub[i][a] += pb[i] * w[a];
      Utp[a] += U[i][a] * pb[i];
      rb[a] += K[i][a] * pb[i];
    }
  for (int a = 0; a < 2; a++)
    for (int bq = 0; bq < 2; bq++) Sib[a][bq] += Utp[a] * r[bq];
  /* chi2 = r^T Si r */
  for (int a = 0; a < 2; a++) {
    rb[a] += 2 * chib * w[a];
    for (int bq = 0; bq < 2; bq++) Sib[a][bq] += chib * r[a] * r[bq];
  }
  /* Si = S^-1 */
  double T[2][2], Smb[2][2];
  for (int a = 0; a < 2; a++)
    for (int bq = 0; bq < 2; bq++) T[a][bq] = Si[a][0] * Sib[0][bq] + Si[a][1] * Sib[1][bq];
  for (int a = 0; a < 2; a++)
    for (int bq = 0; bq < 2; bq++) Smb[a][bq] = -(T[a][0] * Si[0][bq] + T[a][1] * Si[1][bq]);
  Xb[0][0] += Smb[0][0];
  Xb[1][1] += Smb[1][1];
  const double s01 = 0.5 * (Smb[0][1] + Smb[1][0]);
  Xb[0][1] += s01;
  Xb[1][0] += s01;
  /* U = C[:, 0:2] (symmetrised) */
  for (int i = 0; i < 5; i++)
    for (int a = 0; a < 2; a++) {
      Xb[i][a] += 0.5 * Ub[i][a];
      Xb[a][i] += 0.5 * Ub[i][a];
    }
  /* r = m - H p */
  mb[0] = rb[0];
  mb[1] = rb[1];
  pb[0] -= rb[0];
  pb[1] -= rb[1];
}

/* the material step of mat_apply in binary64 with its intermediates, and
 * its adjoint: (pp, C) is the propagated state and covariance on input, the
 * state and covariance after the material on output */
typedef struct {
  double t2, w, bg, sq, path, th2, qt, corr, f, ads, sgn, ix0, K;
  double C2[5][5];  /* covariance after the scattering noise, before the loss */
  double q4;        /* q/pt before the loss */
} mrec;

static void mat_forward(double* pp, double C[5][5], double ads, double sgn, double ix0, double K,
                        mrec* m)
{
  const double snp = pp[2], tgl = pp[3], qpt = pp[4];
  m->ads = ads;
  m->sgn = sgn;
  m->ix0 = ix0;
  m->K = K;
  m->t2 = 1 + tgl * tgl;
  m->w = (qpt * qpt) / m->t2;
  m->bg = 1 + M_PION2 * m->w;
  m->path = ads * sqrt(m->t2);
  m->qt = qpt * tgl;
  m->th2 = ix0 > 0 ? (K_MS * (m->path * ix0)) * (m->w * m->bg) : 0;
  if (ix0 > 0) {
    C[2][2] += m->th2 * (((1 - snp) * (1 + snp)) * m->t2);
    C[3][3] += m->th2 * (m->t2 * m->t2);
    C[4][3] += m->th2 * (m->t2 * m->qt);
    C[3][4] = C[4][3];
    C[4][4] += m->th2 * (m->qt * m->qt);
  }
  memcpy(m->C2, C, sizeof(m->C2));
  m->q4 = qpt;
  m->sq = sqrt(m->w * m->bg);
  m->corr = K > 0 ? (m->sq * (K * m->bg)) * (m->path * sgn) : 0;
  m->f = 1 + m->corr;
  if (K > 0) {
    pp[4] = qpt * m->f;
    for (int j = 0; j < 4; j++) {
      C[4][j] *= m->f;
      C[j][4] = C[4][j];
    }
    C[4][4] = (C[4][4] * m->f) * m->f;
  }
}

/* adjoint of mat_forward: pb, Xb in (adjoints after the material), out
 * (adjoints of the propagated state and covariance); pp1 the propagated
 * state; returns the adjoint of the step's signed arc length ds */
static double mat_backward(const double* pp1, const mrec* m, double* pb, double Xb[5][5])
{
  const double snp = pp1[2], tgl = pp1[3], qpt = pp1[4];
  double t2b = 0, wb = 0, bgb = 0, pathb = 0, qtb = 0;
  if (m->K > 0) {
    /* C = S C2 S with S = diag(1, 1, 1, 1, f); q/pt' = q/pt f */
    double cb = pb[4] * m->q4;
    double s = 0;
    for (int j = 0; j < 4; j++) s += Xb[4][j] * m->C2[4][j];
    cb += 2 * (s + Xb[4][4] * m->C2[4][4] * m->f);
    pb[4] = pb[4] * m->f;
    for (int j = 0; j < 4; j++) {
      Xb[4][j] *= m->f;
      Xb[j][4] = Xb[4][j];
    }
    Xb[4][4] = Xb[4][4] * m->f * m->f;
    /* corr = sq * (K bg) * (path sgn), sq = sqrt(w bg) */
    const double sqb = cb * (m->K * m->bg) * (m->path * m->sgn);
    bgb += cb * m->sq * m->K * (m->path * m->sgn);
    pathb += cb * m->sq * (m->K * m->bg) * m->sgn;
    if (m->sq > 0) {
      const double wbgb = sqb / (2 * m->sq);
      wb += wbgb * m->bg;
      bgb += wbgb * m->w;
    }
  }
  if (m->ix0 > 0) {
    /* <X, Q>: Q22, Q33, Q43 (= Q34), Q44 */
    const double u22 = ((1 - snp) * (1 + snp)) * m->t2, u33 = m->t2 * m->t2;
    const double u43 = m->t2 * m->qt, u44 = m->qt * m->qt;
    const double A = Xb[2][2] * u22 + Xb[3][3] * u33 + 2 * Xb[4][3] * u43 + Xb[4][4] * u44;
    const double th2 = m->th2;
    pb[2] += th2 * Xb[2][2] * (-2 * snp) * m->t2;
    t2b += th2 * (Xb[2][2] * ((1 - snp) * (1 + snp)) + Xb[3][3] * 2 * m->t2 + 2 * Xb[4][3] * m->qt);
    qtb += th2 * (2 * Xb[4][3] * m->t2 + Xb[4][4] * 2 * m->qt);
    /* th2 = K_MS path ix0 w bg */
    pathb += A * K_MS * m->ix0 * m->w * m->bg;
    wb += A * K_MS * m->path * m->ix0 * m->bg;
    bgb += A * K_MS * m->path * m->ix0 * m->w;
  }
  /* qt = qpt tgl; bg = 1 + m2 w; w = qpt^2 / t2; path = ads sqrt(t2); t2 = 1 + tgl^2 */
  pb[4] += qtb * tgl;
  pb[3] += qtb * qpt;
  wb += bgb * M_PION2;
  pb[4] += wb * 2 * qpt / m->t2;
  t2b += wb * (-m->w / m->t2);
  const double st2 = sqrt(m->t2);
  const double adsb = pathb * st2;
  t2b += pathb * m->ads / (2 * st2);
  pb[3] += t2b * 2 * tgl;
  return adsb * m->sgn;  /* ads = sgn ds */
}

/* gradient of sum_t w[t] chi2_t w.r.t. the map (gmap[152*18]) and the
 * cluster coordinates (gx, gy, gz[n_clusters]); all outputs overwritten */
void orc_refit_grad_f64(const orc_geom* g, const orc_params* P, const orc_material* M,
                        int64_t n_tracks,
                        const int32_t* hit_off, const int32_t* hit_clu, const uint8_t* sector,
                        const float* x, const float* y, const float* z, const uint16_t* row,
                        const float* seed, const float* dmap, const double* ckpt,
                        const int32_t* status, const double* w, int64_t n_clusters, double* gmap,
                        double* gx, double* gy, double* gz)
{
  const double vy = g->sigma_y2, vz = g->sigma_z2;
  const int mat = M && (M->ix0 || M->eloss);
  for (int64_t i = 0; i < (int64_t)g->n_rows * NPHI; i++) gmap[i] = 0;
  for (int64_t c = 0; c < n_clusters; c++) gx[c] = gy[c] = gz[c] = 0;
  for (int64_t t = 0; t < n_tracks; t++) {
    const int64_t a = hit_off[t], b = hit_off[t + 1];
    if (b - a < 1 || status[t] != 0 || !hits_valid(g, a, b, hit_clu, row, n_clusters)) continue;
    double pb[5] = {0, 0, 0, 0, 0};
    double Xb[5][5] = {{0}};
    double gX_next = 0; /* adjoint of X_k from step k+1 */
    for (int64_t k = b - 1; k >= a + 1; k--) {
      const int64_t c = hit_clu[k], cp = hit_clu[k - 1];
      const double X2 = (double)x[c] + (double)dmap[(int64_t)row[c] * NPHI + sector[c] % NPHI];
      const double X1 = (double)x[cp] + (double)dmap[(int64_t)row[cp] * NPHI + sector[cp] % NPHI];
      const double* ck = ckpt + (k - 1) * 20;
      double p0[5], C0[5][5];
      for (int j = 0; j < 5; j++) p0[j] = ck[j];
      unpack(ck + 5, C0);
      /* the step's field (R42), in binary64 like the binary64 forward */
      const double kB = -0.299792458e-2 * step_B(g, M, c, z, row);
      prec q;
      prop_record(p0, X2 - X1, kB, &q);
      double F[5][5], Cp[5][5], pp[5];
      fmat(&q, F);
      mm(F, C0, Cp);
      double Ft[5][5];
      for (int i = 0; i < 5; i++)
        for (int j = 0; j < 5; j++) Ft[i][j] = F[j][i];
      mm(Cp, Ft, Cp);
      pp[0] = p0[0] + q.dy;
      pp[1] = p0[1] + p0[3] * q.ds;
      pp[2] = q.s2;
      pp[3] = p0[3];
      pp[4] = p0[4];
      double pp1[5];
      memcpy(pp1, pp, sizeof(pp1));
      mrec mr;
      memset(&mr, 0, sizeof(mr));
      if (mat)
        mat_forward(pp, Cp, q.ds * q.sg, q.sg, M->ix0 ? (double)M->ix0[row[c]] : 0,
                    M->eloss ? (double)M->eloss[row[c]] : 0, &mr);
      double mb[2];
      update_backward(pp, Cp, (double)y[c], (double)z[c], vy, vz, w[t], pb, Xb, mb);
      const double dsb_mat = mat ? mat_backward(pp1, &mr, pb, Xb) : 0;
      /* propagation: covariance part */
      double XF[5][5], XFC[5][5], Xn[5][5];
      mm(Xb, F, XF);
      mm(XF, C0, XFC);
      mtm(F, XF, Xn);
      const double Fb[6] = {2 * XFC[0][2], 2 * XFC[0][4], 2 * XFC[1][2],
                            2 * XFC[1][3], 2 * XFC[1][4], 2 * XFC[2][4]};
      memcpy(Xb, Xn, sizeof(Xn));
      const double dxb = prop_backward(p0, &q, kB, pb, Fb, dsb_mat);
      const double gXk = dxb + gX_next;
      gx[c] = gXk;
      gy[c] = mb[0];
      gz[c] = mb[1];
      gmap[(int64_t)row[c] * NPHI + sector[c] % NPHI] += gXk;
      gX_next = -dxb;
    }
    const int64_t c0 = hit_clu[a];
    gx[c0] = gX_next;
    gy[c0] = pb[0];
    gz[c0] = pb[1];
    gmap[(int64_t)row[c0] * NPHI + sector[c0] % NPHI] += gX_next;
  }
}
#endif
