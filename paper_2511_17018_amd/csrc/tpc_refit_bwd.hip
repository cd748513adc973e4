// Reverse pass of the Kalman refit (a9), gfx950, binary64 arithmetic on the
// binary32 forward's checkpoints (CDNA4 runs FP64 vector at half the FP32
// rate and the pass is memory-bound, so the wider type costs little and
// removes the binary32 cancellation in residuals near zero).
//
// One lane per track walks its hits backwards.  Step k (hits k-1 -> k) is
// rebuilt from checkpoint k-1: the propagation intermediates of R7/R8, the
// predicted state and covariance, the update quantities of R9; then the
// adjoints flow through the update and the propagation (reverse-mode
// differentiation of the formulas as written, including the Jacobian's and
// the gain's dependence on the state).  Covariance adjoints are full
// symmetric 5x5 matrices X with dL = <X, dC> for symmetric dC.
//
// Outputs: d(sum_t w_t chi2_t)/d(cluster x, y, z) (each cluster is on at most
// one track, so plain stores) and d/d(map cell).  The map sums use 64-bit
// fixed-point atomics (scale 2^24): integer addition is associative, so the
// result does not depend on the order in which lanes add, and no float
// atomics are used.
//
// The gradient is compared with the binary64 reference within a tolerance,
// not bit for bit, so this file is built once, with fast math (no contraction
// constraints).
#include <mutex>

#include "tpc_internal.h"
#include "tpc_ckpt.h"

namespace tpcca {
namespace bwd {
namespace {

constexpr double kFix = 16777216.0;  // 2^24
constexpr double kFixMax = 4.0e18;   // |value * 2^24| clamp (overflow flag)

using R = double;  // arithmetic type of the reverse pass

struct PRec {
  R dx, cc, s2, c1, c2, f, dy, L, lc, u2, g, sg, ds, h, ic1, ic2, dfs, dfq, dg, dyl, hlc, Lg;
  R a, dLs, du2s, T1, d, b, dLq, du2q, T2, gq, e, hq;
};

__device__ __forceinline__ void prop_record(const R* p, R dx, R kB, PRec& q)
{
  const R snp = p[2], tgl = p[3], qpt = p[4];
  q.dx = dx;
  q.cc = kB * qpt;
  q.s2 = snp + q.cc * dx;
  q.c1 = sqrt((1.0 - snp) * (1.0 + snp));
  q.c2 = sqrt((1.0 - q.s2) * (1.0 + q.s2));
  q.f = (snp + q.s2) / (q.c1 + q.c2);
  q.dy = dx * q.f;
  q.L = sqrt(dx * dx + q.dy * q.dy);
  q.lc = q.L * q.cc;
  q.u2 = (q.lc * q.lc) * 0.25;
  q.g = 1.0 + q.u2 * (1.0 / 6.0 + q.u2 * (3.0 / 40.0));
  q.sg = dx < 0.0 ? -1.0 : 1.0;
  q.ds = (q.sg * q.L) * q.g;
  q.h = (1.0 + q.f * q.f) * 0.5;
  q.ic1 = 1.0 / q.c1;
  q.ic2 = 1.0 / q.c2;
  q.dfs = q.h * (q.ic1 + q.ic2);
  q.dfq = (q.h * (dx * q.ic2)) * kB;
  q.dg = 1.0 / 6.0 + q.u2 * (3.0 / 20.0);
  q.dyl = q.dy / q.L;
  q.hlc = 0.5 * q.lc;
  q.Lg = q.L * q.dg;
  q.a = dx * q.dfs;
  q.dLs = q.dyl * q.a;
  q.du2s = q.hlc * (q.dLs * q.cc);
  q.T1 = q.dLs * q.g + q.Lg * q.du2s;
  q.d = tgl * (q.sg * q.T1);
  q.b = dx * q.dfq;
  q.dLq = q.dyl * q.b;
  q.du2q = q.hlc * (q.dLq * q.cc + q.L * kB);
  q.T2 = q.dLq * q.g + q.Lg * q.du2q;
  q.gq = tgl * (q.sg * q.T2);
  q.e = q.ds;
  q.hq = kB * dx;
}

// adjoint of the propagation's scalar chain; pb in/out, Fb = adjoints of
// (a, b, d, e, gq, hq); returns the adjoint of dx
__device__ __forceinline__ R prop_backward(const R* p, const PRec& q, R kB, R* pb,
                                               const R* Fb, R dsb_extra = 0.0)
{
  const R tgl = p[3], snp = p[2];
  const R yb = pb[0], zb = pb[1];
  R s2b = pb[2], tglb = pb[3], qptb = pb[4];
  R dyb = yb, dsb = zb * tgl + dsb_extra;
  tglb += zb * q.ds;
  R ab = Fb[0], bb = Fb[1];
  const R db = Fb[2], eb = Fb[3], gqb = Fb[4], hqb = Fb[5];
  R dxb = hqb * kB;
  dsb += eb;
  tglb += gqb * q.sg * q.T2;
  const R T2b = gqb * tgl * q.sg;
  R dLqb = T2b * q.g;
  R gb = T2b * q.dLq;
  R Lgb = T2b * q.du2q;
  const R du2qb = T2b * q.Lg;
  R hlcb = du2qb * (q.dLq * q.cc + q.L * kB);
  dLqb += du2qb * q.hlc * q.cc;
  R ccb = du2qb * q.hlc * q.dLq;
  R Lb = du2qb * q.hlc * kB;
  R dylb = dLqb * q.b;
  bb += dLqb * q.dyl;
  dxb += bb * q.dfq;
  const R dfqb = bb * q.dx;
  tglb += db * q.sg * q.T1;
  const R T1b = db * tgl * q.sg;
  R dLsb = T1b * q.g;
  gb += T1b * q.dLs;
  Lgb += T1b * q.du2s;
  const R du2sb = T1b * q.Lg;
  hlcb += du2sb * q.dLs * q.cc;
  dLsb += du2sb * q.hlc * q.cc;
  ccb += du2sb * q.hlc * q.dLs;
  dylb += dLsb * q.a;
  ab += dLsb * q.dyl;
  dxb += ab * q.dfs;
  const R dfsb = ab * q.dx;
  Lb += Lgb * q.dg;
  const R dgb = Lgb * q.L;
  R lcb = 0.5 * hlcb;
  dyb += dylb / q.L;
  Lb -= dylb * q.dy / (q.L * q.L);
  R u2b = dgb * (3.0 / 20.0);
  R hb = dfqb * q.dx * q.ic2 * kB;
  dxb += dfqb * q.h * q.ic2 * kB;
  R ic2b = dfqb * q.h * q.dx * kB;
  hb += dfsb * (q.ic1 + q.ic2);
  const R ic1b = dfsb * q.h;
  ic2b += dfsb * q.h;
  R c1b = -ic1b / (q.c1 * q.c1);
  R c2b = -ic2b / (q.c2 * q.c2);
  R fb = hb * q.f;
  Lb += dsb * q.sg * q.g;
  gb += dsb * q.sg * q.L;
  u2b += gb * (1.0 / 6.0 + 2.0 * q.u2 * (3.0 / 40.0));
  lcb += u2b * 0.5 * q.lc;
  Lb += lcb * q.cc;
  ccb += lcb * q.L;
  dxb += Lb * q.dx / q.L;
  dyb += Lb * q.dy / q.L;
  dxb += dyb * q.f;
  fb += dyb * q.dx;
  const R den = q.c1 + q.c2;
  const R numb = fb / den, denb = -fb * q.f / den;
  R snpb = numb;
  s2b += numb;
  c1b += denb;
  c2b += denb;
  s2b += c2b * (-q.s2 / q.c2);
  snpb += c1b * (-snp / q.c1);
  snpb += s2b;
  ccb += s2b * q.dx;
  dxb += s2b * q.cc;
  qptb += ccb * kB;
  pb[0] = yb;
  pb[1] = zb;
  pb[2] = snpb;
  pb[3] = tglb;
  pb[4] = qptb;
  return dxb;
}

// Symmetric 5x5 matrices are held as their 15 lower-triangle entries
// (row-major, the checkpoint's covariance order).
__device__ __forceinline__ constexpr int si(int i, int j)
{
  return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
}

// adjoint of the R9 update at predicted state pp, covariance C (symmetric);
// X is the symmetric adjoint of the covariance, updated in place
__device__ __forceinline__ void update_backward(const R* pp, const R* C, R my, R mz, R vy, R vz,
                                                R chib, R* pb, R* X, R* mb)
{
  const R S00 = C[si(0, 0)] + vy, S01 = C[si(0, 1)], S11 = C[si(1, 1)] + vz;
  const R det = S00 * S11 - S01 * S01;
  const R idet = 1.0 / det;
  const R Si[2][2] = {{S11 * idet, -S01 * idet}, {-S01 * idet, S00 * idet}};
  const R r[2] = {my - pp[0], mz - pp[1]};
  R K[5][2];
#pragma unroll
  for (int i = 0; i < 5; i++)
#pragma unroll
    for (int a = 0; a < 2; a++) K[i][a] = C[si(i, 0)] * Si[0][a] + C[si(i, 1)] * Si[1][a];
  const R w[2] = {Si[0][0] * r[0] + Si[0][1] * r[1], Si[1][0] * r[0] + Si[1][1] * r[1]};
  R Ub[5][2], Sib[2][2], rb[2] = {0.0, 0.0}, Utp[2] = {0.0, 0.0};
  // C_out = C - U Si U^T  (U = C[:, 0:2], U Si = K)
#pragma unroll
  for (int i = 0; i < 5; i++)
#pragma unroll
    for (int a = 0; a < 2; a++) {
      R s = 0.0;
#pragma unroll
      for (int j = 0; j < 5; j++) s += X[si(i, j)] * K[j][a];
      Ub[i][a] = -2.0 * s + pb[i] * w[a];  // ... + the p_out = p + U w term
    }
  R XU[5][2];
#pragma unroll
  for (int i = 0; i < 5; i++)
#pragma unroll
    for (int a = 0; a < 2; a++) {
      R s = 0.0;
#pragma unroll
      for (int j = 0; j < 5; j++) s += X[si(i, j)] * C[si(j, a)];
      XU[i][a] = s;
    }
#pragma unroll
  for (int i = 0; i < 5; i++)
#pragma unroll
    for (int a = 0; a < 2; a++) {
      Utp[a] += C[si(i, a)] * pb[i];
      rb[a] += K[i][a] * pb[i];
    }
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int bq = 0; bq < 2; bq++) {
      R s = 0.0;
#pragma unroll
      for (int i = 0; i < 5; i++) s += C[si(i, a)] * XU[i][bq];
      Sib[a][bq] = -s + Utp[a] * r[bq] + chib * r[a] * r[bq];
    }
#pragma unroll
  for (int a = 0; a < 2; a++) rb[a] += 2.0 * chib * w[a];
  // Si = S^-1
  R T[2][2], Smb[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int bq = 0; bq < 2; bq++) T[a][bq] = Si[a][0] * Sib[0][bq] + Si[a][1] * Sib[1][bq];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int bq = 0; bq < 2; bq++) Smb[a][bq] = -(T[a][0] * Si[0][bq] + T[a][1] * Si[1][bq]);
  // symmetric adjoint of S and of U (each off-diagonal pair shares its entry)
  X[si(0, 0)] += Smb[0][0] + Ub[0][0];
  X[si(1, 1)] += Smb[1][1] + Ub[1][1];
  X[si(1, 0)] += 0.5 * (Smb[0][1] + Smb[1][0]) + 0.5 * (Ub[1][0] + Ub[0][1]);
#pragma unroll
  for (int i = 2; i < 5; i++)
#pragma unroll
    for (int a = 0; a < 2; a++) X[si(i, a)] += 0.5 * Ub[i][a];
  mb[0] = rb[0];
  mb[1] = rb[1];
  pb[0] -= rb[0];
  pb[1] -= rb[1];
}

// ---- field map and material (R42-R44) in binary64

constexpr R kHighland2 = 1.8496e-4;   // 0.0136^2 [GeV^2]
constexpr R kPion2 = 0.019479785;     // 0.13957^2 [GeV^2]

// the z bin of a step's field, exactly as the forward pass takes it (this
// file is built with fast math; the bin must not move at a boundary)
#pragma float_control(precise, on, push)
__device__ __forceinline__ int field_zbin(float z, int nzb)
{
  const double f = floor(((double)z + 250.0) * (double)nzb / 500.0);
  if (!(f >= 0.0)) return 0;
  return f > (double)(nzb - 1) ? nzb - 1 : (int)f;
}
#pragma float_control(pop)

// The material step's scalars, a function of the propagated state's snp,
// tgl, q/pt, the step length and the row's material: computed in the
// forward rebuild and again in the adjoint, so that only the inputs (and
// the covariance row of q/pt) stay live across the update's adjoint.
struct MScal {
  R t2, w, bg, sq, path, qt, th2, f;
};

__device__ __forceinline__ MScal mat_scalars(R tgl, R qpt, R ads, R sgn, R ix0, R K)
{
  MScal m;
  m.t2 = 1.0 + tgl * tgl;
  m.w = (qpt * qpt) / m.t2;
  m.bg = 1.0 + kPion2 * m.w;
  m.path = ads * sqrt(m.t2);
  m.qt = qpt * tgl;
  m.th2 = ix0 > 0.0 ? (kHighland2 * (m.path * ix0)) * (m.w * m.bg) : 0.0;
  m.sq = sqrt(m.w * m.bg);
  m.f = 1.0 + (K > 0.0 ? (m.sq * (K * m.bg)) * (m.path * sgn) : 0.0);
  return m;
}

// the material step on the propagated state pp and covariance C (lower
// triangle): the scattering noise on snp, tgl, q/pt, then the energy loss;
// c4 receives the covariance row of q/pt between the two
__device__ __forceinline__ void mat_forward(R* pp, R* C, R ads, R sgn, R ix0, R K, R* c4)
{
  const R snp = pp[2], qpt = pp[4];
  const MScal m = mat_scalars(pp[3], qpt, ads, sgn, ix0, K);
  if (ix0 > 0.0) {
    C[si(2, 2)] += m.th2 * (((1.0 - snp) * (1.0 + snp)) * m.t2);
    C[si(3, 3)] += m.th2 * (m.t2 * m.t2);
    C[si(4, 3)] += m.th2 * (m.t2 * m.qt);
    C[si(4, 4)] += m.th2 * (m.qt * m.qt);
  }
#pragma unroll
  for (int j = 0; j < 5; j++) c4[j] = C[si(4, j)];
  if (K > 0.0) {
    pp[4] = qpt * m.f;
#pragma unroll
    for (int j = 0; j < 4; j++) C[si(4, j)] *= m.f;
    C[si(4, 4)] = (C[si(4, 4)] * m.f) * m.f;
  }
}

// adjoint of mat_forward: pb and X (the symmetric covariance adjoint) go
// from after the material to the propagated state (snp, tgl, q/pt);
// returns the adjoint of the step's signed arc length
__device__ __forceinline__ R mat_backward(R snp, R tgl, R qpt, const R* c4, R ads, R sgn, R ix0,
                                          R K, R* pb, R* X)
{
  const MScal m = mat_scalars(tgl, qpt, ads, sgn, ix0, K);
  R t2b = 0.0, wb = 0.0, bgb = 0.0, pathb = 0.0, qtb = 0.0;
  if (K > 0.0) {
    // q/pt' = q/pt f; row 4 of the covariance scaled by f, its diagonal by f^2
    R s = 0.0;
#pragma unroll
    for (int j = 0; j < 4; j++) s += X[si(4, j)] * c4[j];
    const R cb = pb[4] * qpt + 2.0 * (s + X[si(4, 4)] * c4[4] * m.f);
    pb[4] *= m.f;
#pragma unroll
    for (int j = 0; j < 4; j++) X[si(4, j)] *= m.f;
    X[si(4, 4)] *= m.f * m.f;
    // f - 1 = sq (K bg) (path sgn), sq = sqrt(w bg)
    const R sqb = cb * (K * m.bg) * (m.path * sgn);
    bgb += cb * m.sq * K * (m.path * sgn);
    pathb += cb * m.sq * (K * m.bg) * sgn;
    if (m.sq > 0.0) {
      const R wbgb = sqb / (2.0 * m.sq);
      wb += wbgb * m.bg;
      bgb += wbgb * m.w;
    }
  }
  if (ix0 > 0.0) {
    const R u22 = ((1.0 - snp) * (1.0 + snp)) * m.t2, u33 = m.t2 * m.t2;
    const R u43 = m.t2 * m.qt, u44 = m.qt * m.qt;
    const R x22 = X[si(2, 2)], x33 = X[si(3, 3)], x43 = X[si(4, 3)], x44 = X[si(4, 4)];
    const R A = x22 * u22 + x33 * u33 + 2.0 * x43 * u43 + x44 * u44;
    pb[2] += m.th2 * x22 * (-2.0 * snp) * m.t2;
    t2b += m.th2 * (x22 * ((1.0 - snp) * (1.0 + snp)) + x33 * 2.0 * m.t2 + 2.0 * x43 * m.qt);
    qtb += m.th2 * (2.0 * x43 * m.t2 + x44 * 2.0 * m.qt);
    // th2 = kHighland2 path ix0 w bg
    const R a = A * kHighland2 * ix0;
    pathb += a * m.w * m.bg;
    wb += a * m.path * m.bg;
    bgb += a * m.path * m.w;
  }
  // qt = qpt tgl, bg = 1 + m^2 w, w = qpt^2 / t2, path = ads sqrt(t2), t2 = 1 + tgl^2
  pb[4] += qtb * tgl;
  pb[3] += qtb * qpt;
  wb += bgb * kPion2;
  pb[4] += wb * 2.0 * qpt / m.t2;
  t2b += wb * (-m.w / m.t2);
  const R st2 = sqrt(m.t2);
  const R adsb = pathb * st2;
  t2b += pathb * ads / (2.0 * st2);
  pb[3] += t2b * 2.0 * tgl;
  return adsb * sgn;
}

// adds to the workgroup's partial sums in LDS (flushed once per workgroup);
// true if the term was clamped (the caller raises the overflow flag once)
__device__ __forceinline__ bool acc_add(unsigned long long* acc, int cell, double g)
{
  double v = rint(g * kFix);
  const bool ovf = !(fabs(v) <= kFixMax);
  if (ovf) v = g < 0.0 ? -kFixMax : kFixMax;
  atomicAdd(&acc[cell], (unsigned long long)(long long)v);
  return ovf;
}

// Per-thread LDS buffer of the cluster gradients of kBwdOut hits, written
// to global memory every kBwdOut hits: a load issued after a store is
// waited for together with that store (the counter retires them in order),
// so storing each hit's gradient at once would stall every step's loads.
constexpr int kBwdOut = 8;

struct BwdOut {
  float (*g)[3][kBlock];  // [kBwdOut][x, y, z][thread]
  int32_t (*c)[kBlock];   // [kBwdOut][thread] cluster index
};

__device__ __forceinline__ void out_put(const BwdOut& o, int j, int32_t c, float gx, float gy,
                                        float gz)
{
  const int tx = threadIdx.x;
  o.g[j][0][tx] = gx;
  o.g[j][1][tx] = gy;
  o.g[j][2][tx] = gz;
  o.c[j][tx] = c;
}

__device__ __forceinline__ void out_flush(const RefitBufs& b, const BwdOut& o, int n)
{
  const int tx = threadIdx.x;
  for (int j = 0; j < n; j++) {
    const int32_t c = o.c[j][tx];
    b.gx[c] = o.g[j][0][tx];
    b.gy[c] = o.g[j][1][tx];
    b.gz[c] = o.g[j][2][tx];
  }
}

__global__ __launch_bounds__(kBlock) void k_refit_bwd_zero(RefitBufs b)
{
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < b.n_clusters;
       i += (int64_t)gridDim.x * blockDim.x) {
    b.gx[i] = 0.0f;
    b.gy[i] = 0.0f;
    b.gz[i] = 0.0f;
    if (i < kRows * kPhi) b.acc[i] = 0;
  }
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i < kRows * kPhi; i += blockDim.x) b.acc[i] = 0;
    if (threadIdx.x == 0) b.flags[0] = 0;
  }
}

template <bool MAT>
__device__ __forceinline__ void bwd_track(const Consts& k, const RefitBufs& b, int64_t t,
                                          unsigned long long* acc, const BwdOut& o,
                                          const CkTables& tab, int lmax)
{
  const int64_t a = b.hit_off[t], e = b.hit_off[t + 1];
  if (e - a < 1 || b.status[t] != 0) return;
  // the checkpoints of this wave's group of tracks start at its first hit
  const float4* const ck = reinterpret_cast<const float4*>(b.ckpt) + ck_group_base(b.hit_off) * 5;
  // binary64 throughout: the checkpoints (binary32) are widened on load
  const R kB = -0.299792458e-2 * (R)k.bz, vy = k.vy, vz = k.vz, w = b.grad_chi2[t];
  R pb[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  R X[15];  // symmetric covariance adjoint
#pragma unroll
  for (int i = 0; i < 15; i++) X[i] = 0.0;
  R gXn = 0.0;
  // the forward pass gives status 2 to a track with a hit outside the
  // clusters or the map's rows; the clamps below only keep every access in
  // bounds if the status passed in does not belong to these inputs
  const uint32_t ncl = (uint32_t)b.n_clusters;
  auto clu = [&](int64_t hh) {
    const int32_t v = b.hit_clu[hh > a ? hh : a];
    return (uint32_t)v < ncl ? v : 0;
  };
  auto rowc = [&](int32_t cc) {
    const int r = b.row[cc];
    return r < kRows ? r : kRows - 1;
  };
  int32_t c = clu(e - 1);
  int cell = rowc(c) * kPhi + b.sector[c] % kPhi;
  R X2 = (R)b.x[c] + (R)b.dmap[cell];
  float yc = b.y[c], zc = b.z[c];
  // the hits ahead (downwards) are loaded across steps, with no store in
  // most steps: the cluster index three hits ahead, the cluster's data two
  // ahead and its plane offset one ahead (indices below the first hit are
  // clamped to it; their data is loaded but unused)
  int32_t cp1 = clu(e - 2);
  float x1 = b.x[cp1], y1 = b.y[cp1], z1 = b.z[cp1];
  int cell1 = rowc(cp1) * kPhi + b.sector[cp1] % kPhi;
  float dm1 = b.dmap[cell1];
  int32_t cp2 = clu(e - 3);
  float x2 = b.x[cp2], y2 = b.y[cp2], z2 = b.z[cp2];
  int row2 = rowc(cp2), sec2 = b.sector[cp2];
  int32_t i3 = clu(e - 4);
  bool ovf = false;
  int j = 0;  // gradients buffered in o
  // the wave's lanes step through the hit numbers together, from its
  // longest track's last hit down, each lane from its own last hit on: at
  // every step they read the checkpoints of one hit number, which sit
  // together
  for (int64_t jn = lmax - 1; jn >= 1; jn--) {
    if (jn > e - 1 - a) continue;
    const int64_t h = a + jn;
    const int32_t cp = cp1;
    const int cellp = cell1;
    const R X1 = (R)x1 + (R)dm1;
    const float ycp = y1, zcp = z1;
    // advance the pipeline by one hit
    cp1 = cp2;
    cell1 = row2 * kPhi + sec2 % kPhi;
    dm1 = b.dmap[cell1];
    x1 = x2;
    y1 = y2;
    z1 = z2;
    cp2 = i3;
    x2 = b.x[i3];
    y2 = b.y[i3];
    z2 = b.z[i3];
    row2 = rowc(i3);
    sec2 = b.sector[i3];
    i3 = clu(h - 4);
    // checkpoint h-1: state and covariance (lower triangle, row-major)
    const CkSlot sl = ck_slot(tab, h - 1 - a);
    const float4* q4 = ck + sl.idx;
    const int64_t d4 = sl.stride;
    const float4 v0 = q4[0], v1 = q4[d4], v2 = q4[2 * d4], v3 = q4[3 * d4], v4 = q4[4 * d4];
    const R p0[5] = {v0.x, v0.y, v0.z, v0.w, v1.x};
    const R C0[15] = {v1.y, v1.z, v1.w, v2.x, v2.y, v2.z, v2.w, v3.x,
                      v3.y, v3.z, v3.w, v4.x, v4.y, v4.z, v4.w};
    // the Jacobian F = I + E has six off-identity entries: (0,2) a, (0,4) b,
    // (1,2) d, (1,3) e, (1,4) gq, (2,4) hq
    // the step's field (R42): the destination hit's row and z bin
    R kBs = kB;
    if constexpr (MAT) {
      if (b.bz) kBs = -0.299792458e-2 * (R)b.bz[(int64_t)(cell / kPhi) * b.nzb + field_zbin(zc, b.nzb)];
    }
    R Ea, Eb, Ed, Ee, Egq, Ehq, pp[5], dss = 0.0, sgs = 1.0;
    {
      PRec q;
      prop_record(p0, X2 - X1, kBs, q);
      dss = q.ds;
      sgs = q.sg;
      Ea = q.a;
      Eb = q.b;
      Ed = q.d;
      Ee = q.e;
      Egq = q.gq;
      Ehq = q.hq;
      pp[0] = p0[0] + q.dy;
      pp[1] = p0[1] + p0[3] * q.ds;
      pp[2] = q.s2;
      pp[3] = p0[3];
      pp[4] = p0[4];
    }
    // predicted covariance F C0 F^T: rows 0-2 of B = F C0, then B F^T
    R B[3][5];
#pragma unroll
    for (int j = 0; j < 5; j++) {
      B[0][j] = C0[si(0, j)] + Ea * C0[si(2, j)] + Eb * C0[si(4, j)];
      B[1][j] = C0[si(1, j)] + Ed * C0[si(2, j)] + Ee * C0[si(3, j)] + Egq * C0[si(4, j)];
      B[2][j] = C0[si(2, j)] + Ehq * C0[si(4, j)];
    }
    R Cp[15];
#pragma unroll
    for (int i = 0; i < 5; i++) {
      // row i of B (rows 3, 4 are those of C0)
      R Bi[5];
#pragma unroll
      for (int m = 0; m < 5; m++) Bi[m] = i < 3 ? B[i < 3 ? i : 0][m] : C0[si(i, m)];
      Cp[si(i, 0)] = Bi[0] + Ea * Bi[2] + Eb * Bi[4];
      if (i >= 1) Cp[si(i, 1)] = Bi[1] + Ed * Bi[2] + Ee * Bi[3] + Egq * Bi[4];
      if (i >= 2) Cp[si(i, 2)] = Bi[2] + Ehq * Bi[4];
      if (i >= 3) Cp[si(i, 3)] = Bi[3];
      if (i >= 4) Cp[si(i, 4)] = Bi[4];
    }
    // the material of the step (R43, R44) on the propagated state; what its
    // adjoint needs besides these inputs is recomputed there
    const bool mat = MAT && (b.ix0 || b.eloss);
    R m_snp = 0.0, m_tgl = 0.0, m_qpt = 0.0, m_ix0 = 0.0, m_K = 0.0, c4[5];
    if constexpr (MAT) {
      if (mat) {
        m_snp = pp[2];
        m_tgl = pp[3];
        m_qpt = pp[4];
        const int rr = cell / kPhi;
        m_ix0 = b.ix0 ? (R)b.ix0[rr] : 0.0;
        m_K = b.eloss ? (R)b.eloss[rr] : 0.0;
        mat_forward(pp, Cp, dss * sgs, sgs, m_ix0, m_K, c4);
      }
    }
    R mb[2];
    update_backward(pp, Cp, (R)yc, (R)zc, vy, vz, w, pb, X, mb);
    R dsb_mat = 0.0;
    if constexpr (MAT) {
      if (mat)
        dsb_mat = mat_backward(m_snp, m_tgl, m_qpt, c4, dss * sgs, sgs, m_ix0, m_K, pb, X);
    }
    // covariance part of the propagation: XF = X F, Fb = 2 (X F C0) at the
    // entries of E, X <- F^T X F
    R XF[5][5];
#pragma unroll
    for (int i = 0; i < 5; i++) {
      const R x0 = X[si(i, 0)], x1 = X[si(i, 1)], x2 = X[si(i, 2)];
      XF[i][0] = x0;
      XF[i][1] = x1;
      XF[i][2] = x2 + Ea * x0 + Ed * x1;
      XF[i][3] = X[si(i, 3)] + Ee * x1;
      XF[i][4] = X[si(i, 4)] + Eb * x0 + Egq * x1 + Ehq * x2;
    }
    R Fb[6];
    {
      const int fi[6] = {0, 0, 1, 1, 1, 2}, fj[6] = {2, 4, 2, 3, 4, 4};
#pragma unroll
      for (int u = 0; u < 6; u++) {
        R s = 0.0;
#pragma unroll
        for (int m = 0; m < 5; m++) s += XF[fi[u]][m] * C0[si(m, fj[u])];
        Fb[u] = 2.0 * s;
      }
    }
    // F^T XF, lower triangle (row i of F^T XF adds the E entries of column i)
#pragma unroll
    for (int i = 0; i < 5; i++)
#pragma unroll
      for (int j = 0; j <= i; j++) {
        R v = XF[i][j];
        if (i == 2) v += Ea * XF[0][j] + Ed * XF[1][j];
        if (i == 3) v += Ee * XF[1][j];
        if (i == 4) v += Eb * XF[0][j] + Egq * XF[1][j] + Ehq * XF[2][j];
        X[si(i, j)] = v;
      }
    // the scalar chain of the propagation (its record rebuilt here, so that
    // it is not held through the covariance part; the empty asm statements
    // make the inputs opaque, so the compiler rebuilds instead of keeping the
    // first record)
    R dxr = X2 - X1;
    R pr[5] = {p0[0], p0[1], p0[2], p0[3], p0[4]};
    asm volatile("" : "+v"(dxr), "+v"(pr[2]), "+v"(pr[3]), "+v"(pr[4]));
    PRec q;
    prop_record(pr, dxr, kBs, q);
    const R dxb = prop_backward(pr, q, kBs, pb, Fb, dsb_mat);
    const R gX = dxb + gXn;
    out_put(o, j, c, (float)gX, (float)mb[0], (float)mb[1]);
    if (++j == kBwdOut) {
      out_flush(b, o, j);
      j = 0;
    }
    ovf |= acc_add(acc, cell, gX);
    gXn = -dxb;
    c = cp;
    cell = cellp;
    X2 = X1;
    yc = ycp;
    zc = zcp;
  }
  out_put(o, j, c, (float)gXn, (float)pb[0], (float)pb[1]);
  out_flush(b, o, j + 1);
  ovf |= acc_add(acc, cell, gXn);
  if (ovf) atomicOr(b.flags, 1);
}

// One lane per track; the map sums of the workgroup's tracks are gathered
// in LDS and added to the device accumulators once per cell.  MAT: field
// map and material.
template <bool MAT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_refit_bwd(Consts k, RefitBufs b)
{
  __shared__ unsigned long long s_acc[kRows * kPhi];
  __shared__ float s_og[kBwdOut][3][kBlock];
  __shared__ int32_t s_oc[kBwdOut][kBlock];
  __shared__ CkTables s_ck;
  for (int i = threadIdx.x; i < kRows * kPhi; i += kBlock) s_acc[i] = 0ull;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int lmax;
  ck_build(s_ck, b.hit_off, b.n_tracks, t, lmax);  // ends with a barrier
  if (t < b.n_tracks) bwd_track<MAT>(k, b, t, s_acc, BwdOut{s_og, s_oc}, s_ck, lmax);
  __syncthreads();
  for (int i = threadIdx.x; i < kRows * kPhi; i += kBlock) {
    const unsigned long long v = s_acc[i];
    if (v) atomicAdd(reinterpret_cast<unsigned long long*>(&b.acc[i]), v);
  }
}

__global__ void k_refit_bwd_map(RefitBufs b)
{
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kRows * kPhi) b.grad_map[i] = (float)((double)b.acc[i] / kFix);
}

}  // namespace

// Device memory of the allocation-free entry point: the reverse pass's map
// accumulators and overflow flag (the same layout as its workspace).  Each
// GPU holds its own copy until the process ends; every allocation-free call
// on a GPU shares it.  Host code never uses the array's name as an address:
// kernels get the device address that hipGetSymbolAddress returns.
constexpr size_t kScratchBytes = 8 * kRows * kPhi + 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// the current device's address of `scratch`, looked up once per device
hipError_t scratch_address(void** out)
{
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

size_t refit_scratch_bytes() { return kScratchBytes; }

hipError_t refit_backward_noalloc(const Consts& k, RefitBufs b, hipStream_t s)
{
  void* p = nullptr;
  const hipError_t e = scratch_address(&p);
  if (e != hipSuccess) return e;
  b.acc = static_cast<long long*>(p);
  b.flags = reinterpret_cast<int*>(static_cast<char*>(p) + 8 * kRows * kPhi);
  return refit_backward(k, b, s);
}

hipError_t refit_backward(const Consts& k, const RefitBufs& b, hipStream_t s)
{
  const int64_t zc = b.n_clusters > kRows * kPhi ? b.n_clusters : kRows * kPhi;
  int64_t zb = (zc + kBlock - 1) / kBlock;
  if (zb > 65535) zb = 65535;
  int slot = prof_begin(s, "refit_bwd_zero");
  k_refit_bwd_zero<<<(unsigned)zb, kBlock, 0, s>>>(b);
  prof_end(s, slot);
  if (b.n_tracks > 0) {
    const unsigned nb = (unsigned)((b.n_tracks + kBlock - 1) / kBlock);
    const bool mat = b.bz || b.ix0 || b.eloss;
    slot = prof_begin(s, mat ? "refit_bwd_mat" : "refit_bwd");
    if (mat)
      k_refit_bwd<true><<<nb, kBlock, 0, s>>>(k, b);
    else
      k_refit_bwd<false><<<nb, kBlock, 0, s>>>(k, b);
    prof_end(s, slot);
  }
  slot = prof_begin(s, "refit_bwd_map");
  k_refit_bwd_map<<<(kRows * kPhi + kBlock - 1) / kBlock, kBlock, 0, s>>>(b);
  prof_end(s, slot);
  return hipGetLastError();
}

}  // namespace bwd
}  // namespace tpcca
