// Kalman refit of found tracks under a per-row distortion map (a8), gfx950.
// Compiled into the deterministic and the production build like the tracker
// kernels: in the deterministic build the chi2 and the checkpoints equal the
// binary32 CPU reference bit for bit.
#include "tpc_internal.h"
#include "tpc_ckpt.h"

#ifndef TPC_NS
#error "TPC_NS must name the build (det or prod)"
#endif

namespace tpcca {
namespace TPC_NS {
namespace {

#include "tpc_kalman.h"

// the five 16-byte parts of a checkpoint at q[0], q[d], .. q[4 d]
__device__ __forceinline__ void store_ckpt(float4* q, int64_t d, const KSt& st)
{
  q[0] = make_float4(st.p[0], st.p[1], st.p[2], st.p[3]);
  q[d] = make_float4(st.p[4], st.c[0], st.c[1], st.c[2]);
  q[2 * d] = make_float4(st.c[3], st.c[4], st.c[5], st.c[6]);
  q[3 * d] = make_float4(st.c[7], st.c[8], st.c[9], st.c[10]);
  q[4 * d] = make_float4(st.c[11], st.c[12], st.c[13], st.c[14]);
}

constexpr int kFwdBlk = 8;  // hits per load block of the forward pass

// every hit of [h, e) names a cluster below ncl on a row of the map
__device__ __noinline__ bool hits_valid(const RefitBufs& b, int64_t h, int64_t e, uint32_t ncl)
{
  for (; h < e; h++) {
    const int32_t c = b.hit_clu[h];
    if ((uint32_t)c >= ncl || b.row[c] >= kRows) return false;
  }
  return true;
}

// Highland constant squared [GeV^2] and the pion mass squared [GeV^2] of
// the material model, as binary32 constants (rounded from these decimals)
constexpr float kHighland2 = (float)1.8496e-4;
constexpr float kPion2 = (float)0.019479785;

// R42: curvature constant of a step from the field at the destination
// hit's row and the z bin of its measured z (binary64, rounded once)
__device__ __forceinline__ float step_kB(const Consts& k, const RefitBufs& b, int row, float z)
{
  if (!b.bz) return k.kB;
  const int nzb = b.nzb;
  const double f = floor(((double)z + 250.0) * (double)nzb / 500.0);
  int zb = 0;
  if (f >= 0.0) zb = f > (double)(nzb - 1) ? nzb - 1 : (int)f;
  return (float)(-0.299792458e-2 * (double)b.bz[(int64_t)row * nzb + zb]);
}

// R43, R44: the material of a step, applied to the propagated state: the
// scattering noise on snp, tgl, q/pt, then the energy loss scaling q/pt and
// the covariance row of q/pt.  ads = |ds|, sgn = sign of the step in x.
__device__ __forceinline__ void mat_step(KSt& s, float ads, float sgn, float ix0, float K)
{
  const float one = 1.0f;
  const float snp = s.p[2], tgl = s.p[3], qpt = s.p[4];
  const float t2 = one + tgl * tgl;
  const float w = (qpt * qpt) / t2;
  const float bg = one + kPion2 * w;
  const float path = ads * sqrtf(t2);
  if (ix0 > 0.0f) {
    const float th2 = (kHighland2 * (path * ix0)) * (w * bg);
    const float qt = qpt * tgl;
    s.c[ci(2, 2)] = s.c[ci(2, 2)] + th2 * (((one - snp) * (one + snp)) * t2);
    s.c[ci(3, 3)] = s.c[ci(3, 3)] + th2 * (t2 * t2);
    s.c[ci(4, 3)] = s.c[ci(4, 3)] + th2 * (t2 * qt);
    s.c[ci(4, 4)] = s.c[ci(4, 4)] + th2 * (qt * qt);
  }
  if (K > 0.0f) {
    const float corr = (sqrtf(w * bg) * (K * bg)) * (path * sgn);
    const float f = one + corr;
    s.p[4] = qpt * f;
#pragma unroll
    for (int j = 0; j < 4; j++) s.c[ci(4, j)] = s.c[ci(4, j)] * f;
    s.c[ci(4, 4)] = (s.c[ci(4, 4)] * f) * f;
  }
}

// R21-R24: one lane per track; planes X_k = x_k + D[row_k][sector_k mod 18].
// MAT: field map and material (R42-R44), read per hit.
template <bool MAT>
__global__ __launch_bounds__(kBlock) void k_refit_fwd(Consts k, RefitBufs b)
{
  __shared__ CkTables s_ck;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int lmax;
  ck_build(s_ck, b.hit_off, b.n_tracks, t, lmax);
  if (t >= b.n_tracks) return;
  // the checkpoints of this wave's group of tracks start at its first hit
  float4* const ck = reinterpret_cast<float4*>(b.ckpt) + ck_group_base(b.hit_off) * 5;
  const int64_t a = b.hit_off[t], e = b.hit_off[t + 1];
  if (e <= a) {
    b.chi2[t] = 0.0f;
    b.status[t] = 0;
    return;
  }
  const float kB = k.kB, vy = k.vy, vz = k.vz, smax = k.snp_max;
  // a hit must name a cluster on one of the map's rows; a track with any
  // other hit is rejected as a whole (status 2), and the loads below use
  // in-range indices whatever the hit list holds
  const uint32_t ncl = (uint32_t)b.n_clusters;
  int32_t c = b.hit_clu[a];
  if ((uint32_t)c >= ncl || b.row[c] >= kRows) {
    b.chi2[t] = 0.0f;
    b.status[t] = 2;
    return;
  }
  KSt st;
  st.p[0] = b.y[c];
  st.p[1] = b.z[c];
  st.p[2] = b.seed[t * 5 + 2];
  st.p[3] = b.seed[t * 5 + 3];
  st.p[4] = b.seed[t * 5 + 4];
  kinit_cov(st, vy, vz);
  {
    const CkSlot sl = ck_slot(s_ck, 0);
    store_ckpt(ck + sl.idx, sl.stride, st);
  }
  float xprev = b.x[c] + b.dmap[(int)b.row[c] * kPhi + b.sector[c] % kPhi];
  float chi2 = 0.0f;
  // the hits go in blocks of kFwdBlk: the block's cluster indices, then
  // its clusters' data and plane offsets are loaded at once, then its hits
  // are filtered and checkpointed.  A load issued after a store is only
  // waited for together with that store (one in-order counter), so the
  // stores cost one wait per block instead of one per hit.
  const int64_t last = e - 1;
  for (int64_t h0 = a + 1; h0 < e; h0 += kFwdBlk) {
    int32_t ci[kFwdBlk];
    bool bad = false;
#pragma unroll
    for (int u = 0; u < kFwdBlk; u++) {
      ci[u] = b.hit_clu[h0 + u < last ? h0 + u : last];
      bad |= (uint32_t)ci[u] >= ncl;
      ci[u] = (uint32_t)ci[u] < ncl ? ci[u] : 0;
    }
    int rw[kFwdBlk];
#pragma unroll
    for (int u = 0; u < kFwdBlk; u++) {
      rw[u] = b.row[ci[u]];
      bad |= rw[u] >= kRows;
      rw[u] = rw[u] < kRows ? rw[u] : 0;
    }
    float xs[kFwdBlk], ys[kFwdBlk], zs[kFwdBlk];
#pragma unroll
    for (int u = 0; u < kFwdBlk; u++) {
      xs[u] = b.x[ci[u]] + b.dmap[rw[u] * kPhi + b.sector[ci[u]] % kPhi];
      ys[u] = b.y[ci[u]];
      zs[u] = b.z[ci[u]];
    }
    // MAT: each hit's field and material (zero where a table is absent)
    float kbs[MAT ? kFwdBlk : 1], ixs[MAT ? kFwdBlk : 1], els[MAT ? kFwdBlk : 1];
    if constexpr (MAT) {
#pragma unroll
      for (int u = 0; u < kFwdBlk; u++) {
        kbs[u] = step_kB(k, b, rw[u], zs[u]);
        ixs[u] = b.ix0 ? b.ix0[rw[u]] : 0.0f;
        els[u] = b.eloss ? b.eloss[rw[u]] : 0.0f;
      }
    }
    if (bad) {
      b.chi2[t] = 0.0f;
      b.status[t] = 2;
      return;
    }
#pragma unroll
    for (int u = 0; u < kFwdBlk; u++) {
      const int64_t h = h0 + u;
      if (h >= e) break;
      float ds;
      if (!kprop_ds(st, xprev, xs[u], MAT ? kbs[MAT ? u : 0] : kB, smax, ds)) {
        // an invalid hit further on still makes the track status 2
        b.chi2[t] = 0.0f;
        b.status[t] = hits_valid(b, h0 + kFwdBlk, e, ncl) ? 1 : 2;
        return;
      }
      if constexpr (MAT) {
        if (b.ix0 || b.eloss) {
          const float sgn = xs[u] - xprev < 0.0f ? -1.0f : 1.0f;
          mat_step(st, ds * sgn, sgn, ixs[u], els[u]);
        }
      }
      chi2 += kupdate(st, ys[u], zs[u], vy, vz);
      const CkSlot sl = ck_slot(s_ck, h - a);
      store_ckpt(ck + sl.idx, sl.stride, st);
      xprev = xs[u];
    }
  }
  b.chi2[t] = chi2;
  b.status[t] = 0;
}

}  // namespace

hipError_t refit_forward(const Consts& k, const RefitBufs& b, hipStream_t s)
{
  if (b.n_tracks > 0) {
    const unsigned nb = (unsigned)((b.n_tracks + kBlock - 1) / kBlock);
    const bool mat = b.bz || b.ix0 || b.eloss;
    const int slot = prof_begin(s, mat ? "refit_fwd_mat" : "refit_fwd");
    if (mat)
      k_refit_fwd<true><<<nb, kBlock, 0, s>>>(k, b);
    else
      k_refit_fwd<false><<<nb, kBlock, 0, s>>>(k, b);
    prof_end(s, slot);
  }
  return hipGetLastError();
}

}  // namespace TPC_NS
}  // namespace tpcca
