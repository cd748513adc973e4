// Kalman refit of found tracks under a per-row distortion map (a8), gfx950.
// Compiled into the deterministic and the production build like the tracker
// kernels: in the deterministic build the chi2 and the checkpoints equal the
// binary32 CPU reference bit for bit.
#include "tpc_internal.h"

#ifndef TPC_NS
#error "TPC_NS must name the build (det or prod)"
#endif

namespace tpcca {
namespace TPC_NS {
namespace {

#include "tpc_kalman.h"

__device__ __forceinline__ void store_ckpt(float* ck, const KSt& st)
{
  float4* q = reinterpret_cast<float4*>(ck);  // 80 bytes, 16-byte aligned
  q[0] = make_float4(st.p[0], st.p[1], st.p[2], st.p[3]);
  q[1] = make_float4(st.p[4], st.c[0], st.c[1], st.c[2]);
  q[2] = make_float4(st.c[3], st.c[4], st.c[5], st.c[6]);
  q[3] = make_float4(st.c[7], st.c[8], st.c[9], st.c[10]);
  q[4] = make_float4(st.c[11], st.c[12], st.c[13], st.c[14]);
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

// R21-R24: one lane per track; planes X_k = x_k + D[row_k][sector_k mod 18].
__global__ __launch_bounds__(kBlock) void k_refit_fwd(Consts k, RefitBufs b)
{
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= b.n_tracks) return;
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
  store_ckpt(b.ckpt + a * 20, st);
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
    if (bad) {
      b.chi2[t] = 0.0f;
      b.status[t] = 2;
      return;
    }
#pragma unroll
    for (int u = 0; u < kFwdBlk; u++) {
      const int64_t h = h0 + u;
      if (h >= e) break;
      if (!kprop(st, xprev, xs[u], kB, smax)) {
        // an invalid hit further on still makes the track status 2
        b.chi2[t] = 0.0f;
        b.status[t] = hits_valid(b, h0 + kFwdBlk, e, ncl) ? 1 : 2;
        return;
      }
      chi2 += kupdate(st, ys[u], zs[u], vy, vz);
      store_ckpt(b.ckpt + h * 20, st);
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
    const int slot = prof_begin(s, "refit_fwd");
    k_refit_fwd<<<nb, kBlock, 0, s>>>(k, b);
    prof_end(s, slot);
  }
  return hipGetLastError();
}

}  // namespace TPC_NS
}  // namespace tpcca
