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
  int32_t c = b.hit_clu[a];
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
  // software pipeline over the hits: the cluster index is loaded two hits
  // ahead and the cluster's data one hit ahead, so that their gathers overlap
  // the propagation and update of the current hit
  int32_t cn = a + 1 < e ? b.hit_clu[a + 1] : 0;   // index of hit h
  int32_t cnn = a + 2 < e ? b.hit_clu[a + 2] : 0;  // index of hit h + 1
  float xn = b.x[cn], yn = b.y[cn], zn = b.z[cn];
  int rown = b.row[cn], secn = b.sector[cn];
  for (int64_t h = a + 1; h < e; h++) {
    const float xk = xn + b.dmap[rown * kPhi + secn % kPhi];
    const float yk = yn, zk = zn;
    if (h + 1 < e) {
      xn = b.x[cnn];
      yn = b.y[cnn];
      zn = b.z[cnn];
      rown = b.row[cnn];
      secn = b.sector[cnn];
      cnn = h + 2 < e ? b.hit_clu[h + 2] : 0;
    }
    if (!kprop(st, xprev, xk, kB, smax)) {
      b.chi2[t] = 0.0f;
      b.status[t] = 1;
      return;
    }
    chi2 += kupdate(st, yk, zk, vy, vz);
    store_ckpt(b.ckpt + h * 20, st);
    xprev = xk;
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
