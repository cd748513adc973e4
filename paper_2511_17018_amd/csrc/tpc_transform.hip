// Cluster coordinate transformation with corrections (f3), gfx950: raw
// readout coordinates (sector, row, pad, time) to the tracker's local
// (x, y, z) -- the step before the grid build.  Compiled into the
// deterministic build (no contraction, correctly rounded division: the
// output equals the binary32 CPU reference bit for bit) and the production
// build.
//
// The work is elementwise and HBM-bound (11 bytes in, 14 out per cluster):
// each thread takes four consecutive clusters with one vector load per input
// array and one vector store per output array; the per-row constants sit in
// LDS (a lane's row is arbitrary), the two correction maps are read through
// the cache (the clusters of one instance share a sector, so neighbouring
// lanes read neighbouring nodes).
#include "tpc_internal.h"

#ifndef TPC_NS
#error "TPC_NS must name the build (det or prod)"
#endif

namespace tpcca {
namespace TPC_NS {
namespace {

struct RowC {
  float x, w, c, pad_;
};

// one axis of the trilinear lookup: cell index and fraction (outside the
// grid the boundary values continue)
__device__ __forceinline__ void cell(float q, float q0, float iq, int n, int& i, float& a)
{
  const float f = (q - q0) * iq;
  const float fl = floorf(f);
  int k;
  if (!(fl > 0.0f)) k = 0;
  else if (fl > (float)(n - 2)) k = n - 2;
  else k = (int)fl;
  float t = f - (float)k;
  if (!(t > 0.0f)) t = 0.0f;
  if (t > 1.0f) t = 1.0f;
  i = k;
  a = t;
}

__device__ __forceinline__ float lerp1(float a, float b, float t) { return a + (b - a) * t; }

__device__ __forceinline__ float4 lerp4(float4 a, float4 b, float t)
{
  return make_float4(lerp1(a.x, b.x, t), lerp1(a.y, b.y, t), lerp1(a.z, b.z, t), 0.0f);
}

struct Out1 {
  float x, y, z;
  uint16_t row;
};

__device__ __forceinline__ Out1 transform1(const TransformConsts& k, const TransformBufs& b,
                                           const RowC* s_row, int s, int r, float pad,
                                           float time)
{
  Out1 o;
  if (s >= 2 * kPhi || r >= kRows) {
    o.x = o.y = o.z = 0.0f;
    o.row = 0xFFFF;
    return o;
  }
  const bool side = s >= kPhi;
  const int kk = s - (side ? kPhi : 0);
  const RowC rc = s_row[r];
  float xc = rc.x;
  float yc = (pad - rc.c) * rc.w;
  const float d = (time * k.tbin - k.t0) * k.vdrift;
  const float za = k.zlen - d;
  float zc = side ? -za : za;
  if (b.dmap) xc = xc + b.dmap[r * kPhi + kk];
  if (b.rmap) {
    int iu, iv, iw;
    float au, av, aw;
    cell((float)r, k.u0, k.iu, k.nu, iu, au);
    cell(yc / xc, k.v0, k.iv, k.nv, iv, av);
    cell(d, k.w0, k.iw, k.nw, iw, aw);
    const float4* m = b.rmap;
    const int64_t su = (int64_t)k.nv * k.nw;  // node stride of u
    const int64_t base = (((int64_t)s * k.nu + iu) * k.nv + iv) * k.nw + iw;
    const float4 n000 = m[base], n001 = m[base + 1];
    const float4 n010 = m[base + k.nw], n011 = m[base + k.nw + 1];
    const float4 n100 = m[base + su], n101 = m[base + su + 1];
    const float4 n110 = m[base + su + k.nw], n111 = m[base + su + k.nw + 1];
    const float4 e00 = lerp4(n000, n001, aw), e01 = lerp4(n010, n011, aw);
    const float4 e10 = lerp4(n100, n101, aw), e11 = lerp4(n110, n111, aw);
    const float4 f0 = lerp4(e00, e01, av), f1 = lerp4(e10, e11, av);
    const float4 cr = lerp4(f0, f1, au);
    xc = xc + cr.x;
    yc = yc + cr.y;
    zc = zc + cr.z;
  }
  o.x = xc;
  o.y = yc;
  o.z = zc;
  o.row = (uint16_t)r;
  return o;
}

constexpr int kPer = 4;  // clusters per thread

__global__ __launch_bounds__(kBlock) void k_transform(TransformConsts k, TransformBufs b)
{
  __shared__ RowC s_row[kRows];
  for (int r = threadIdx.x; r < kRows; r += kBlock)
    s_row[r] = RowC{k.row_x[r], k.pad_w[r], k.pad_c[r], 0.0f};
  __syncthreads();
  const int64_t c0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kPer;
  if (c0 >= b.n) return;
  if (c0 + kPer <= b.n && b.aligned) {
    // four clusters with one load per input array, one store per output
    const uint32_t sv = *reinterpret_cast<const uint32_t*>(b.sector + c0);
    const uint2 rv = *reinterpret_cast<const uint2*>(b.row + c0);
    const float4 pv = *reinterpret_cast<const float4*>(b.pad + c0);
    const float4 tv = *reinterpret_cast<const float4*>(b.time + c0);
    const int ss[kPer] = {(int)(sv & 0xFF), (int)((sv >> 8) & 0xFF), (int)((sv >> 16) & 0xFF),
                          (int)(sv >> 24)};
    const int rr[kPer] = {(int)(rv.x & 0xFFFF), (int)(rv.x >> 16), (int)(rv.y & 0xFFFF),
                          (int)(rv.y >> 16)};
    const float pp[kPer] = {pv.x, pv.y, pv.z, pv.w};
    const float tt[kPer] = {tv.x, tv.y, tv.z, tv.w};
    Out1 o[kPer];
#pragma unroll
    for (int u = 0; u < kPer; u++) o[u] = transform1(k, b, s_row, ss[u], rr[u], pp[u], tt[u]);
    *reinterpret_cast<float4*>(b.x + c0) = make_float4(o[0].x, o[1].x, o[2].x, o[3].x);
    *reinterpret_cast<float4*>(b.y + c0) = make_float4(o[0].y, o[1].y, o[2].y, o[3].y);
    *reinterpret_cast<float4*>(b.z + c0) = make_float4(o[0].z, o[1].z, o[2].z, o[3].z);
    *reinterpret_cast<uint2*>(b.row_out + c0) =
        make_uint2((uint32_t)o[0].row | ((uint32_t)o[1].row << 16),
                   (uint32_t)o[2].row | ((uint32_t)o[3].row << 16));
  } else {
    for (int64_t c = c0; c < c0 + kPer && c < b.n; c++) {
      const Out1 o = transform1(k, b, s_row, b.sector[c], b.row[c], b.pad[c], b.time[c]);
      b.x[c] = o.x;
      b.y[c] = o.y;
      b.z[c] = o.z;
      b.row_out[c] = o.row;
    }
  }
}

}  // namespace

hipError_t cluster_transform(const TransformConsts& k, const TransformBufs& b, hipStream_t s)
{
  if (b.n > 0) {
    const int64_t threads = (b.n + kPer - 1) / kPer;
    const unsigned nb = (unsigned)((threads + kBlock - 1) / kBlock);
    const int slot = prof_begin(s, "transform");
    k_transform<<<nb, kBlock, 0, s>>>(k, b);
    prof_end(s, slot);
  }
  return hipGetLastError();
}

}  // namespace TPC_NS
}  // namespace tpcca
