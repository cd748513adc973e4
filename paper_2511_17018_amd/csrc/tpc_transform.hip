// Cluster coordinate transformation with corrections (f3), gfx950: raw
// readout coordinates (sector, row, pad, time) to the tracker's local
// (x, y, z) -- the step before the grid build.  Compiled into the
// deterministic build (no contraction, correctly rounded division: the
// output equals the binary32 CPU reference bit for bit) and the production
// build.
//
// The work is elementwise and HBM-bound (11 bytes in, 14 out per cluster):
// each thread takes four consecutive clusters per pass with one vector load
// per input array and one vector store per output array, and a workgroup
// runs kTPass such passes over a contiguous range.  The per-row constants
// sit in LDS (a lane's row is arbitrary), and so does the residual map of
// one sector -- the sector of the range's first cluster, which in practice
// is the sector of the whole range, since a sector's clusters are contiguous
// -- because its eight corner nodes per cluster, gathered from global
// memory, cost one cache-line request per lane each.  Clusters of another
// sector, and maps larger than the LDS copy, read the nodes through the
// cache.  The radial map is read through the cache.
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

constexpr int kMapLds = 4096;  // residual-map nodes (float4) of one sector in LDS

__device__ __forceinline__ Out1 transform1(const TransformConsts& k, const TransformBufs& b,
                                           const RowC* s_row, const float4* s_map, int s_sec,
                                           int s, int r, float pad, float time)
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
    const int64_t su = (int64_t)k.nv * k.nw;  // node stride of u
    const int64_t cb = ((int64_t)iu * k.nv + iv) * k.nw + iw;  // within the sector
    // the sector staged in LDS, else the global map
    const float4* m = s == s_sec ? s_map : b.rmap + (int64_t)s * k.nu * su;
    const float4 n000 = m[cb], n001 = m[cb + 1];
    const float4 n010 = m[cb + k.nw], n011 = m[cb + k.nw + 1];
    const float4 n100 = m[cb + su], n101 = m[cb + su + 1];
    const float4 n110 = m[cb + su + k.nw], n111 = m[cb + su + k.nw + 1];
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

constexpr int kPer = 4;    // clusters per thread and pass
constexpr int kTPass = 8;  // passes per workgroup

__global__ __launch_bounds__(kBlock) void k_transform(TransformConsts k, TransformBufs b)
{
  __shared__ RowC s_row[kRows];
  __shared__ float4 s_map[kMapLds];
  for (int r = threadIdx.x; r < kRows; r += kBlock)
    s_row[r] = RowC{k.row_x[r], k.pad_w[r], k.pad_c[r], 0.0f};
  const int64_t r0 = (int64_t)blockIdx.x * kBlock * kPer * kTPass;  // the workgroup's range
  // the residual map of the range's first sector in LDS (-1: none staged)
  int s_sec = -1;
  const int64_t nodes = (int64_t)k.nu * k.nv * k.nw;
  if (b.rmap && nodes <= kMapLds) {
    const int s = b.sector[r0];
    if (s < 2 * kPhi) {
      s_sec = s;
      const float4* src = b.rmap + (int64_t)s * nodes;
      for (int i = threadIdx.x; i < nodes; i += kBlock) s_map[i] = src[i];
    }
  }
  __syncthreads();
  for (int pass = 0; pass < kTPass; pass++) {
    const int64_t c0 = r0 + ((int64_t)pass * kBlock + threadIdx.x) * kPer;
    if (c0 >= b.n) break;
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
      for (int u = 0; u < kPer; u++)
        o[u] = transform1(k, b, s_row, s_map, s_sec, ss[u], rr[u], pp[u], tt[u]);
      *reinterpret_cast<float4*>(b.x + c0) = make_float4(o[0].x, o[1].x, o[2].x, o[3].x);
      *reinterpret_cast<float4*>(b.y + c0) = make_float4(o[0].y, o[1].y, o[2].y, o[3].y);
      *reinterpret_cast<float4*>(b.z + c0) = make_float4(o[0].z, o[1].z, o[2].z, o[3].z);
      *reinterpret_cast<uint2*>(b.row_out + c0) =
          make_uint2((uint32_t)o[0].row | ((uint32_t)o[1].row << 16),
                     (uint32_t)o[2].row | ((uint32_t)o[3].row << 16));
    } else {
      for (int64_t c = c0; c < c0 + kPer && c < b.n; c++) {
        const Out1 o =
            transform1(k, b, s_row, s_map, s_sec, b.sector[c], b.row[c], b.pad[c], b.time[c]);
        b.x[c] = o.x;
        b.y[c] = o.y;
        b.z[c] = o.z;
        b.row_out[c] = o.row;
      }
    }
  }
}

}  // namespace

hipError_t cluster_transform(const TransformConsts& k, const TransformBufs& b, hipStream_t s)
{
  if (b.n > 0) {
    const int64_t per_block = (int64_t)kBlock * kPer * kTPass;
    const unsigned nb = (unsigned)((b.n + per_block - 1) / per_block);
    const int slot = prof_begin(s, "transform");
    k_transform<<<nb, kBlock, 0, s>>>(k, b);
    prof_end(s, slot);
  }
  return hipGetLastError();
}

}  // namespace TPC_NS
}  // namespace tpcca
