// Sector-track merging and global refit (f1), gfx950.  Compiled into the
// deterministic build (no contraction, correctly rounded division and
// square root: the outputs equal the binary32 CPU reference bit for bit) and
// the production build.
//
// Steps (one kernel each; counts come from the tracker's device result, so
// no host round trip):
//   seg_info     one lane per segment: its sector, the global positions of
//                its first and last hit, its outer state (outward filter over
//                its own hits)
//   buckets      every segment filed twice, by (instance, z bin) of its
//                first hit and of its last hit: counts, one-block offsets,
//                scatter
//   pairs        three lanes per segment (one per neighbouring instance),
//                groups in bucket order (neighbouring lanes search
//                neighbouring buckets): best successor among the segments
//                whose first hit lies in the z bins that R37's z cut can
//                reach from the lane's last hit -- a superset of the pairs
//                that pass it, with the pick a total order (chi2, index), so
//                the result equals the search over all pairs; each passing
//                pair also bids for its candidate's best predecessor by an
//                atomic minimum of the same order
//   link, chain  mutual links; chain heads compacted by scans in index order
//                (link cycles after them, from their lowest segment); chain
//                lengths and hit counts scanned into offsets (workgroup
//                sums, one-workgroup scan of the sums, ordered write)
//   chain_hits   one wave per chain: segment list, merged hit list (and the
//                tracker's hit data in merged order)
//   refit        one lane per chain: outward and inward filter with
//                rotations between the sector frames
#include "tpc_internal.h"

#ifndef TPC_NS
#error "TPC_NS must name the build (det or prod)"
#endif

namespace tpcca {
namespace TPC_NS {
namespace {

#include "tpc_kalman.h"

constexpr int kInst = 2 * kPhi;
constexpr float kSmax = 0.99f;
constexpr float kInwardScale = 100.0f;

__device__ __forceinline__ int64_t gid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

// instance of input index c (inst_off has kInst + 1 entries)
__device__ __forceinline__ int inst_of(const int64_t* off, int64_t c)
{
  int lo = 0, hi = kInst;
  while (hi - lo > 1) {
    const int m = (lo + hi) / 2;
    if (off[m] <= c) lo = m;
    else hi = m;
  }
  return lo;
}

// R36: rotation by (ca, sa) at the state's point x; new plane in xn
__device__ __forceinline__ bool mrot(KSt& s, float x, float ca, float sa, float kB, float& xn)
{
  const float one = 1.0f;
  const float snp = s.p[2];
  if (!(fabsf(snp) < kSmax)) return false;
  const float csp = sqrtf((one - snp) * (one + snp));
  const float csn = csp * ca + snp * sa;
  const float snn = snp * ca - csp * sa;
  if (!(csn > 0.0f) || !(fabsf(snn) < kSmax)) return false;
  const float y = s.p[0];
  xn = x * ca + y * sa;
  s.p[0] = y * ca - x * sa;
  s.p[2] = snn;
  const float j00 = ca - sa * (snn / csn);
  const float j10 = -(s.p[3] * (sa / csn));
  const float j20 = -(kB * s.p[4]) * sa;
  const float j22 = csn / csp;
  float c[5][5];
#pragma unroll
  for (int i = 0; i < 5; i++)
#pragma unroll
    for (int j = 0; j < 5; j++) c[i][j] = s.c[ci(i, j)];
  float t[5][5];
#pragma unroll
  for (int j = 0; j < 5; j++) {
    t[0][j] = j00 * c[0][j];
    t[1][j] = c[1][j] + j10 * c[0][j];
    t[2][j] = j20 * c[0][j] + j22 * c[2][j];
    t[3][j] = c[3][j];
    t[4][j] = c[4][j];
  }
#pragma unroll
  for (int i = 0; i < 5; i++) {
    const float r[5] = {j00 * t[i][0], t[i][1] + j10 * t[i][0], j20 * t[i][0] + j22 * t[i][2],
                        t[i][3], t[i][4]};
#pragma unroll
    for (int j = 0; j <= i; j++) s.c[ci(i, j)] = r[j];
  }
  return true;
}

__device__ __forceinline__ bool mmove(KSt& s, float x1, float x2, float kB)
{
  if (x1 == x2) return true;
  return kprop(s, x1, x2, kB, kSmax);
}

// R36: into the rotated frame and onto plane xh (target point (xh, yh));
// rotation at the state's point, else at the target point
__device__ __forceinline__ bool mtransport(KSt& s, float& x, float ca, float sa, float xh, float yh,
                                        float kB)
{
  KSt t = s;
  float xr;
  if (mrot(t, x, ca, sa, kB, xr) && mmove(t, xr, xh, kB)) {
    s = t;
    x = xh;
    return true;
  }
  t = s;
  const float xc = xh * ca - yh * sa;
  if (mmove(t, x, xc, kB) && mrot(t, xc, ca, sa, kB, xr) && mmove(t, xr, xh, kB)) {
    s = t;
    x = xh;
    return true;
  }
  return false;
}

// R37: d^T S^-1 d by LDL^T (negative if S is not positive definite)
__device__ __forceinline__ float mchi2(const float* S, const float* d)
{
  float L[5][5], D[5];
#pragma unroll
  for (int i = 0; i < 5; i++) {
#pragma unroll
    for (int j = 0; j < i; j++) {
      float v = S[ci(i, j)];
#pragma unroll
      for (int k = 0; k < j; k++) v = v - L[i][k] * (L[j][k] * D[k]);
      L[i][j] = v / D[j];
    }
    float v = S[ci(i, i)];
#pragma unroll
    for (int k = 0; k < i; k++) v = v - L[i][k] * (L[i][k] * D[k]);
    if (!(v > 0.0f)) return -1.0f;
    D[i] = v;
  }
  float w[5], chi2 = 0.0f;
#pragma unroll
  for (int i = 0; i < 5; i++) {
    float v = d[i];
#pragma unroll
    for (int k = 0; k < i; k++) v = v - L[i][k] * w[k];
    w[i] = v;
    chi2 = chi2 + (v * v) / D[i];
  }
  return chi2;
}

// R40: filter pass over the hits at first + dir q, q < count, from state s
// at plane x in frame k; chi2 accumulates.  The hits go in blocks of kMBlk.
// HD = false: hits[] holds cluster indices, and the block's indices, then
// their rows, positions and sectors, then the row planes are loaded at once
// (three memory latencies per block instead of three per hit); HD = true:
// hd[] holds each hit's plane, position and sector (the tracker's hit data),
// one contiguous load per hit.  The block's hits in the current frame are
// filtered in an unrolled loop; the first hit of another sector ends it,
// is transported (one copy of that code) and filtered, and the next block
// starts after it.
constexpr int kMBlk = 8;

template <bool HD>
__device__ __forceinline__ bool mpass(const Consts& k, const MergeBufs& b, const int64_t* s_off,
                                   KSt& s, float& x, int& kf, const int32_t* hits,
                                   const float4* hd, int64_t first, int64_t count, int dir,
                                   float& chi2)
{
  const float kB = k.kB, vy = k.vy, vz = k.vz;
  int64_t q = 0;
  while (q < count) {
    int kk[kMBlk];
    float xh[kMBlk], yc[kMBlk], zc[kMBlk];
    if constexpr (HD) {
#pragma unroll
      for (int u = 0; u < kMBlk; u++) {
        const float4 d = hd[first + dir * (q + u < count ? q + u : count - 1)];
        xh[u] = d.x;
        yc[u] = d.y;
        zc[u] = d.z;
        kk[u] = (int)d.w;
      }
    } else {
      int64_t c[kMBlk];
#pragma unroll
      for (int u = 0; u < kMBlk; u++)
        c[u] = hits[first + dir * (q + u < count ? q + u : count - 1)];
      int rw[kMBlk];
#pragma unroll
      for (int u = 0; u < kMBlk; u++) {
        rw[u] = b.row[c[u]];
        yc[u] = b.y[c[u]];
        zc[u] = b.z[c[u]];
        kk[u] = inst_of(s_off, c[u]) % kPhi;
      }
#pragma unroll
      for (int u = 0; u < kMBlk; u++) xh[u] = k.row_x[rw[u]];
    }
    int done = 0;
    bool rot = false;
#pragma unroll
    for (int u = 0; u < kMBlk; u++) {
      if (!rot && q + u < count) {
        if (kk[u] != kf) {
          rot = true;
        } else {
          if (!mmove(s, x, xh[u], kB)) return false;
          x = xh[u];
          chi2 = chi2 + kupdate(s, yc[u], zc[u], vy, vz);
          done = u + 1;
        }
      }
    }
    if (rot) {
      // the hit at q + done enters another sector
      float xt = xh[0], yt = yc[0], zt = zc[0];
      int kt = kk[0];
#pragma unroll
      for (int u = 1; u < kMBlk; u++) {
        const bool m = u == done;
        xt = m ? xh[u] : xt;
        yt = m ? yc[u] : yt;
        zt = m ? zc[u] : zt;
        kt = m ? kk[u] : kt;
      }
      const bool up = (kt - kf + kPhi) % kPhi == 1;
      const float sa = up ? b.mp.sin_d : -b.mp.sin_d;
      if (!mtransport(s, x, b.mp.cos_d, sa, xt, yt, kB)) return false;
      kf = kt;
      chi2 = chi2 + kupdate(s, yt, zt, vy, vz);
      done++;
    }
    q += done;
  }
  return true;
}

__device__ __forceinline__ void mseed(const Consts& k, KSt& s, const MergeBufs& b, int64_t c,
                                      const float* p5)
{
  s.p[0] = b.y[c];
  s.p[1] = b.z[c];
  s.p[2] = p5[2];
  s.p[3] = p5[3];
  s.p[4] = p5[4];
  kinit_cov(s, k.vy, k.vz);
}

__device__ __forceinline__ void load_off(const MergeBufs& b, int64_t* s_off)
{
  for (int i = threadIdx.x; i <= kInst; i += blockDim.x) s_off[i] = b.inst_off[i];
  __syncthreads();
}

// Pair-search buckets.  The bin function is monotone (NaN goes to bin 0),
// so the bins between those of z - w and z + w hold every value within w
// of z.
__device__ __forceinline__ int merge_zbin(float z)
{
  const float f = floorf((z - kMergeZ0) * kMergeZInv);
  if (!(f >= 0.0f)) return 0;
  return f > (float)(kMergeZBins - 1) ? kMergeZBins - 1 : (int)f;
}

__device__ __forceinline__ int bucket_of(int inst, float z) { return inst * kMergeZBins + merge_zbin(z); }

// --------------------------------------------------------------- seg_info
__global__ __launch_bounds__(kBlock) void k_seg_info(Consts k, MergeBufs b)
{
  __shared__ int64_t s_off[kInst + 1];
  load_off(b, s_off);
  const int64_t n = *b.n_seg;
  const int64_t t = gid();
  if (t >= n) return;
  const int64_t a = b.seg.hit_off[t], e = b.seg.hit_off[t + 1];
  if (e <= a) {  // the tracker emits no empty track; kept safe all the same
    b.seg_inst[t] = 0;
    b.out_ok[t] = 0;
    for (int j = 0; j < 6; j++) b.seg_pos[t * 6 + j] = NAN;
    b.seg_key[t] = 0;
    b.seg_key[b.cap_seg + t] = 0;
    return;
  }
  const int64_t c0 = b.seg.hit_clu[a], c1 = b.seg.hit_clu[e - 1];
  const int inst = inst_of(s_off, c0);
  const int kk = inst % kPhi;
  b.seg_inst[t] = inst;
  // global positions of the first and last hit (pair pre-filter)
  const float x0 = k.row_x[b.row[c0]], x1 = k.row_x[b.row[c1]];
  const float ca = b.mp.cos_a[kk], sa = b.mp.sin_a[kk];
  b.seg_pos[t * 6 + 0] = x0 * ca - b.y[c0] * sa;
  b.seg_pos[t * 6 + 1] = x0 * sa + b.y[c0] * ca;
  b.seg_pos[t * 6 + 2] = b.z[c0];
  b.seg_pos[t * 6 + 3] = x1 * ca - b.y[c1] * sa;
  b.seg_pos[t * 6 + 4] = x1 * sa + b.y[c1] * ca;
  b.seg_pos[t * 6 + 5] = b.z[c1];
  // outer state: outward filter over the segment's own hits
  float p5[5];
#pragma unroll
  for (int j = 0; j < 5; j++) p5[j] = b.seg.param[t * 5 + j];
  KSt s;
  mseed(k, s, b, c0, p5);
  float x = x0, chi2 = 0.0f;
  int kf = kk;
  const float4* const hd = reinterpret_cast<const float4*>(b.seg.hit_data);
  const bool ok = hd ? mpass<true>(k, b, s_off, s, x, kf, nullptr, hd, a + 1, e - a - 1, 1, chi2)
                     : mpass<false>(k, b, s_off, s, x, kf, b.seg.hit_clu, nullptr, a + 1,
                                    e - a - 1, 1, chi2);
  b.out_ok[t] = ok ? 1 : 0;
#pragma unroll
  for (int j = 0; j < 5; j++) b.out_p[t * 5 + j] = ok ? s.p[j] : 0.0f;
#pragma unroll
  for (int j = 0; j < 15; j++) b.out_c[t * 15 + j] = ok ? s.c[j] : 0.0f;
  b.out_x[t] = x;  // the outer plane, or where the pass stopped
  b.seg_key[t] = bucket_of(inst, b.seg_pos[t * 6 + 2]);
  b.seg_key[b.cap_seg + t] = bucket_of(inst, b.seg_pos[t * 6 + 5]);
}

// --------------------------------------------------------------- buckets
__global__ __launch_bounds__(kBlock) void k_bkt_clear(MergeBufs b)
{
  for (int64_t i = gid(); i < 2 * kMergeBuckets; i += (int64_t)gridDim.x * blockDim.x)
    b.bkt_cur[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_bkt_count(MergeBufs b)
{
  const int64_t n = *b.n_seg;
  const int64_t t = gid();
  if (t >= n) return;
  atomicAdd(&b.bkt_cur[b.seg_key[t]], 1);
  atomicAdd(&b.bkt_cur[kMergeBuckets + b.seg_key[b.cap_seg + t]], 1);
}

// exclusive scans of both keys' counts in one block; the offsets are copied
// into the cursors of the scatter
__global__ __launch_bounds__(1024) void k_bkt_scan(MergeBufs b)
{
  __shared__ int s_w[16];
  for (int w = 0; w < 2; w++) {
    int* const cnt = b.bkt_cur + w * kMergeBuckets;
    int* const off = b.bkt_off + w * (kMergeBuckets + 1);
    int carry = 0;
    for (int i0 = 0; i0 < kMergeBuckets; i0 += 1024) {
      const int i = i0 + threadIdx.x;
      const int v = i < kMergeBuckets ? cnt[i] : 0;
      int x = v;
      const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      if (lane == 63) s_w[wid] = x;
      __syncthreads();
      int wofs = 0, tot = 0;
      for (int q = 0; q < 16; q++) {
        if (q < wid) wofs += s_w[q];
        tot += s_w[q];
      }
      if (i < kMergeBuckets) {
        off[i] = carry + wofs + x - v;
        cnt[i] = carry + wofs + x - v;
      }
      carry += tot;
      __syncthreads();
    }
    if (threadIdx.x == 0) off[kMergeBuckets] = carry;
  }
}

// a segment's place within its bucket comes from an atomic cursor: the
// order within a bucket is arbitrary, and the pair search does not depend
// on it
__global__ __launch_bounds__(kBlock) void k_bkt_scatter(MergeBufs b)
{
  const int64_t n = *b.n_seg;
  const int64_t t = gid();
  if (t >= n) return;
  const float ok = b.out_ok[t] ? 1.0f : 0.0f;
#pragma unroll
  for (int w = 0; w < 2; w++) {
    const int p = atomicAdd(&b.bkt_cur[w * kMergeBuckets + b.seg_key[w * b.cap_seg + t]], 1);
    b.bkt_order[w * b.cap_seg + p] = (int32_t)t;
    // what the pair search's cuts read, in bucket order next to the index:
    // the end (first hit for key 0, last hit for key 1) and the tgl and q/pt
    // terms of the state the pair compares there (the tracker's inner state
    // for key 0, the outer state for key 1)
    b.bkt_pos[w * b.cap_seg + p] = make_float4(b.seg_pos[t * 6 + 3 * w], b.seg_pos[t * 6 + 3 * w + 1],
                                               b.seg_pos[t * 6 + 3 * w + 2], ok);
    b.bkt_tq[w * b.cap_seg + p] =
        w == 0 ? make_float4(b.seg.param[t * 5 + 3], b.seg.param[t * 5 + 4], b.seg.cov[t * 15 + 9],
                             b.seg.cov[t * 15 + 14])
               : make_float4(b.out_p[t * 5 + 3], b.out_p[t * 5 + 4], b.out_c[t * 15 + 9],
                             b.out_c[t * 15 + 14]);
  }
}

// --------------------------------------------------------------- pairs
// R37's position cuts: A's last hit (pa) against B's first hit (pb)
__device__ __forceinline__ bool mpair_near(const MergeBufs& b, float4 pa, float4 pb)
{
  const float d0 = pa.x - pb.x;
  const float d1 = pa.y - pb.y;
  if (!(fabsf(pa.z - pb.z) <= b.mp.max_dz)) return false;
  return d0 * d0 + d1 * d1 <= b.mp.max_dist * b.mp.max_dist;
}

// A's tgl and q/pt, and their variances, leave the rotation and the
// propagation unchanged (copies, no arithmetic), so two terms of the pair's
// chi2 are known before the transport (ta: A's outer, tb: B's inner tgl,
// q/pt, var tgl, var q/pt): for the SPD sum S of the covariances,
// d^T S^-1 d >= d_i^2 / S_ii for every component i.  A pair whose larger
// such bound exceeds one and a half times the cut cannot pass it: the
// binary32 LDL^T solve errs by far less than a third (a Cholesky-type solve
// is accurate relative to the diagonal scaling, with an error set by the
// correlations, about 1e-4 at worst here), so skipping the transport leaves
// every decision as it is.
__device__ __forceinline__ bool mpair_bound(const MergeBufs& b, float4 ta, float4 tb)
{
  const float d3 = ta.x - tb.x;
  const float d4 = ta.y - tb.y;
  const float s33 = ta.z + tb.z;
  const float s44 = ta.w + tb.w;
  const float cut = 1.5f * b.mp.chi2_max;
  return !((s33 > 0.0f && (d3 * d3) / s33 > cut) || (s44 > 0.0f && (d4 * d4) / s44 > cut));
}

// R37: chi2 of A's outer state against B's inner state, -1 if no candidate.
// The caller has found A's outer state valid, B in one of the three
// instances A pairs with (nb: sector of B minus sector of A, modulo 18),
// the two ends within the position cuts and the pair within the bound.
__device__ __forceinline__ float mpair_fit(const Consts& k, const MergeBufs& b, int64_t A,
                                           int64_t B, int nb)
{
  const float kB = k.kB;
  KSt s;
#pragma unroll
  for (int j = 0; j < 5; j++) s.p[j] = b.out_p[A * 5 + j];
#pragma unroll
  for (int j = 0; j < 15; j++) s.c[j] = b.out_c[A * 15 + j];
  float x = b.out_x[A];
  const float xb = b.seg.x_ref[B];
  if (nb != 0) {
    const float sa = nb == 1 ? b.mp.sin_d : -b.mp.sin_d;
    if (!mtransport(s, x, b.mp.cos_d, sa, xb, b.seg.param[B * 5 + 0], kB)) return -1.0f;
  } else if (!mmove(s, x, xb, kB)) {
    return -1.0f;
  }
  float d[5], S[15];
#pragma unroll
  for (int j = 0; j < 5; j++) d[j] = s.p[j] - b.seg.param[B * 5 + j];
#pragma unroll
  for (int j = 0; j < 15; j++) S[j] = s.c[j] + b.seg.cov[B * 15 + j];
  const float chi2 = mchi2(S, d);
  if (!(chi2 >= 0.0f) || !(chi2 <= b.mp.chi2_max)) return -1.0f;
  return chi2;
}

// the three instances a segment of instance i pairs with: k - 1, k + 1 on
// its side, k on the other side
__device__ __forceinline__ int nbr_inst(int i, int which)
{
  const int kk = i % kPhi, side = i / kPhi;
  if (which == 0) return (kk + kPhi - 1) % kPhi + kPhi * side;
  if (which == 1) return (kk + 1) % kPhi + kPhi * side;
  return kk + kPhi * (1 - side);
}

// The pair search (R37, R38), one pass over the pairs: each segment A's
// best successor over the candidates B of the three neighbouring instances
// in the z bins within R37's z cut (plus a margin for rounding) of A's last
// hit, the pick being the smallest (chi2, index); every pair that passes
// also offers A as B's predecessor through a 64-bit atomic minimum of
// (chi2 bits, A), which is B's smallest (chi2, index) over the same pairs
// (the neighbour relation and the cuts are symmetric) in any order.
constexpr int kPairBlk = 4;  // candidates loaded at once

// Four lanes per segment: lane w < 3 scans the candidates of neighbouring
// instance w, and the group's picks are combined by the same order.
__global__ __launch_bounds__(kBlock) void k_best(Consts k, MergeBufs b)
{
  const int64_t n = *b.n_seg;
  const int64_t q = gid() >> 2;
  const int w = (int)(gid() & 3);
  if (q >= n) return;  // whole groups of four
  // groups in the bucket order of their own last hit (key 1), candidates
  // by their first hit (key 0)
  const int64_t me = b.bkt_order[b.cap_seg + q];
  const float4 mine = b.bkt_pos[b.cap_seg + q];
  const float4 mtq = b.bkt_tq[b.cap_seg + q];
  const int im = b.seg_inst[me];
  const float wz = b.mp.max_dz + 0.1f;
  const int zlo = merge_zbin(mine.z - wz), zhi = merge_zbin(mine.z + wz);
  const int32_t* const off = b.bkt_off;
  const int32_t* const ord = b.bkt_order;
  const float4* const pos = b.bkt_pos;
  const float4* const tqs = b.bkt_tq;
  int32_t best = -1;
  float bchi = 0.0f;
  // a segment without a valid outer state has no successor
  if (w < 3 && mine.w != 0.0f) {
    // the instance's bins zlo..zhi are one contiguous range of positions;
    // each candidate's end and tgl, q/pt terms are stored in bucket order
    // too, so the cuts take blocks of kPairBlk candidates with contiguous
    // loads, and only the candidates within them are fitted
    const int ic = nbr_inst(im, w);
    const int nb = ((ic % kPhi) - (im % kPhi) + kPhi) % kPhi;
    const int bb = ic * kMergeZBins;
    const int pa = off[bb + zlo], pe = off[bb + zhi + 1];
    for (int p0 = pa; p0 < pe; p0 += kPairBlk) {
      float4 pv[kPairBlk], tv[kPairBlk];
#pragma unroll
      for (int u = 0; u < kPairBlk; u++) {
        const int p = p0 + u < pe ? p0 + u : pe - 1;
        pv[u] = pos[p];
        tv[u] = tqs[p];
      }
      unsigned pass = 0;
#pragma unroll
      for (int u = 0; u < kPairBlk; u++) {
        const bool c = mpair_near(b, mine, pv[u]) && mpair_bound(b, mtq, tv[u]);
        if (p0 + u < pe && c) pass |= 1u << u;
      }
      // the fit, one copy of its code, for the candidates within the cuts
      while (pass) {
        const int u = __builtin_ctz(pass);
        pass &= pass - 1;
        const int32_t cand = ord[p0 + u];
        const float c2 = mpair_fit(k, b, me, cand, nb);
        if (c2 < 0.0f) continue;
        if (best < 0 || c2 < bchi || (c2 == bchi && cand < best)) {
          best = cand;
          bchi = c2;
        }
        // chi2 >= 0 here (-0 made +0), so its bits order like its value
        const float cz = c2 + 0.0f;
        atomicMin(&b.pred_key[cand],
                  ((unsigned long long)__float_as_uint(cz) << 32) | (unsigned long long)(uint32_t)me);
      }
    }
  }
  // the smallest (chi2, index) of the group
#pragma unroll
  for (int o = 1; o < 4; o <<= 1) {
    const int32_t ob = __shfl_xor(best, o, 64);
    const float oc = __shfl_xor(bchi, o, 64);
    if (ob >= 0 && (best < 0 || oc < bchi || (oc == bchi && ob < best))) {
      best = ob;
      bchi = oc;
    }
  }
  if (w == 0) b.succ[me] = best;
}

// --------------------------------------------------------------- links, chains
__global__ __launch_bounds__(kBlock) void k_link(MergeBufs b)
{
  const int64_t n = *b.n_seg;
  const int64_t a = gid();
  if (a >= n) return;
  const int32_t s = b.succ[a];
  // the predecessor of s is the segment in the low half of its key
  const bool keep = s >= 0 && b.pred_key[s] != ~0ull && (uint32_t)b.pred_key[s] == (uint32_t)a;
  b.out.next[a] = keep ? s : -1;
  if (keep) b.has_pred[s] = 1;
}

// Chain starts: item i < n is segment i as a head (no kept predecessor),
// item n + i is segment i as the lowest segment of a link cycle.  An item
// that starts a chain gets its segment and hit counts (both > 0), any
// other item zeros; chains are numbered in item order, so heads come in
// index order and then the cycles.
__device__ __forceinline__ void chain_item(const MergeBufs& b, int64_t n, int64_t i, int32_t& ns,
                                           int32_t& nh)
{
  ns = 0;
  nh = 0;
  if (i >= 2 * n) return;
  const int64_t t = i < n ? i : i - n;
  bool start;
  if (i < n) {
    start = b.has_pred[t] == 0;
  } else if (b.has_pred[t]) {
    // every segment has at most one predecessor, so a segment with one is
    // either on a head's chain (its successors end at -1) or on a link
    // cycle (they come back to it); the cycle's lowest segment starts it
    int64_t lowest = t, u = b.out.next[t];
    for (int64_t step = 0; step < n && u >= 0 && u != t; step++) {
      if (u < lowest) lowest = u;
      u = b.out.next[u];
    }
    start = u == t && lowest == t;
  } else {
    start = false;
  }
  if (!start) return;
  // at most n segments: the walk ends whatever next holds
  int64_t u = t;
  for (int64_t step = 0; step < n; step++) {
    ns++;
    nh += b.seg.hit_off[u + 1] - b.seg.hit_off[u];
    u = b.out.next[u];
    if (u < 0 || u == t) break;
  }
}

// exclusive scans of three values over the workgroup (kBlock threads)
__device__ __forceinline__ void block_scan3(const int64_t v[3], int64_t ex[3], int64_t tot[3])
{
  __shared__ int64_t s_w[3][kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t x[3];
#pragma unroll
  for (int q = 0; q < 3; q++) {
    x[q] = v[q];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(x[q], o, 64);
      if (lane >= o) x[q] += y;
    }
    if (lane == 63) s_w[q][wid] = x[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 3; q++) {
    int64_t wofs = 0, tt = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; w++) {
      if (w < wid) wofs += s_w[q][w];
      tt += s_w[q][w];
    }
    ex[q] = x[q] - v[q] + wofs;
    tot[q] = tt;
  }
  __syncthreads();
}

// pass 1: every item's counts, and each workgroup's sums (starts, segments, hits)
__global__ __launch_bounds__(kBlock) void k_chain_count(MergeBufs b)
{
  const int64_t n = *b.n_seg;
  const int64_t i = gid();
  int32_t ns, nh;
  chain_item(b, n, i, ns, nh);
  if (i < 2 * n) {
    b.it_ns[i] = ns;
    b.it_nh[i] = nh;
  }
  const int64_t v[3] = {ns > 0 ? 1 : 0, ns, nh};
  int64_t ex[3], tot[3];
  block_scan3(v, ex, tot);
  if (threadIdx.x < 3) b.ch_part[blockIdx.x * 3 + threadIdx.x] = tot[threadIdx.x];
}

// pass 2, one workgroup: exclusive scan of the workgroup sums; the totals
// close the offset arrays
__global__ __launch_bounds__(kBlock) void k_chain_partials(MergeBufs b, int64_t nblk)
{
  __shared__ int64_t s_carry[3];
  if (threadIdx.x < 3) s_carry[threadIdx.x] = 0;
  __syncthreads();
  // the workgroups past the call's 2 n items hold zero sums and write
  // nothing, so the scan stops at the last one that has items
  const int64_t nact = (2 * *b.n_seg + kBlock - 1) / kBlock;
  const int64_t nscan = nact < nblk ? nact : nblk;
  for (int64_t i0 = 0; i0 < nscan; i0 += kBlock) {
    const int64_t i = i0 + threadIdx.x;
    int64_t v[3];
#pragma unroll
    for (int q = 0; q < 3; q++) v[q] = i < nscan ? b.ch_part[i * 3 + q] : 0;
    int64_t ex[3], tot[3];
    block_scan3(v, ex, tot);
    if (i < nscan) {
#pragma unroll
      for (int q = 0; q < 3; q++) b.ch_part[i * 3 + q] = s_carry[q] + ex[q];
    }
    __syncthreads();
    if (threadIdx.x < 3) s_carry[threadIdx.x] += tot[threadIdx.x];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t m = s_carry[0];
    b.out.seg_off[m] = (int32_t)s_carry[1];
    b.out.hit_off[m] = (int32_t)s_carry[2];
    b.out.counts[0] = m;
    b.out.counts[1] = s_carry[2];
  }
}

// pass 3: chain heads and offsets in item order
__global__ __launch_bounds__(kBlock) void k_chain_write(MergeBufs b)
{
  const int64_t n = *b.n_seg;
  const int64_t i = gid();
  const int32_t ns = i < 2 * n ? b.it_ns[i] : 0;
  const int32_t nh = i < 2 * n ? b.it_nh[i] : 0;
  const int64_t v[3] = {ns > 0 ? 1 : 0, ns, nh};
  int64_t ex[3], tot[3];
  block_scan3(v, ex, tot);
  if (ns > 0) {
    const int64_t* const base = b.ch_part + blockIdx.x * 3;
    const int64_t m = base[0] + ex[0];
    b.chain_head[m] = (int32_t)(i < n ? i : i - n);
    b.out.seg_off[m] = (int32_t)(base[1] + ex[1]);
    b.out.hit_off[m] = (int32_t)(base[2] + ex[2]);
  }
}

// one wave per chain: its segment list (lane 0) and merged hit list (and
// hit data), each segment's hits copied by the wave's lanes together
// (coalesced)
__global__ __launch_bounds__(kBlock) void k_chain_hits(MergeBufs b)
{
  const int64_t m = gid() >> 6;
  const int lane = threadIdx.x & 63;
  if (m >= b.out.counts[0]) return;  // whole waves
  const int64_t n = *b.n_seg;
  int64_t so = b.out.seg_off[m], ho = b.out.hit_off[m];
  const int64_t se = b.out.seg_off[m + 1];
  int64_t u = b.chain_head[m];
  const float4* const hd = reinterpret_cast<const float4*>(b.seg.hit_data);
  // the segment count of the chain was fixed by k_chain_count
  while (so < se) {
    if (lane == 0) b.out.seg[so] = (int32_t)u;
    so++;
    const int64_t a = b.seg.hit_off[u], e = b.seg.hit_off[u + 1];
    for (int64_t h = a + lane; h < e; h += 64) b.out.hit_clu[ho + (h - a)] = b.seg.hit_clu[h];
    if (hd)  // the tracker's hit data, in merged order for the global refit
      for (int64_t h = a + lane; h < e; h += 64) b.hit_md[ho + (h - a)] = hd[h];
    ho += e - a;
    u = b.out.next[u];
    if (u < 0 || u >= n) break;
  }
}

// --------------------------------------------------------------- refit
__global__ __launch_bounds__(kBlock) void k_merge_refit(Consts k, MergeBufs b)
{
  __shared__ int64_t s_off[kInst + 1];
  load_off(b, s_off);
  const int64_t m = gid();
  if (m >= b.out.counts[0]) return;
  const int64_t a = b.out.hit_off[m], e = b.out.hit_off[m + 1];
  const int64_t t0 = b.out.seg[b.out.seg_off[m]];
  if (e <= a) {
    b.out.status[m] = 1;
    return;
  }
  const int32_t* hits = b.out.hit_clu;
  // with the tracker's hit data the passes read the merged hits' data as
  // the chain copy laid it out (contiguous, merged order)
  const float4* const hd = reinterpret_cast<const float4*>(b.seg.hit_data);
  KSt s;
  float x, chi2 = 0.0f;
  int kf = b.seg_inst[t0] % kPhi;
  bool good;
  const int64_t l0 = b.seg.hit_off[t0 + 1] - b.seg.hit_off[t0];
  if (l0 > 0) {
    // the merged hits start with the first segment's, so the outward pass
    // through them is the outer-state pass of the pair search (same seed,
    // hits and operations, no sector change within a segment): its state
    // is taken over and the pass goes on from the second segment
    good = b.out_ok[t0] != 0;
    x = b.out_x[t0];
    if (good) {
#pragma unroll
      for (int j = 0; j < 5; j++) s.p[j] = b.out_p[t0 * 5 + j];
#pragma unroll
      for (int j = 0; j < 15; j++) s.c[j] = b.out_c[t0 * 15 + j];
      if (hd) {
        good = mpass<true>(k, b, s_off, s, x, kf, nullptr, b.hit_md, a + l0, e - a - l0, 1, chi2);
      } else {
        good = mpass<false>(k, b, s_off, s, x, kf, hits, nullptr, a + l0, e - a - l0, 1, chi2);
      }
    }
  } else {
    float p5[5];
#pragma unroll
    for (int j = 0; j < 5; j++) p5[j] = b.seg.param[t0 * 5 + j];
    mseed(k, s, b, hits[a], p5);
    x = k.row_x[b.row[hits[a]]];
    good = mpass<false>(k, b, s_off, s, x, kf, hits, nullptr, a + 1, e - a - 1, 1, chi2);
  }
  if (good) {
#pragma unroll
    for (int j = 0; j < 15; j++) s.c[j] = s.c[j] * kInwardScale;
    chi2 = 0.0f;
    if (hd) {
      good = mpass<true>(k, b, s_off, s, x, kf, nullptr, b.hit_md, e - 1, e - a, -1, chi2);
    } else {
      good = mpass<false>(k, b, s_off, s, x, kf, hits, nullptr, e - 1, e - a, -1, chi2);
    }
  }
  b.out.status[m] = good ? 0 : 1;
#pragma unroll
  for (int j = 0; j < 5; j++) b.out.param[m * 5 + j] = good ? s.p[j] : 0.0f;
#pragma unroll
  for (int j = 0; j < 15; j++) b.out.cov[m * 15 + j] = good ? s.c[j] : 0.0f;
  b.out.chi2[m] = good ? chi2 : 0.0f;
  b.out.ndf[m] = (int32_t)(2 * (e - a) - 5);
  b.out.sector[m] = kf;
  b.out.x_ref[m] = x;
}

__global__ void k_merge_init(MergeBufs b)
{
  if (threadIdx.x == 0 && blockIdx.x == 0)
    *b.n_seg = b.res->n_tracks < b.cap_seg ? b.res->n_tracks : b.cap_seg;
}

__global__ __launch_bounds__(kBlock) void k_merge_clear(MergeBufs b)
{
  for (int64_t i = gid(); i < b.cap_seg; i += (int64_t)gridDim.x * blockDim.x) {
    b.has_pred[i] = 0;
    b.pred_key[i] = ~0ull;  // no predecessor
  }
}

}  // namespace

hipError_t merge_tracks(const Consts& k, const MergeBufs& b, hipStream_t s)
{
  const unsigned nb = (unsigned)((b.cap_seg + kBlock - 1) / kBlock);
  if (b.cap_seg <= 0) return hipGetLastError();
  int slot = prof_begin(s, "merge_init");
  k_merge_init<<<1, 1, 0, s>>>(b);
  prof_end(s, slot);
  slot = prof_begin(s, "merge_clear");
  k_merge_clear<<<nb < 1024u ? nb : 1024u, kBlock, 0, s>>>(b);
  prof_end(s, slot);
  slot = prof_begin(s, "merge_seg_info");
  k_seg_info<<<nb, kBlock, 0, s>>>(k, b);
  prof_end(s, slot);
  slot = prof_begin(s, "merge_buckets");
  k_bkt_clear<<<(2 * kMergeBuckets + kBlock - 1) / kBlock, kBlock, 0, s>>>(b);
  k_bkt_count<<<nb, kBlock, 0, s>>>(b);
  k_bkt_scan<<<1, 1024, 0, s>>>(b);
  k_bkt_scatter<<<nb, kBlock, 0, s>>>(b);
  prof_end(s, slot);
  const unsigned nb4 = (unsigned)((4 * b.cap_seg + kBlock - 1) / kBlock);
  slot = prof_begin(s, "merge_pairs");
  k_best<<<nb4, kBlock, 0, s>>>(k, b);
  prof_end(s, slot);
  slot = prof_begin(s, "merge_link");
  k_link<<<nb, kBlock, 0, s>>>(b);
  const int64_t nblk = (2 * b.cap_seg + kBlock - 1) / kBlock;
  k_chain_count<<<(unsigned)nblk, kBlock, 0, s>>>(b);
  k_chain_partials<<<1, kBlock, 0, s>>>(b, nblk);
  k_chain_write<<<(unsigned)nblk, kBlock, 0, s>>>(b);
  prof_end(s, slot);
  slot = prof_begin(s, "merge_chain_hits");
  k_chain_hits<<<(unsigned)((64 * b.cap_seg + kBlock - 1) / kBlock), kBlock, 0, s>>>(b);
  prof_end(s, slot);
  slot = prof_begin(s, "merge_refit");
  k_merge_refit<<<nb, kBlock, 0, s>>>(k, b);
  prof_end(s, slot);
  return hipGetLastError();
}

}  // namespace TPC_NS
}  // namespace tpcca
