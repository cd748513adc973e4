// HIP kernels of the sector tracker for gfx950 (CDNA4, wave64).
//
// This file is compiled twice: into namespace tpcca::det with
// -ffp-contract=off and correctly rounded division / square root (the
// deterministic mode's compile-time part, Sec. 2 of the paper), and into
// tpcca::prod with contraction and fast reciprocal allowed (production mode).
// TPC_DET also selects the run-time part: an ordering kernel after the grid's
// atomic scatter (per-bin sort by input index) and scan-ordered track
// compaction; the production build skips the sort and appends tracks with
// atomics.  Start hits are compacted in scan order in both builds.
//
// Every floating-point expression on the deterministic path is written in the
// operand order of the algorithm readings (R7-R11, R13-R20) so that, with
// contraction off, each operation rounds exactly as in the CPU reference.
#include <algorithm>
#include <climits>

#include "tpc_defaults.h"
#include "tpc_internal.h"

#ifndef TPC_NS
#error "TPC_NS must name the build (det or prod)"
#endif
#ifndef TPC_DET
#error "TPC_DET must be 0 or 1"
#endif

namespace tpcca {
namespace TPC_NS {

namespace {

constexpr int kItems = 8;                       // items per thread in scans
constexpr int kTile = kBlock * kItems;          // items per block in scans
constexpr int kStatItems = 1024;                // clusters per block in the row statistics

enum { CNT_START = 0, CNT_TRACKS = 1, CNT_CHUNKS = 2 };

// ------------------------------------------------------------------ helpers

// The constants a kernel reads: its arguments, or -- in the instantiation
// for the standard configuration -- the compile-time copy.
template <bool SPEC>
__device__ __forceinline__ const Consts& kconsts(const Consts& arg)
{
  if constexpr (SPEC) return kStdConsts;
  else return arg;
}

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }

// Workgroup w runs on XCD w % 8 (round-robin dispatch).  A launch of
// xcd_grid(nblk) workgroups that takes its block index from xcd_block gives
// each XCD one contiguous eighth of the nblk logical blocks, so that blocks
// working on neighbouring data share one L2; -1 for the padding workgroups
// (whole workgroups, so it is safe before a barrier).
__device__ __forceinline__ int64_t xcd_block(int64_t nblk)
{
  const int64_t per = (nblk + 7) / 8;
  const int64_t blk = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
  return blk < nblk ? blk : -1;
}

__device__ __forceinline__ int find_inst(const int64_t* off, int n_inst, int64_t c)
{
  int lo = 0, hi = n_inst;  // off[lo] <= c < off[hi]
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= c) lo = mid;
    else hi = mid;
  }
  return lo;
}

// order-preserving map of binary32 to uint32 (for atomic min / max)
__device__ __forceinline__ uint32_t f2o(float f)
{
  uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float o2f(uint32_t o)
{
  return __uint_as_float((o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o);
}

// R10: bin coordinate (monotone in q)
__device__ __forceinline__ int bin_coord(float q, float q0, float iw, int n)
{
  float f = (q - q0) * iw;
  if (!(f > 0.0f)) return 0;
  if (f >= (float)(n - 1)) return n - 1;
  return (int)f;
}

__device__ __forceinline__ int axis_bins(float d, float w)
{
  float t = ceilf(d / w);
  if (t < 1.0f) return 1;
  if (t > 65535.0f) return 65535;
  return (int)t;
}

__device__ __forceinline__ int64_t shfl_up64(int64_t v, int d)
{
  int lo = __shfl_up((int)(uint32_t)v, d, 64);
  int hi = __shfl_up((int)(v >> 32), d, 64);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Exclusive scan of one value per thread over a 256-thread block.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* total)
{
  __shared__ int64_t s_w[kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int64_t y = shfl_up64(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_w[wid] = x;
  __syncthreads();
  int64_t wofs = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; w++) {
    if (w < wid) wofs += s_w[w];
    tot += s_w[w];
  }
  __syncthreads();
  *total = tot;
  return x - v + wofs;
}

// ------------------------------------------------------------------ scans
// Exclusive in-place scan of data[0, n) with n = min(n_max, *n_dev): tile
// sums, one-block scan of the tile sums (total to *total_out), apply.

template <class T>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const T* data, int64_t n_max,
                                                        const int64_t* n_dev, int64_t* part)
{
  int64_t n = n_dev ? min(n_max, *n_dev) : n_max;
  int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; k++)
    if (base + k < n) s += (int64_t)data[base + k];
  int64_t tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_scan_partials(int64_t* part, int64_t nb, int64_t* total_out)
{
  __shared__ int64_t s_w[16];
  __shared__ int64_t s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
    int64_t i = b0 + threadIdx.x;
    int64_t v = i < nb ? part[i] : 0;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int64_t y = shfl_up64(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) s_w[wid] = x;
    __syncthreads();
    int64_t wofs = 0, tot = 0;
    for (int w = 0; w < 16; w++) {
      if (w < wid) wofs += s_w[w];
      tot += s_w[w];
    }
    int64_t carry = s_carry;
    if (i < nb) part[i] = carry + x - v + wofs;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total_out) *total_out = s_carry;
}

template <class T>
__global__ __launch_bounds__(kBlock) void k_scan_apply(T* data, int64_t n_max, const int64_t* n_dev,
                                                       const int64_t* part)
{
  int64_t n = n_dev ? min(n_max, *n_dev) : n_max;
  if ((int64_t)blockIdx.x * kTile >= n) return;
  int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
  T v[kItems];
  int64_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; k++) {
    v[k] = base + k < n ? data[base + k] : T(0);
    s += (int64_t)v[k];
  }
  int64_t tot;
  int64_t ex = block_exclusive_scan(s, &tot) + part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kItems; k++) {
    if (base + k < n) data[base + k] = (T)ex;
    ex += (int64_t)v[k];
  }
}

unsigned blocks_for(int64_t n, int per = kBlock)
{
  int64_t b = (n + per - 1) / per;
  return (unsigned)(b > 0 ? b : 1);
}

unsigned xcd_grid(int64_t nblk) { return (unsigned)(((nblk + 7) / 8) * 8); }

// Launch with optional event timing (tpc_profile_enable).
#define TPC_LAUNCH(name, grid, block, stream, kern, ...)   \
  do {                                                     \
    const int slot_ = prof_begin((stream), (name));        \
    kern<<<(grid), (block), 0, (stream)>>>(__VA_ARGS__);   \
    prof_end((stream), slot_);                             \
  } while (0)

template <class T>
void scan_exclusive(T* data, int64_t n_max, const int64_t* n_dev, int64_t* total_out,
                    int64_t* part, hipStream_t s)
{
  int64_t nb = (n_max + kTile - 1) / kTile;
  if (nb == 0) nb = 1;
  TPC_LAUNCH("scan_reduce", dim3((unsigned)nb), kBlock, s, k_scan_reduce<T>, data, n_max, n_dev, part);
  TPC_LAUNCH("scan_partials", 1, 1024, s, k_scan_partials, part, nb, total_out);
  TPC_LAUNCH("scan_apply", dim3((unsigned)nb), kBlock, s, k_scan_apply<T>, data, n_max, n_dev, part);
}


// ------------------------------------------------------------------ a1 grid

__global__ void k_grid_clear(GridBufs b)
{
  const int64_t n_seg = (int64_t)b.n_inst * kRows;
  for (int64_t s = gtid(); s < n_seg; s += (int64_t)gridDim.x * blockDim.x) {
    b.seg_cnt[s] = 0;
    b.seg_mm[s] = 0xFFFFFFFFu;
    b.seg_mm[n_seg + s] = 0u;
    b.seg_mm[2 * n_seg + s] = 0xFFFFFFFFu;
    b.seg_mm[3 * n_seg + s] = 0u;
    b.seg_cursor[s] = 0;
    if (s < b.n_inst) b.inst_bad[s] = 0;
  }
  if (gtid() == 0) {
    b.res->n_valid = 0;
    b.res->n_bad = 0;
    b.res->n_bins = 0;
    b.res->overflow = 0;
  }
}

// Row statistics: count and data box per (instance,row), validity of each
// cluster.  Blocks aggregate in LDS for the instance of their first cluster.
__global__ __launch_bounds__(kBlock) void k_grid_stats(Consts k, GridBufs b)
{
  __shared__ int s_cnt[kRows];
  __shared__ uint32_t s_mm[4][kRows];
  __shared__ int s_bad;
  __shared__ int s_inst;
  const int64_t n_seg = (int64_t)b.n_inst * kRows;
  const int64_t c0 = (int64_t)blockIdx.x * kStatItems;
  for (int r = threadIdx.x; r < kRows; r += blockDim.x) {
    s_cnt[r] = 0;
    s_mm[0][r] = 0xFFFFFFFFu;
    s_mm[1][r] = 0u;
    s_mm[2][r] = 0xFFFFFFFFu;
    s_mm[3][r] = 0u;
  }
  if (threadIdx.x == 0) {
    s_bad = 0;
    s_inst = find_inst(b.inst_off, b.n_inst, c0);
  }
  __syncthreads();
  const int i0 = s_inst;
  const int64_t end0 = b.inst_off[i0 + 1];
  // the rows and coordinates of this thread's clusters are loaded at once
  constexpr int kPer = kStatItems / kBlock;
  int rv[kPer];
  float yv[kPer], zv[kPer];
#pragma unroll
  for (int u = 0; u < kPer; u++) {
    const int64_t c = c0 + u * kBlock + threadIdx.x;
    rv[u] = c < b.n ? (int)b.row[c] : 0;
    yv[u] = c < b.n ? b.y[c] : 0.0f;
    zv[u] = c < b.n ? b.z[c] : 0.0f;
  }
#pragma unroll
  for (int u = 0; u < kPer; u++) {
    const int64_t c = c0 + u * kBlock + threadIdx.x;
    if (c >= b.n) break;
    int i = c < end0 ? i0 : find_inst(b.inst_off, b.n_inst, c);
    int row = rv[u];
    float y = yv[u], z = zv[u];
    bool ok = row < kRows;
    if (ok) {
      float lim = k.row_x[row] * k.tan_half + k.y_valid_margin;
      ok = fabsf(y) <= lim && fabsf(z) <= 1.0e5f;
    }
    if (!ok) {
      b.cseg[c] = -1;
      if (i == i0) atomicAdd(&s_bad, 1);
      else atomicAdd(&b.inst_bad[i], 1);
      continue;
    }
    int64_t seg = (int64_t)i * kRows + row;
    b.cseg[c] = (int32_t)seg;
    uint32_t oy = f2o(y), oz = f2o(z);
    if (i == i0) {
      atomicAdd(&s_cnt[row], 1);
      atomicMin(&s_mm[0][row], oy);
      atomicMax(&s_mm[1][row], oy);
      atomicMin(&s_mm[2][row], oz);
      atomicMax(&s_mm[3][row], oz);
    } else {
      atomicAdd(&b.seg_cnt[seg], 1);
      atomicMin(&b.seg_mm[seg], oy);
      atomicMax(&b.seg_mm[n_seg + seg], oy);
      atomicMin(&b.seg_mm[2 * n_seg + seg], oz);
      atomicMax(&b.seg_mm[3 * n_seg + seg], oz);
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < kRows; r += blockDim.x) {
    if (s_cnt[r] == 0) continue;
    int64_t seg = (int64_t)i0 * kRows + r;
    atomicAdd(&b.seg_cnt[seg], s_cnt[r]);
    atomicMin(&b.seg_mm[seg], s_mm[0][r]);
    atomicMax(&b.seg_mm[n_seg + seg], s_mm[1][r]);
    atomicMin(&b.seg_mm[2 * n_seg + seg], s_mm[2][r]);
    atomicMax(&b.seg_mm[3 * n_seg + seg], s_mm[3][r]);
  }
  if (threadIdx.x == 0 && s_bad) atomicAdd(&b.inst_bad[i0], s_bad);
}

// Grid dimensions of each (instance,row) from its data box (R10).
__global__ void k_grid_meta(Consts k, GridBufs b)
{
  const int64_t n_seg = (int64_t)b.n_inst * kRows;
  const int64_t s = gtid();
  if (s >= n_seg) return;
  int cnt = b.seg_cnt[s];
  int ny = 1, nz = 1;
  float y0 = 0.0f, z0 = 0.0f, iwy = 0.0f, iwz = 0.0f;
  if (cnt > 0) {
    // + 0.0f turns a -0 extreme into +0 (one canonical zero)
    float ymin = o2f(b.seg_mm[s]) + 0.0f, ymax = o2f(b.seg_mm[n_seg + s]) + 0.0f;
    float zmin = o2f(b.seg_mm[2 * n_seg + s]) + 0.0f, zmax = o2f(b.seg_mm[3 * n_seg + s]) + 0.0f;
    float dy = ymax - ymin, dz = zmax - zmin;
    float nb = floorf((float)cnt / k.grid_occupancy);
    if (nb < 1.0f) nb = 1.0f;
    float w = sqrtf((dy * dz) / nb);
    if (w < 1.0f) w = 1.0f;
    float m = (dy > dz ? dy : dz) / nb;
    if (w < m) w = m;
    ny = axis_bins(dy, w);
    nz = axis_bins(dz, w);
    iwy = dy > 0.0f ? (float)ny / dy : 0.0f;
    iwz = dz > 0.0f ? (float)nz / dz : 0.0f;
    y0 = ymin;
    z0 = zmin;
    atomicAdd((unsigned long long*)&b.res->n_valid, (unsigned long long)cnt);
  }
  tpc_row_meta mt;
  mt.ny = ny;
  mt.nz = nz;
  mt.bin_base = 0;
  mt.count = cnt;
  mt.y0 = y0;
  mt.z0 = z0;
  mt.iwy = iwy;
  mt.iwz = iwz;
  b.meta[s] = mt;
  b.nb1[s] = ny * nz + 1;
  if (s < b.n_inst)
    atomicAdd((unsigned long long*)&b.res->n_bad, (unsigned long long)b.inst_bad[s]);
}

// Bin bases, segment lengths (valid clusters, plus the instance's padding
// positions after its last row) and the bin-capacity check.
__global__ void k_grid_meta2(GridBufs b)
{
  const int64_t n_seg = (int64_t)b.n_inst * kRows;
  const int64_t s = gtid();
  if (s == 0 && b.res->n_bins > b.bin_cap) b.res->overflow |= 1;
  if (s >= n_seg) return;
  b.meta[s].bin_base = b.nb1[s];
  b.seg_pos[s] = b.seg_cnt[s] + (s % kRows == kRows - 1 ? b.inst_bad[s / kRows] : 0);
}

// Partition by segment: every valid cluster goes to its (instance,row)
// segment's range of a temporary array (in any order within the segment).
// A workgroup takes kPartItems consecutive clusters (mostly one instance),
// counts them per segment in LDS and claims each segment's run with one
// device atomic.  The clusters are then ordered by segment in LDS and
// written out from there, consecutive threads to consecutive slots of a
// run, so the stores coalesce although the input order is arbitrary.  A
// workgroup whose clusters span kPartSegs or more segment ids claims per
// cluster and writes directly.
constexpr int kPartPer = 8;                        // clusters per thread
constexpr int kPartItems = kBlock * kPartPer;
constexpr int kPartSegs = 2048;

__global__ __launch_bounds__(kBlock) void k_grid_part(GridBufs b)
{
  __shared__ int s_cnt[kPartSegs];   // per segment: count, then tile offset
  __shared__ int s_dst[kPartSegs];   // per segment: destination of tile slot 0
  __shared__ int32_t s_idx[kPartItems];
  __shared__ float2 s_q[kPartItems];
  __shared__ uint16_t s_seg[kPartItems];
  __shared__ int s_smin, s_smax;
  const int tx = threadIdx.x;
  // contiguous eighths per XCD: an instance's segment runs fill in one L2
  const int64_t blk = xcd_block((b.n + kPartItems - 1) / kPartItems);
  if (blk < 0) return;
  const int64_t c0 = blk * kPartItems;
  if (tx == 0) {
    s_smin = INT_MAX;
    s_smax = -1;
  }
  int seg[kPartPer], rank[kPartPer];
  float2 q[kPartPer];
  int lmin = INT_MAX, lmax = -1;
#pragma unroll
  for (int k = 0; k < kPartPer; k++) {
    const int64_t c = c0 + k * kBlock + tx;
    seg[k] = c < b.n ? b.cseg[c] : -1;
    q[k] = c < b.n ? make_float2(b.y[c], b.z[c]) : make_float2(0.0f, 0.0f);
    if (seg[k] >= 0) {
      lmin = min(lmin, seg[k]);
      lmax = max(lmax, seg[k]);
    }
  }
  __syncthreads();
  if (lmax >= 0) {
    atomicMin(&s_smin, lmin);
    atomicMax(&s_smax, lmax);
  }
  __syncthreads();
  const int smin = s_smin, smax = s_smax;
  if (smax < 0) return;  // no valid cluster here (uniform)
  if (smax - smin >= kPartSegs) {
#pragma unroll
    for (int k = 0; k < kPartPer; k++) {
      if (seg[k] < 0) continue;
      const int32_t dst = b.seg_pos[seg[k]] + atomicAdd(&b.seg_cursor[seg[k]], 1);
      b.tmp_perm[dst] = (int32_t)(c0 + k * kBlock + tx);
      b.tmp_yz[dst] = q[k];
    }
    return;
  }
  const int ns = smax - smin + 1;
  for (int j = tx; j < ns; j += kBlock) s_cnt[j] = 0;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPartPer; k++)
    if (seg[k] >= 0) rank[k] = atomicAdd(&s_cnt[seg[k] - smin], 1);
  __syncthreads();
  // tile offsets (exclusive scan of the counts) and each run's claim
  int64_t carry = 0;
  for (int j0 = 0; j0 < ns; j0 += kBlock) {
    const int j = j0 + tx;
    const int n = j < ns ? s_cnt[j] : 0;
    int64_t tot;
    const int off = (int)(carry + block_exclusive_scan(n, &tot));
    if (j < ns) {
      s_cnt[j] = off;
      if (n) s_dst[j] = b.seg_pos[smin + j] + atomicAdd(&b.seg_cursor[smin + j], n) - off;
    }
    carry += tot;
  }
  const int nv = (int)carry;
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPartPer; k++) {
    if (seg[k] < 0) continue;
    const int slot = s_cnt[seg[k] - smin] + rank[k];
    s_idx[slot] = (int32_t)(c0 + k * kBlock + tx);
    s_q[slot] = q[k];
    s_seg[slot] = (uint16_t)(seg[k] - smin);
  }
  __syncthreads();
  for (int i = tx; i < nv; i += kBlock) {
    const int32_t dst = s_dst[s_seg[i]] + i;
    b.tmp_perm[dst] = s_idx[i];
    b.tmp_yz[dst] = s_q[i];
  }
}

// Counting sort of one segment by bin (R10), one workgroup per segment: the
// workgroup owns the segment's positions and bins, so its bin counters live
// in LDS (or, for more than kSegBinsBig bins, in the segment's own range of
// the workspace counters) with no other writer.  Histogram, exclusive scan
// (written as the bins' first positions, sentinel included), placement with
// the scanned counters as cursors, and in the deterministic build the
// ordering of each bin by input index -- an ordering kernel after atomic
// placement (Sec. 2, run-time part), here inside the workgroup.
//
// Two instantiations split the segments by bin count: up to kSegBins bins
// with 16 KB of LDS (ten workgroups per CU), more with 48 KB (the rows of
// a whole time frame in one sector hold several thousand clusters).
constexpr int kSegBins = 4096;
constexpr int kSegBinsBig = 12288;
constexpr int kSegBatch = 4;
constexpr int kSortReg = 8;

template <int NB>
__global__ __launch_bounds__(kBlock) void k_grid_seg(GridBufs b)
{
  __shared__ int32_t s_c[NB];
  if (b.res->overflow & 1) return;
  const int64_t s = blockIdx.x;
  const int tx = threadIdx.x;
  const tpc_row_meta m = b.meta[s];
  const int nb = m.ny * m.nz;
  // the small instantiation takes the segments whose bins fit its LDS, the
  // big one all others
  if ((nb + 1 <= kSegBins) != (NB == kSegBins)) return;
  const int cnt = b.seg_cnt[s];
  const int32_t P = b.seg_pos[s];
  const bool lds = nb + 1 <= NB;
  int32_t* const gc = b.fill + m.bin_base;
  for (int j = tx; j <= nb; j += kBlock) {
    if (lds) s_c[j] = 0;
    else gc[j] = 0;
  }
  __syncthreads();
  for (int j0 = tx; j0 < cnt; j0 += kBlock * kSegBatch) {
    float2 qv[kSegBatch];
#pragma unroll
    for (int u = 0; u < kSegBatch; u++) {
      const int j = j0 + u * kBlock;
      qv[u] = j < cnt ? b.tmp_yz[P + j] : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int u = 0; u < kSegBatch; u++) {
      if (j0 + u * kBlock >= cnt) continue;
      const int bin = bin_coord(qv[u].y, m.z0, m.iwz, m.nz) * m.ny + bin_coord(qv[u].x, m.y0, m.iwy, m.ny);
      if (lds) atomicAdd(&s_c[bin], 1);
      else atomicAdd(&gc[bin], 1);
    }
  }
  __syncthreads();
  int64_t carry = 0;
  for (int j0 = 0; j0 <= nb; j0 += kBlock) {
    const int j = j0 + tx;
    const int v = j <= nb ? (lds ? s_c[j] : atomicAdd(&gc[j], 0)) : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan(v, &tot);
    if (j <= nb) {
      const int off = (int)(carry + ex);
      b.bin_off[m.bin_base + j] = P + off;
      if (lds) s_c[j] = off;
      else atomicExch(&gc[j], off);
    }
    carry += tot;
  }
  __syncthreads();
  for (int j0 = tx; j0 < cnt; j0 += kBlock * kSegBatch) {
    int32_t cv[kSegBatch];
    float2 qv[kSegBatch];
#pragma unroll
    for (int u = 0; u < kSegBatch; u++) {
      const int j = j0 + u * kBlock;
      cv[u] = j < cnt ? b.tmp_perm[P + j] : 0;
      qv[u] = j < cnt ? b.tmp_yz[P + j] : make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int u = 0; u < kSegBatch; u++) {
      if (j0 + u * kBlock >= cnt) continue;
      const float2 q = qv[u];
      const int bin = bin_coord(q.y, m.z0, m.iwz, m.nz) * m.ny + bin_coord(q.x, m.y0, m.iwy, m.ny);
      const int pos = P + (lds ? atomicAdd(&s_c[bin], 1) : atomicAdd(&gc[bin], 1));
      b.perm[pos] = cv[u];
      b.yz[pos] = q;
      b.sseg[pos] = (int32_t)s;
    }
  }
#if TPC_DET
  __syncthreads();
  // the cursors now hold each bin's end; bin j starts where bin j-1 ends.
  // A bin of at most kSortReg entries is loaded into registers at once and
  // sorted there (odd-even transposition network); longer bins are sorted
  // in place.  Input indices are distinct, so the order is unique.
  for (int j = tx; j < nb; j += kBlock) {
    const int e = lds ? s_c[j] : atomicAdd(&gc[j], 0);
    const int a = j == 0 ? 0 : (lds ? s_c[j - 1] : atomicAdd(&gc[j - 1], 0));
    const int len = e - a;
    if (len < 2) continue;
    if (len <= kSortReg) {
      int32_t kp[kSortReg];
      float2 kv[kSortReg];
#pragma unroll
      for (int u = 0; u < kSortReg; u++) {
        kp[u] = u < len ? b.perm[P + a + u] : INT_MAX;
        kv[u] = u < len ? b.yz[P + a + u] : make_float2(0.0f, 0.0f);
      }
#pragma unroll
      for (int pass = 0; pass < kSortReg; pass++) {
#pragma unroll
        for (int u = pass & 1; u + 1 < kSortReg; u += 2) {
          if (kp[u] > kp[u + 1]) {
            const int32_t ti = kp[u];
            kp[u] = kp[u + 1];
            kp[u + 1] = ti;
            const float2 tq = kv[u];
            kv[u] = kv[u + 1];
            kv[u + 1] = tq;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kSortReg; u++) {
        if (u < len) {
          b.perm[P + a + u] = kp[u];
          b.yz[P + a + u] = kv[u];
        }
      }
      continue;
    }
    for (int p = P + a + 1; p < P + e; p++) {
      const int32_t kp = b.perm[p];
      const float2 kv = b.yz[p];
      int q = p - 1;
      while (q >= P + a && b.perm[q] > kp) {
        b.perm[q + 1] = b.perm[q];
        b.yz[q + 1] = b.yz[q];
        q--;
      }
      b.perm[q + 1] = kp;
      b.yz[q + 1] = kv;
    }
  }
#endif
}

__global__ void k_grid_rowoff(GridBufs b)
{
  if (b.res->overflow & 1) return;
  const int64_t n_seg = (int64_t)b.n_inst * kRows;
  const int64_t s = gtid();
  if (s >= n_seg) return;
  const int64_t i = s / kRows;
  const int r = (int)(s % kRows);
  b.row_off[i * (kRows + 1) + r] = b.seg_pos[s];
  if (r == kRows - 1) {
    const int end = b.seg_pos[s] + b.seg_cnt[s];
    b.row_off[i * (kRows + 1) + kRows] = end;
    for (int64_t p = end; p < b.inst_off[i + 1]; p++) {
      b.sseg[p] = -1;
      b.perm[p] = -1;
      b.yz[p] = make_float2(0.0f, 0.0f);
    }
  }
}

// ------------------------------------------------------------------ a2..a4

__global__ void k_track_init(TrackBufs b)
{
  if (gtid() == 0) {
    b.res->n_start = 0;
    b.res->n_tracklets_kept = 0;
    b.res->n_tracks = 0;
    b.res->n_hits = 0;
    b.res->need_tracklets = 0;
    b.res->need_tracks = 0;
    b.res->need_hits = 0;
    b.res->overflow &= 1;
    for (int i = 0; i < 8; i++) b.counters[i] = 0;
    if (b.out.hit_off) b.out.hit_off[0] = 0;
  }
}

// NeighboursFinder (R11): best (u on r+1, d on r-1) straight-line pair, one
// thread per position.  Positions are in (segment, z bin, y bin) order, so
// the threads of a wave search neighbouring windows of the same two rows
// and read them from the cache; staging the rows' reachable slabs in LDS
// first (with a workgroup loop over its segments) measured slower.  The
// pair choice is a total order (score, then the input indices of u and d),
// so the visit order does not change the result; input indices are read
// only on an exact tie.
struct NfBest {
  int32_t u = -1, d = -1;
  float s = 0.0f;
};

__device__ __forceinline__ void nf_consider(const TrackBufs& b, NfBest& best, float sc, int32_t u,
                                            int32_t d)
{
  if (best.u < 0 || sc < best.s) {
    best.u = u;
    best.d = d;
    best.s = sc;
  } else if (sc == best.s) {
    const int32_t pu = b.perm[u], pd = b.perm[d];
    const int32_t bu = b.perm[best.u], bd = b.perm[best.d];
    if (pu < bu || (pu == bu && pd < bd)) {
      best.u = u;
      best.d = d;
    }
  }
}

// The pair search of cluster (yh, zh) of row r over the windows of rows
// r+1 (mu, bin boundaries offu) and r-1 (md, offd), nested loops over the
// two windows (the fallback for windows longer than the lists below).
__device__ __forceinline__ void nf_search(const Consts& k, const TrackBufs& b, NfBest& best,
                                          float yh, float zh, float t, const tpc_row_meta& mu,
                                          const int32_t* offu, const tpc_row_meta& md,
                                          const int32_t* offd)
{
  const float wy = k.nf_win_y, wz = k.nf_win_z;
  const float wym = wy + k.search_margin, wzm = wz + k.search_margin;
  const float cmax = k.nf_chi2_max, ivy = k.ivy, ivz = k.ivz;
  const int uylo = bin_coord(yh - wym, mu.y0, mu.iwy, mu.ny);
  const int uyhi = bin_coord(yh + wym, mu.y0, mu.iwy, mu.ny);
  const int uzlo = bin_coord(zh - wzm, mu.z0, mu.iwz, mu.nz);
  const int uzhi = bin_coord(zh + wzm, mu.z0, mu.iwz, mu.nz);
  const int dylo = bin_coord(yh - wym, md.y0, md.iwy, md.ny);
  const int dyhi = bin_coord(yh + wym, md.y0, md.iwy, md.ny);
  const int dzlo = bin_coord(zh - wzm, md.z0, md.iwz, md.nz);
  const int dzhi = bin_coord(zh + wzm, md.z0, md.iwz, md.nz);
  for (int izu = uzlo; izu <= uzhi; izu++) {
    const int ub = izu * mu.ny;
    const int ue = offu[ub + uyhi + 1];
    for (int u = offu[ub + uylo]; u < ue; u++) {
      const float2 qu = b.yz[u];
      const float yu = qu.x, zu = qu.y;
      if (!(fabsf(yu - yh) <= wy && fabsf(zu - zh) <= wz)) continue;
      for (int izd = dzlo; izd <= dzhi; izd++) {
        const int db = izd * md.ny;
        const int de = offd[db + dyhi + 1];
        for (int d = offd[db + dylo]; d < de; d++) {
          const float2 qd = b.yz[d];
          const float yd = qd.x, zd = qd.y;
          if (!(fabsf(yd - yh) <= wy && fabsf(zd - zh) <= wz)) continue;
          const float ey = yh - (yd + (yu - yd) * t);
          const float ez = zh - (zd + (zu - zd) * t);
          const float sc = (ey * ey) * ivy + (ez * ez) * ivz;
          if (sc <= cmax) nf_consider(b, best, sc, u, d);
        }
      }
    }
  }
}

// List search: each window is scanned once into a per-thread list of
// row-relative indices (thread-major in LDS; rows of fewer than 65536
// positions), the down window first so that a cluster without a down
// candidate skips the up window.  The pairs are then evaluated with the
// down candidates loaded in batches into registers.  Windows with more than
// kNfList candidates fall back to nf_search.  yzu = yz + Pu and yzd = yz + Pd
// are the two rows' positions.
constexpr int kNfList = 32;
constexpr int kNfBatch = 8;

// One window scan into a per-thread list: the bin ranges of kNfZ z rows are
// loaded at once, then kNfC candidates at once, so a window costs a few
// memory latencies instead of one per z row and candidate.
constexpr int kNfZ = 2, kNfC = 8;

__device__ __forceinline__ int nf_window(const tpc_row_meta& m, const int32_t* off,
                                         const float2* yz, int32_t P, float yh, float zh,
                                         float wy, float wz, float wym, float wzm,
                                         uint16_t (*list)[kBlock])
{
  const int tx = threadIdx.x;
  const int ylo = bin_coord(yh - wym, m.y0, m.iwy, m.ny);
  const int yhi = bin_coord(yh + wym, m.y0, m.iwy, m.ny);
  const int zlo = bin_coord(zh - wzm, m.z0, m.iwz, m.nz);
  const int zhi = bin_coord(zh + wzm, m.z0, m.iwz, m.nz);
  int n = 0;
  for (int z0 = zlo; z0 <= zhi; z0 += kNfZ) {
    int ra[kNfZ], re[kNfZ];
#pragma unroll
    for (int u = 0; u < kNfZ; u++) {
      ra[u] = re[u] = 0;
      if (z0 + u <= zhi) {
        const int bb = (z0 + u) * m.ny;
        ra[u] = off[bb + ylo] - P;
        re[u] = off[bb + yhi + 1] - P;
      }
    }
#pragma unroll
    for (int u = 0; u < kNfZ; u++) {
      for (int p0 = ra[u]; p0 < re[u]; p0 += kNfC) {
        float2 qv[kNfC];
#pragma unroll
        for (int c = 0; c < kNfC; c++)
          qv[c] = p0 + c < re[u] ? yz[p0 + c] : make_float2(0.0f, 0.0f);
#pragma unroll
        for (int c = 0; c < kNfC; c++) {
          if (p0 + c >= re[u]) continue;
          if (!(fabsf(qv[c].x - yh) <= wy && fabsf(qv[c].y - zh) <= wz)) continue;
          if (n < kNfList) list[n][tx] = (uint16_t)(p0 + c);
          n++;
        }
      }
    }
  }
  return n;
}

// The list search of cluster (yh, zh) of row r (see above).
__device__ __forceinline__ void nf_search_lists(const Consts& k, const TrackBufs& b, NfBest& best,
                                                float yh, float zh, float t,
                                                const tpc_row_meta& mu, const int32_t* offu,
                                                int32_t Pu, const tpc_row_meta& md,
                                                const int32_t* offd, int32_t Pd,
                                                uint16_t (*s_ul)[kBlock], uint16_t (*s_dl)[kBlock])
{
  const int tx = threadIdx.x;
  const float2* const yzu = b.yz + Pu;
  const float2* const yzd = b.yz + Pd;
  const float wy = k.nf_win_y, wz = k.nf_win_z;
  const float wym = wy + k.search_margin, wzm = wz + k.search_margin;
  const float cmax = k.nf_chi2_max, ivy = k.ivy, ivz = k.ivz;
  const int nd = nf_window(md, offd, yzd, Pd, yh, zh, wy, wz, wym, wzm, s_dl);
  if (nd == 0) return;
  const int nu = nf_window(mu, offu, yzu, Pu, yh, zh, wy, wz, wym, wzm, s_ul);
  if (nu == 0) return;
  if (nu > kNfList || nd > kNfList) {
    nf_search(k, b, best, yh, zh, t, mu, offu, md, offd);
    return;
  }
  // down candidates in register batches of kNfBatch (static indices,
  // unrolled), each up candidate against a whole batch: no LDS load per pair
  for (int j0 = 0; j0 < nd; j0 += kNfBatch) {
    float by[kNfBatch], bz[kNfBatch];
    int bi[kNfBatch];
#pragma unroll
    for (int j = 0; j < kNfBatch; j++) {
      const int d = s_dl[j0 + j < nd ? j0 + j : j0][tx];
      const float2 q = yzd[d];
      by[j] = q.x;
      bz[j] = q.y;
      bi[j] = d;
    }
    const int nb = min(nd - j0, kNfBatch);
    // the next up candidate is loaded while the current one is scored
    int un = s_ul[0][tx];
    float2 qn = yzu[un];
    for (int iu = 0; iu < nu; iu++) {
      const int u = un;
      const float yu = qn.x, zu = qn.y;
      if (iu + 1 < nu) {
        un = s_ul[iu + 1][tx];
        qn = yzu[un];
      }
      // the batch's scores, then one candidate per batch: its smallest
      // score (slots beyond the list score +inf); the rare exact tie of two
      // down candidates goes through the pair order one by one
      float sc[kNfBatch];
      float m = INFINITY;
#pragma unroll
      for (int j = 0; j < kNfBatch; j++) {
        const float yd = by[j], zd = bz[j];
        const float ey = yh - (yd + (yu - yd) * t);
        const float ez = zh - (zd + (zu - zd) * t);
        sc[j] = j < nb ? (ey * ey) * ivy + (ez * ez) * ivz : INFINITY;
        m = fminf(m, sc[j]);
      }
      // nothing here can beat the running best (scores only decrease)
      if (!(m <= cmax) || (best.u >= 0 && m > best.s)) continue;
      int db = 0, ne = 0;
#pragma unroll
      for (int j = kNfBatch - 1; j >= 0; j--) {
        const bool e = sc[j] == m;
        db = e ? bi[j] : db;
        ne += e ? 1 : 0;
      }
      if (ne == 1) {
        nf_consider(b, best, m, Pu + u, Pd + db);
      } else {
#pragma unroll
        for (int j = 0; j < kNfBatch; j++)
          if (sc[j] == m) nf_consider(b, best, m, Pu + u, Pd + bi[j]);
      }
    }
  }
}

template <bool SPEC>
__global__ __launch_bounds__(kBlock) void k_neighbours(Consts karg, TrackBufs b)
{
  const Consts& k = kconsts<SPEC>(karg);
  __shared__ uint16_t s_ul[kNfList][kBlock];
  __shared__ uint16_t s_dl[kNfList][kBlock];
  // contiguous eighths per XCD: neighbouring positions search the same rows
  const int64_t blk = xcd_block((b.n + kBlock - 1) / kBlock);
  if (blk < 0) return;
  const int64_t h = blk * kBlock + threadIdx.x;
  if (h >= b.n) return;
  const int seg = b.sseg[h];
  const int r = seg >= 0 ? seg % kRows : 0;
  NfBest best;
  // no pair on the first and last row
  if (seg >= 0 && r > 0 && r < kRows - 1) {
    const float2 qh = b.yz[h];
    const tpc_row_meta mu = b.meta[seg + 1];
    const tpc_row_meta md = b.meta[seg - 1];
    const float xm = k.row_x[r - 1], x0 = k.row_x[r], xp = k.row_x[r + 1];
    const float t = (x0 - xm) / (xp - xm);
    const int32_t* const offu = b.bin_off + mu.bin_base;
    const int32_t* const offd = b.bin_off + md.bin_base;
    const int32_t Pu = offu[0], Pd = offd[0];
    if (offu[mu.ny * mu.nz] - Pu < 65536 && offd[md.ny * md.nz] - Pd < 65536)
      nf_search_lists(k, b, best, qh.x, qh.y, t, mu, offu, Pu, md, offd, Pd, s_ul, s_dl);
    else
      nf_search(k, b, best, qh.x, qh.y, t, mu, offu, md, offd);
  }
  b.up[h] = best.u;
  b.dn[h] = best.d;
}

// NeighboursCleaner: mutual links only (reads the uncleaned arrays).
__global__ __launch_bounds__(kBlock) void k_clean(TrackBufs b)
{
  const int64_t blk = xcd_block((b.n + kBlock - 1) / kBlock);
  if (blk < 0) return;
  const int64_t h = blk * kBlock + threadIdx.x;
  if (h >= b.n) return;
  int32_t u = b.up[h], d = b.dn[h];
  b.up2[h] = (u >= 0 && b.dn[u] == (int32_t)h) ? u : -1;
  b.dn2[h] = (d >= 0 && b.up[d] == (int32_t)h) ? d : -1;
}

__device__ __forceinline__ bool is_start(const TrackBufs& b, int min_chain, int64_t h)
{
  if (h >= b.n) return false;
  if (b.dn2[h] != -1) return false;
  int32_t q = b.up2[h];
  if (q < 0) return false;
  int len = 2;
  while (len < min_chain) {
    q = b.up2[q];
    if (q < 0) return false;
    len++;
  }
  return true;
}

// StartHitsFinder, deterministic: tile counts, scan, ordered write.  The
// count pass keeps each thread's eight flags (one byte each) for the write
// pass, so the chains are walked once.
template <bool SPEC>
__global__ __launch_bounds__(kBlock) void k_start_count(Consts karg, TrackBufs b, int64_t* part)
{
  const Consts& k = kconsts<SPEC>(karg);
  const int64_t blk = xcd_block((b.n + kTile - 1) / kTile);
  if (blk < 0) return;
  const int64_t tid = blk * kBlock + threadIdx.x;
  const int64_t base = tid * kItems;
  int64_t s = 0;
  unsigned long long fl = 0ull;
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    const bool f = is_start(b, k.min_chain, base + j);
    s += f ? 1 : 0;
    fl |= (unsigned long long)(f ? 1u : 0u) << (8 * j);
  }
  b.start_flag[tid] = fl;
  int64_t tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) part[blk] = tot;
}

__global__ __launch_bounds__(kBlock) void k_start_write(TrackBufs b, const int64_t* part)
{
  const int64_t blk = xcd_block((b.n + kTile - 1) / kTile);
  if (blk < 0) return;
  const int64_t tid = blk * kBlock + threadIdx.x;
  const int64_t base = tid * kItems;
  const unsigned long long fl = b.start_flag[tid];
  const int64_t s = __popcll(fl);
  int64_t tot;
  int64_t o = block_exclusive_scan(s, &tot) + part[blk];
#pragma unroll
  for (int j = 0; j < kItems; j++) {
    if ((fl >> (8 * j)) & 1ull) {
      if (o < b.cap) b.start[o] = (int32_t)(base + j);
      o++;
    }
  }
}

__global__ void k_start_finish(TrackBufs b)
{
  int64_t S = b.counters[CNT_START];
  b.res->n_start = S;
  b.res->need_tracklets = S;
  if (S > b.cap) b.res->overflow |= 2;
}

// ------------------------------------------------------------------ a5 tracklets

#include "tpc_kalman.h"

constexpr int kSrchZ = 4, kSrchC = 4;
// R16: rows per propagation step of the walk back to the start row
constexpr int kWalkRows = 8;

// R15: best grid position of row segment m for the predicted state, or -1.
// The pick is a total order -- smallest chi2, then smallest input index --
// so the scan order does not matter; the input index is read only on an
// exact tie.  bq receives the picked position (left alone if none).
template <bool COUNT>
__device__ __forceinline__ int32_t ksearch(const Consts& k, const TrackBufs& b,
                                           const tpc_row_meta& m, const KSt& st,
                                           const Innov& q, int& ncand, float2& bq)
{
  const int32_t* const off = b.bin_off + m.bin_base;  // the segment's bin boundaries
  const float2* const yz = b.yz;
  const float y = st.p[0], z = st.p[1];
  const float pick = k.tc_chi2_pick;
  const float wy = sqrtf(pick * q.S00) + k.search_margin;
  const float wz = sqrtf(pick * q.S11) + k.search_margin;
  const int ylo = bin_coord(y - wy, m.y0, m.iwy, m.ny);
  const int yhi = bin_coord(y + wy, m.y0, m.iwy, m.ny);
  const int zlo = bin_coord(z - wz, m.z0, m.iwz, m.nz);
  const int zhi = bin_coord(z + wz, m.z0, m.iwz, m.nz);
  int32_t best = -1;
  float bchi = 0.0f;
  // loads batched: the bin ranges of kSrchZ z rows at once, then up to
  // kSrchC candidates of a range at once (one memory latency each instead of
  // one per load)
  for (int z0 = zlo; z0 <= zhi; z0 += kSrchZ) {
    int ra[kSrchZ], re[kSrchZ];
#pragma unroll
    for (int u = 0; u < kSrchZ; u++) {
      ra[u] = re[u] = 0;
      if (z0 + u <= zhi) {
        const int bb = (z0 + u) * m.ny;
        ra[u] = off[bb + ylo];
        re[u] = off[bb + yhi + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < kSrchZ; u++) {
      for (int p0 = ra[u]; p0 < re[u]; p0 += kSrchC) {
        float2 qv[kSrchC];
#pragma unroll
        for (int c = 0; c < kSrchC; c++)
          qv[c] = p0 + c < re[u] ? yz[p0 + c] : make_float2(0.0f, 0.0f);
#pragma unroll
        for (int c = 0; c < kSrchC; c++) {
          const int p = p0 + c;
          if (p >= re[u]) continue;
          const float r0 = qv[c].x - y, r1 = qv[c].y - z;
          // instrumentation only: the candidates inside the window box, the
          // ones any implementation of the search has to examine
          if constexpr (COUNT) ncand += (fabsf(r0) <= wy) & (fabsf(r1) <= wz);
          const float ch = chi2_of(q, r0, r1);
          if (!(ch <= pick)) continue;
          if (best < 0 || ch < bchi) {
            best = p;
            bchi = ch;
            bq = qv[c];
          } else if (ch == bchi && b.perm[p] < b.perm[best]) {
            best = p;
            bq = qv[c];
          }
        }
      }
    }
  }
  return best;
}

// Selection key of a kept tracklet (R20): hits (8 bits), then ~bits(chi2)
// (31 bits), then 2^25 - 1 minus the start hit's instance-local input index
// (25 bits), which does not depend on the grid.
__device__ __forceinline__ unsigned long long sel_key(int nhit, float chi2, int64_t lid)
{
  const uint32_t bits = __float_as_uint(chi2);
  return ((unsigned long long)(uint32_t)nhit << 56) |
         ((unsigned long long)(~bits & 0x7FFFFFFFu) << 25) |
         (unsigned long long)(0x1FFFFFFull - (unsigned long long)lid);
}

// TrackletConstructor (R13-R17), one workgroup per chunk of at most CH
// tracklets of one instance, one tracklet per thread.  Start hits are in
// (row, bin) order, so a chunk's start rows form a short range; the
// workgroup sweeps the rows upward from the lowest start row (phases 1 and
// 2), each lane walks its state back to its start row (phase 3, no data),
// and the workgroup sweeps downward from the highest start row.  The lanes
// of a sweep search the same row at the same time, so the row's bin
// boundaries and cluster positions are read from the cache (staging each
// row in LDS first cost more instructions than it saved).  Hit slots are [row][tracklet], so the lanes'
// writes of one row are contiguous.
//
// Chunks of one instance are consecutive; workgroup w runs on XCD w % 8
// (round-robin dispatch), so the chunk index is taken from a per-XCD range
// and an instance's rows are cached in one L2.

// first tracklet of every instance (start hits are in instance order)
__global__ __launch_bounds__(kBlock) void k_tl_first(TrackBufs b)
{
  const int64_t S = min(b.counters[CNT_START], b.cap);
  const int64_t t = gtid();
  if (t > S) return;
  const int it = t < S ? b.sseg[b.start[t]] / kRows : b.n_inst;
  const int ip = t > 0 ? b.sseg[b.start[t - 1]] / kRows : -1;
  for (int i = ip + 1; i <= it; i++) b.tl_first[i] = t;
}

// chunk offsets per instance (exclusive scan of ceil(tracklets / CH))
__global__ __launch_bounds__(kBlock) void k_tl_chunks(TrackBufs b, int ch)
{
  int64_t carry = 0;
  for (int64_t i0 = 0; i0 < b.n_inst; i0 += kBlock) {
    const int64_t i = i0 + threadIdx.x;
    const int64_t c = i < b.n_inst ? (b.tl_first[i + 1] - b.tl_first[i] + ch - 1) / ch : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan(c, &tot);
    if (i < b.n_inst) b.chunk_off[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    b.chunk_off[b.n_inst] = carry;
    b.counters[CNT_CHUNKS] = carry;
  }
}

// The 64-lane kernel asks for six waves per SIMD (at most 80 VGPRs): with
// the compiler's own choice of 81 registers it ran at five and took 5 %
// longer.  The wider chunks and the counting build keep the compiler's
// choice (held to 80 registers they spill).
template <int CH, bool COUNT>
constexpr int tl_min_waves() { return CH == 64 && !COUNT ? 6 : 1; }

template <int CH, bool SPEC, bool COUNT>
__global__ __launch_bounds__(CH) __attribute__((amdgpu_waves_per_eu(tl_min_waves<CH, COUNT>())))
void k_tracklets(Consts karg, TrackBufs b)
{
  const Consts& k = kconsts<SPEC>(karg);
  __shared__ int s_inst;
  const int64_t C = b.counters[CNT_CHUNKS];
  const int64_t per = (C + 7) / 8;
  const int64_t slot = blockIdx.x / 8;
  if (slot >= per) return;
  const int64_t lc = (int64_t)(blockIdx.x % 8) * per + slot;
  if (lc >= C) return;
  if (threadIdx.x == 0) s_inst = find_inst(b.chunk_off, b.n_inst, lc);
  __syncthreads();
  const int inst = __builtin_amdgcn_readfirstlane(s_inst);
  const int64_t t0 = b.tl_first[inst] + (lc - b.chunk_off[inst]) * CH;
  const int64_t t1 = min(t0 + CH, b.tl_first[inst + 1]);
  const int segb = inst * kRows;
  const int rlo = b.sseg[b.start[t0]] - segb;
  const int rhi = b.sseg[b.start[t1 - 1]] - segb;
  const int64_t t = t0 + threadIdx.x;
  const bool mine = t < t1;
  const int64_t cap = b.cap;
  int32_t* const H = b.tl_hit + t;  // hit slot of row r at H[r * cap]

  const float kB = k.kB, vy = k.vy, vz = k.vz, smax = k.snp_max;
  const float edge = k.edge_margin, tanh_ = k.tan_half;
  KSt st;
  // the state after the last update (restart and output state), per thread
  // in LDS ([element][lane]): in registers it took 20 more VGPRs, four waves
  // per SIMD instead of seven
  __shared__ float s_keep[20][CH];
  const int tx = threadIdx.x;
  auto put_keep = [&](const KSt& x) {
#pragma unroll
    for (int j = 0; j < 5; j++) s_keep[j][tx] = x.p[j];
#pragma unroll
    for (int j = 0; j < 15; j++) s_keep[5 + j][tx] = x.c[j];
  };
  auto get_keep = [&](KSt& x) {
#pragma unroll
    for (int j = 0; j < 5; j++) x.p[j] = s_keep[j][tx];
#pragma unroll
    for (int j = 0; j < 15; j++) x.c[j] = s_keep[5 + j][tx];
  };
  float chi2 = 0.0f;
  int n = 1, r0 = kRows, rmax = 0, rmin = 0, ncand = 0;
  int32_t hn = -1;  // phase 1: cleaned upward link of the last hit
  if (mine) {
    const int32_t h0 = b.start[t];
    r0 = b.sseg[h0] - segb;
    const int32_t h1 = b.up2[h0];
    const int32_t h2 = b.up2[h1];
    const float dxi = k.row_x[r0 + 2] - k.row_x[r0];
    const float2 q0 = b.yz[h0], q2 = b.yz[h2];
    const float dyi = q2.x - q0.x;
    const float dzi = q2.y - q0.y;
    const float Li = sqrtf(dxi * dxi + dyi * dyi);
    st.p[0] = q0.x;
    st.p[1] = q0.y;
    st.p[2] = dyi / Li;
    st.p[3] = dzi / Li;
    st.p[4] = 0.0f;
    kinit_cov(st, vy, vz);
    rmax = rmin = r0;
    H[(int64_t)r0 * cap] = h0;
    hn = h1;
  }

  // upward sweep: phase 1 follows the cleaned links without a cut (R14),
  // phase 2 searches the rows (R15)
  bool up = mine;
  int phase = 1, miss = 0;
  // every lane writes its slot of each row the sweeps visit (the hit, -1 for
  // a miss, -1 above or below where it stopped), so that each row's slots
  // of the chunk are written together; the rows neither sweep reaches get
  // -1 at the end
  int r_up = rlo + 1;
  for (; r_up < kRows; r_up++) {
    const int r = r_up;
    if constexpr (CH == 64) {
      if (!__ballot(up)) break;  // one wave: a vote, no barrier
    } else {
      if (!__syncthreads_or(up)) break;
    }
    const tpc_row_meta m = b.meta[segb + r];
    // this row's slot: the hit, or -1 (a miss, or a lane that has stopped)
    int32_t slot = -1;
    if (up && r > r0) {
      if (phase == 1 && hn < 0) {
        // links exhausted at row r - 1: the phase-2 restart state is kept
        phase = 2;
        put_keep(st);
      }
      // phase 1: the link's position and its next link are loaded before
      // the propagation, phase 2 takes the position from the search
      float2 qb = make_float2(0.0f, 0.0f);
      int32_t hnext = -1;
      if (phase == 1) {
        qb = b.yz[hn];
        hnext = b.up2[hn];
      }
      if (!kprop(st, k.row_x[r - 1], k.row_x[r], kB, smax)) {
        up = false;
      } else if (phase == 2 && !(fabsf(st.p[0]) <= k.row_x[r] * tanh_ + edge)) {
        up = false;
      } else {
        // one filter update for both phases: the link's hit (phase 1, no cut)
        // or the row's best cluster (phase 2)
        const Innov q = innov(st, vy, vz);
        const int32_t bh = phase == 1 ? hn : ksearch<COUNT>(k, b, m, st, q, ncand, qb);
        if (bh >= 0) {
          chi2 += kupdate_q(st, q, qb.x, qb.y);
          slot = bh;
          n++;
          rmax = r;
          if (phase == 1) {
            hn = hnext;
          } else {
            put_keep(st);
            miss = 0;
          }
        } else if (++miss >= k.tc_max_miss) {
          up = false;
        }
      }
    }
    if (mine && r > r0) H[(int64_t)r * cap] = slot;
  }
  // a lane that never left phase 1 restarts from its last linked row
  if (phase == 1) put_keep(st);

  // phase 3 (R16): back to the start row in steps of at most kWalkRows
  // rows (no updates on the way), then downward
  int stat = 0;
  if (mine) {
    get_keep(st);
    for (int r = rmax; r > r0;) {
      const int rn = r - kWalkRows > r0 ? r - kWalkRows : r0;
      if (!kprop(st, k.row_x[r], k.row_x[rn], kB, smax)) {
        stat = 2;
        break;
      }
      r = rn;
    }
    put_keep(st);  // output state (innermost hit)
  }
  bool dn = mine && stat == 0;
  miss = 0;
  int r_dn = rhi - 1;
  for (; r_dn >= 0; r_dn--) {
    const int r = r_dn;
    if constexpr (CH == 64) {
      if (!__ballot(dn)) break;  // one wave: a vote, no barrier
    } else {
      if (!__syncthreads_or(dn)) break;
    }
    const tpc_row_meta m = b.meta[segb + r];
    int32_t slot = -1;
    if (dn && r < r0) {
      if (!kprop(st, k.row_x[r + 1], k.row_x[r], kB, smax)) {
        dn = false;
      } else if (!(fabsf(st.p[0]) <= k.row_x[r] * tanh_ + edge)) {
        dn = false;
      } else {
        const Innov q = innov(st, vy, vz);
        float2 qb = make_float2(0.0f, 0.0f);
        const int32_t bh = ksearch<COUNT>(k, b, m, st, q, ncand, qb);
        if (bh >= 0) {
          chi2 += kupdate_q(st, q, qb.x, qb.y);
          slot = bh;
          n++;
          rmin = r;
          put_keep(st);
          miss = 0;
        } else if (++miss >= k.tc_max_miss) {
          dn = false;
        }
      }
    }
    if (mine && r < r0) H[(int64_t)r * cap] = slot;
  }
  if (mine) {
    if (stat == 0) {
      if (n < k.min_tracklet_hits) stat = 1;
      else if (!(chi2 >= 0.0f && chi2 <= 3.0e38f)) stat = 3;
    }
#pragma unroll
    for (int j = 0; j < 5; j++) b.tl_par[j * cap + t] = s_keep[j][tx];
#pragma unroll
    for (int j = 0; j < 15; j++) b.tl_cov[j * cap + t] = s_keep[5 + j][tx];
    b.tl_chi2[t] = chi2;
    b.tl_nhit[t] = n;
    b.tl_rmin[t] = rmin;
    b.tl_rmax[t] = rmax;
    b.tl_status[t] = stat;
    if constexpr (COUNT) b.tl_ncand[t] = ncand;
  }
  // the rows neither sweep visited (above where the upward sweep ended,
  // below where the downward sweep ended) read -1 too, since the selection
  // scans whole rows; the lanes write each of them together, so a wave's
  // stores of one row are contiguous.  Every lane that took part in the
  // downward sweep went below its start row before the sweep ended, but a
  // lane that failed the way back (status 2) never did: its start row and
  // the rows above stay as the upward sweep left them.
  for (int r = r_up; r < kRows; r++)
    if (mine) H[(int64_t)r * cap] = -1;
  for (int r = 0; r <= r_dn; r++)
    if (mine && r < r0) H[(int64_t)r * cap] = -1;
  if (mine) {
    // selection key, 0 for a rejected tracklet (it never owns a hit)
    const int64_t lid = (int64_t)b.perm[b.start[t]] - b.inst_off[inst];
    b.tl_key[t] = stat == 0 ? sel_key(n, chi2, lid) : 0ull;
  }
  // one counter update per wave
  const unsigned long long kept = __ballot(mine && stat == 0);
  if ((threadIdx.x & 63) == 0 && kept)
    atomicAdd((unsigned long long*)&b.res->n_tracklets_kept, (unsigned long long)__popcll(kept));
}

// ------------------------------------------------------------------ a6 selection

__global__ __launch_bounds__(kBlock) void k_sel_prep(TrackBufs b)
{
  for (int64_t h = gtid(); h < b.n; h += (int64_t)gridDim.x * blockDim.x) {
    b.owner[h] = 0ull;
    b.own_t[h] = -1;
    b.out.clu2trk[h] = -1;
  }
}

// Ownership (R20), one workgroup per (instance, row).  A position of row r of
// instance i can only be claimed by a tracklet of instance i at row r, so the
// workgroup owns the row: it max-reduces the keys of all the instance's
// tracklets with a hit on the row in LDS (coalesced reads of the [row]
// [tracklet] hit slots and the keys), and after a barrier -- every claim on
// the row is in -- writes per (row, tracklet) whether the tracklet owns its
// hit there, and the row's owner keys.  A row of more than kSelRowPosBig
// positions is reduced with device atomics on the owner array instead (still
// claimed only by this workgroup).  Two instantiations split the rows by
// position count, as in the segment sort: up to kSelRowPos with 32 KB of
// LDS, more with 64 KB.
constexpr int kSelRowPos = 4096;
constexpr int kSelRowPosBig = 8192;
constexpr int kSelBatch = 8;

template <int NP>
__global__ __launch_bounds__(kBlock) void k_sel_rows(TrackBufs b)
{
  __shared__ unsigned long long s_own[NP];
  const int inst = blockIdx.x / kRows, r = blockIdx.x % kRows;
  const int64_t tf = b.tl_first[inst], tl = b.tl_first[inst + 1];
  if (tf == tl) return;
  const int32_t p0 = b.row_off[inst * (kRows + 1) + r];
  const int cnt = b.row_off[inst * (kRows + 1) + r + 1] - p0;
  if ((cnt <= kSelRowPos) != (NP == kSelRowPos)) return;
  const bool lds = cnt <= NP;
  const int32_t* H = b.tl_hit + (int64_t)r * b.cap;
  if (lds)
    for (int j = threadIdx.x; j < cnt; j += kBlock) s_own[j] = 0ull;
  __syncthreads();
  // slots and keys of kSelBatch tracklets per thread are loaded together
  for (int64_t t0 = tf + threadIdx.x; t0 < tl; t0 += kBlock * kSelBatch) {
    int32_t hv[kSelBatch];
    unsigned long long kv[kSelBatch];
#pragma unroll
    for (int u = 0; u < kSelBatch; u++) {
      const int64_t t = t0 + u * kBlock;
      hv[u] = t < tl ? H[t] : -1;
      kv[u] = t < tl ? b.tl_key[t] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kSelBatch; u++) {
      if (hv[u] < 0 || !kv[u]) continue;
      if (lds) atomicMax(&s_own[hv[u] - p0], kv[u]);
      else atomicMax(&b.owner[hv[u]], kv[u]);
    }
  }
  __syncthreads();
  uint8_t* O = b.tl_owned + (int64_t)r * b.cap;
  for (int64_t t0 = tf + threadIdx.x; t0 < tl; t0 += kBlock * kSelBatch) {
    int32_t hv[kSelBatch];
    unsigned long long kv[kSelBatch];
#pragma unroll
    for (int u = 0; u < kSelBatch; u++) {
      const int64_t t = t0 + u * kBlock;
      hv[u] = t < tl ? H[t] : -1;
      kv[u] = t < tl ? b.tl_key[t] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kSelBatch; u++) {
      const int64_t t = t0 + u * kBlock;
      if (t >= tl) continue;
      uint8_t o = 0;
      if (hv[u] >= 0 && kv[u]) {
        // the atomic reads the device-coherent value on the global path
        const unsigned long long w = lds ? s_own[hv[u] - p0] : atomicMax(&b.owner[hv[u]], 0ull);
        o = w == kv[u];
        if (o) b.own_t[hv[u]] = (int32_t)t;
      }
      O[t] = o;
    }
  }
  if (lds)
    for (int j = threadIdx.x; j < cnt; j += kBlock) b.owner[p0 + j] = s_own[j];
}

// The counting kernel runs one thread per tracklet and walks the union of
// the wave's row ranges, so that the ownership bytes of one row ([row]
// [tracklet]) are read contiguously by the wave.  Lanes without a tracklet
// take part in the range reduction with an empty range.
__device__ __forceinline__ void wave_rows(int lo, int hi, int& wlo, int& whi)
{
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = min(lo, __shfl_xor(lo, o, 64));
    hi = max(hi, __shfl_xor(hi, o, 64));
  }
  wlo = lo;
  whi = hi;
}

template <bool SPEC>
__global__ __launch_bounds__(kBlock) void k_sel_count(Consts karg, TrackBufs b, int32_t* own_out)
{
  const Consts& k = kconsts<SPEC>(karg);
  const int64_t S = min(b.counters[CNT_START], b.cap);
  const int64_t t = gtid();
  const int lane = threadIdx.x & 63;
  if (t - lane >= S) return;
  const bool act = t < S && b.tl_status[t] == 0;
  int lo = kRows, hi = -1;
  if (act) {
    lo = b.tl_rmin[t];
    hi = b.tl_rmax[t];
  }
  int wlo, whi;
  wave_rows(lo, hi, wlo, whi);
  const uint8_t* O = b.tl_owned + t;
  // owned rows as a 152-bit mask, 32 rows per word
  uint32_t m[5];
  int own = 0;
#pragma unroll
  for (int w = 0; w < 5; w++) {
    uint32_t mw = 0;
    const int ra = max(wlo, 32 * w), rb = min(whi, 32 * w + 31);
    for (int r = ra; r <= rb; r++) {
      if (r < lo || r > hi) continue;
      if (O[(int64_t)r * b.cap]) mw |= 1u << (r - 32 * w);
    }
    m[w] = mw;
    own += __popc(mw);
  }
  if (own < k.min_track_hits) own = 0;
  if (own) {
    b.tl_rec[2 * t].z = (int)m[0];
    b.tl_rec[2 * t].w = (int)m[1];
    b.tl_rec[2 * t + 1] = make_int4((int)m[2], (int)m[3], (int)m[4], 0);
  }
  const int64_t v = own ? ((int64_t)1 << 32) | own : 0;
#if TPC_DET
  if (t < S) {
    own_out[t] = own;
    b.tsv[t] = v;
  }
#else
  // one append per wave: inclusive scan of the packed (tracks, hits) pairs
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = shfl_up64(x, o);
    if (lane >= o) x += y;
  }
  const int64_t tot = (int64_t)(uint32_t)__shfl((int)(uint32_t)x, 63, 64) |
                      ((int64_t)__shfl((int)(x >> 32), 63, 64) << 32);
  int64_t base = 0;
  if (lane == 0 && tot)
    base = (int64_t)atomicAdd((unsigned long long*)&b.counters[CNT_TRACKS], (unsigned long long)tot);
  base = (int64_t)(uint32_t)__shfl((int)(uint32_t)base, 0, 64) |
         ((int64_t)__shfl((int)(base >> 32), 0, 64) << 32);
  if (t < S) {
    own_out[t] = own;
    b.tsv[t] = own ? base + (x - v) : 0;
  }
#endif
}

// Track records, one thread per tracklet: an accepted tracklet writes its
// track's parameters and its (track, first hit) pair into its record.
template <bool SPEC>
__global__ __launch_bounds__(kBlock) void k_sel_write(Consts karg, TrackBufs b, const int32_t* own_in)
{
  const Consts& k = kconsts<SPEC>(karg);
  const int64_t S = min(b.counters[CNT_START], b.cap);
  const int64_t t = gtid();
  if (t >= S) return;
  const int own = own_in[t];
  int64_t kk = -1, off = 0;
  if (own) {
    const int64_t v = b.tsv[t];
    kk = v >> 32;
    off = v & 0xFFFFFFFFll;
    if (!(kk < b.out.cap_tracks && off + own <= b.out.cap_hits)) kk = -1;
  }
  b.tl_rec[2 * t].x = (int)kk;
  if (kk < 0) return;
  b.tl_rec[2 * t].y = (int)off;
  const int64_t cap = b.cap;
#pragma unroll
  for (int j = 0; j < 5; j++) b.out.param[kk * 5 + j] = b.tl_par[j * cap + t];
#pragma unroll
  for (int j = 0; j < 15; j++) b.out.cov[kk * 15 + j] = b.tl_cov[j * cap + t];
  b.out.chi2[kk] = b.tl_chi2[t];
  b.out.ndf[kk] = 2 * b.tl_nhit[t] - 5;
  b.out.x_ref[kk] = k.row_x[b.tl_rmin[t]];
  b.out.hit_off[kk + 1] = (int32_t)(off + own);
  // with enough capacity every track is written and the totals are the
  // counts; only a truncated output needs the largest written index
  const int64_t tot = b.counters[CNT_TRACKS];
  if ((tot >> 32) > b.out.cap_tracks || (tot & 0xFFFFFFFFll) > b.out.cap_hits) {
    atomicMax((unsigned long long*)&b.res->n_tracks, (unsigned long long)(kk + 1));
    atomicMax((unsigned long long*)&b.res->n_hits, (unsigned long long)(off + own));
  }
}

// Hit lists and the cluster-to-track map, one thread per position: the
// position's owner (k_sel_rows) decides, and the hit's place in its track's
// list is the number of the track's owned rows below the position's row, so
// every list is in ascending row order whatever the thread order.
template <bool SPEC>
__global__ __launch_bounds__(kBlock) void k_sel_hits(Consts karg, TrackBufs b)
{
  const Consts& k = kconsts<SPEC>(karg);
  // contiguous eighths per XCD: the scattered writes of one instance's
  // clusters and tracks meet in one L2
  const int64_t blk = xcd_block((b.n + kBlock - 1) / kBlock);
  if (blk < 0) return;
  const int64_t p = blk * kBlock + threadIdx.x;
  if (p >= b.n) return;
  const int32_t t = b.own_t[p];
  const int32_t seg = b.sseg[p];
  const int32_t c = b.perm[p];
  if (t < 0) return;
  const int4 r0 = b.tl_rec[2 * (int64_t)t];
  const int4 r1 = b.tl_rec[2 * (int64_t)t + 1];
  if (r0.x < 0) return;
  const int r = seg % kRows;
  const uint32_t m[5] = {(uint32_t)r0.z, (uint32_t)r0.w, (uint32_t)r1.x, (uint32_t)r1.y,
                         (uint32_t)r1.z};
  const int w = r >> 5;
  int rank = __popc(m[0] & (w == 0 ? (1u << (r & 31)) - 1 : ~0u));
#pragma unroll
  for (int j = 1; j < 5; j++)
    if (j <= w) rank += __popc(m[j] & (j == w ? (1u << (r & 31)) - 1 : ~0u));
  b.out.hit_clu[(int64_t)r0.y + rank] = c;
  b.out.clu2trk[c] = r0.x;
  if (b.out.hit_data) {
    // the hit's plane, position and sector beside its slot (optional)
    const float2 q = b.yz[p];
    reinterpret_cast<float4*>(b.out.hit_data)[(int64_t)r0.y + rank] =
        make_float4(k.row_x[r], q.x, q.y, (float)((seg / kRows) % kPhi));
  }
}

__global__ void k_sel_finish(TrackBufs b)
{
  const int64_t v = b.counters[CNT_TRACKS];
  const int64_t nt = v >> 32, nh = v & 0xFFFFFFFFll;
  b.res->need_tracks = nt;
  b.res->need_hits = nh;
  if (nt <= b.out.cap_tracks && nh <= b.out.cap_hits) {
    b.res->n_tracks = nt;
    b.res->n_hits = nh;
  } else {
    if (nt > b.out.cap_tracks) b.res->overflow |= 4;
    if (nh > b.out.cap_hits) b.res->overflow |= 8;
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t grid_build(const Consts& k, const GridBufs& b, hipStream_t s)
{
  const int64_t n_seg = (int64_t)b.n_inst * kRows;
  TPC_LAUNCH("grid_clear", blocks_for(n_seg), kBlock, s, k_grid_clear, b);
  if (b.n > 0) TPC_LAUNCH("grid_stats", blocks_for(b.n, kStatItems), kBlock, s, k_grid_stats, k, b);
  TPC_LAUNCH("grid_meta", blocks_for(n_seg), kBlock, s, k_grid_meta, k, b);
  scan_exclusive<int32_t>(b.nb1, n_seg, nullptr, &b.res->n_bins, b.scan_tmp, s);
  TPC_LAUNCH("grid_meta2", blocks_for(n_seg), kBlock, s, k_grid_meta2, b);
  scan_exclusive<int32_t>(b.seg_pos, n_seg, nullptr, nullptr, b.scan_tmp, s);
  if (b.n > 0)
    TPC_LAUNCH("grid_part", xcd_grid(blocks_for(b.n, kPartItems)), kBlock, s, k_grid_part, b);
  TPC_LAUNCH("grid_seg", (unsigned)n_seg, kBlock, s, k_grid_seg<kSegBins>, b);
  TPC_LAUNCH("grid_seg_big", (unsigned)n_seg, kBlock, s, k_grid_seg<kSegBinsBig>, b);
  TPC_LAUNCH("grid_rowoff", blocks_for(n_seg), kBlock, s, k_grid_rowoff, b);
  return hipGetLastError();
}

template <bool SPEC>
hipError_t sector_track_t(const Consts& k, const TrackBufs& b, hipStream_t s)
{
  TPC_LAUNCH("track_init", 1, 64, s, k_track_init, b);
  if (b.n > 0) {
    TPC_LAUNCH("neighbours", xcd_grid(blocks_for(b.n)), kBlock, s, k_neighbours<SPEC>, k, b);
    TPC_LAUNCH("clean", xcd_grid(blocks_for(b.n)), kBlock, s, k_clean, b);
    // ordered compaction in both modes: start-list order sets the tracklet
    // kernel's memory locality, so the scan is cheaper than atomic append
    const int64_t nb = (b.n + kTile - 1) / kTile;
    TPC_LAUNCH("start_count", xcd_grid(nb), kBlock, s, k_start_count<SPEC>, k, b, b.scan_tmp);
    TPC_LAUNCH("scan_partials", 1, 1024, s, k_scan_partials, b.scan_tmp, nb, &b.counters[CNT_START]);
    TPC_LAUNCH("start_write", xcd_grid(nb), kBlock, s, k_start_write, b, b.scan_tmp);
  }
  TPC_LAUNCH("start_finish", 1, 1, s, k_start_finish, b);
  TPC_LAUNCH("sel_prep", blocks_for(b.n > 0 ? b.n : 1), kBlock, s, k_sel_prep, b);
  if (b.cap > 0) {
    TPC_LAUNCH("tl_first", blocks_for(b.cap + 1), kBlock, s, k_tl_first, b);
    TPC_LAUNCH("tl_chunks", 1, kBlock, s, k_tl_chunks, b, k.tl_chunk);
    // chunks are at most cap / CH + n_inst; whole groups of 8 workgroups
    const int64_t ub = (b.cap + k.tl_chunk - 1) / k.tl_chunk + b.n_inst;
    const unsigned tl_blocks = (unsigned)(((ub + 7) / 8) * 8);
    const bool cnt = b.count_candidates;
    const auto kt64 = cnt ? k_tracklets<64, SPEC, true> : k_tracklets<64, SPEC, false>;
    const auto kt128 = cnt ? k_tracklets<128, SPEC, true> : k_tracklets<128, SPEC, false>;
    const auto kt256 = cnt ? k_tracklets<256, SPEC, true> : k_tracklets<256, SPEC, false>;
    if (k.tl_chunk == 64)
      TPC_LAUNCH("tracklets", tl_blocks, 64, s, kt64, k, b);
    else if (k.tl_chunk == 128)
      TPC_LAUNCH("tracklets", tl_blocks, 128, s, kt128, k, b);
    else
      TPC_LAUNCH("tracklets", tl_blocks, 256, s, kt256, k, b);
    const unsigned tblocks = blocks_for(b.cap);
    TPC_LAUNCH("sel_rows", (unsigned)((int64_t)b.n_inst * kRows), kBlock, s,
               k_sel_rows<kSelRowPos>, b);
    TPC_LAUNCH("sel_rows_big", (unsigned)((int64_t)b.n_inst * kRows), kBlock, s,
               k_sel_rows<kSelRowPosBig>, b);
    TPC_LAUNCH("sel_count", tblocks, kBlock, s, k_sel_count<SPEC>, k, b, b.tl_own);
#if TPC_DET
    scan_exclusive<int64_t>(b.tsv, b.cap, &b.counters[CNT_START], &b.counters[CNT_TRACKS],
                            b.scan_tmp, s);
#endif
    TPC_LAUNCH("sel_write", tblocks, kBlock, s, k_sel_write<SPEC>, k, b, b.tl_own);
    if (b.n > 0)
      TPC_LAUNCH("sel_hits", xcd_grid(blocks_for(b.n)), kBlock, s, k_sel_hits<SPEC>, k, b);
  }
  TPC_LAUNCH("sel_finish", 1, 1, s, k_sel_finish, b);
  return hipGetLastError();
}

hipError_t sector_track(const Consts& k, const TrackBufs& b, bool standard, hipStream_t s)
{
  return standard ? sector_track_t<true>(k, b, s) : sector_track_t<false>(k, b, s);
}

}  // namespace TPC_NS
}  // namespace tpcca
