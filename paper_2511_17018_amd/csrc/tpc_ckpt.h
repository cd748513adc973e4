// Checkpoint layout of the refit (forward writes, reverse pass reads).
//
// One lane runs one track, and a wave runs the 64 consecutive tracks of its
// group g (tracks 64 g .. 64 g + 63).  The group's checkpoints fill the
// same entries as its hits, [hit_off[64 g], hit_off[64 g + 64]), ordered by
// hit number j (0 = the track's first hit) and, within one j, by track:
//   entry(t, j) = hit_off[64 g] + sum_k min(L_k, j) + #{k < t : L_k > j}
// over the group's tracks k, L_k their hit counts.  At every step the
// wave's lanes then write (and the reverse pass reads) adjacent entries,
// where one entry per track and hit in hit order put each lane's 80 bytes
// in a different place.
//
// Each wave tabulates, for hit numbers j below kCkTab, the mask of its
// lanes whose track has more than j hits and the sum of min(L_k, j), in
// LDS at the start of the kernel; longer tracks (beyond any pad-row count)
// take a loop over the 64 lengths for their later hits.
#pragma once

namespace tpcca {

constexpr int kCkTab = 160;
constexpr int kCkWaves = kBlock / 64;

struct CkTables {
  unsigned long long mask[kCkWaves][kCkTab];
  int32_t off[kCkWaves][kCkTab + 1];
  int32_t len[kCkWaves][64];
};

// The calling thread's track length (0 when it has no track); fills the
// wave's tables and gives the wave's longest track length in wave_max.
// Every thread of the workgroup must call it (barrier).
__device__ __forceinline__ int64_t ck_build(CkTables& T, const int32_t* hit_off, int64_t n_tracks,
                                            int64_t t, int& wave_max)
{
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int64_t L = 0;
  if (t < n_tracks) {
    const int64_t a = hit_off[t], e = hit_off[t + 1];
    L = e > a ? e - a : 0;
  }
  const int Lc = L < (int64_t)0x7fffffff ? (int)L : 0x7fffffff;
  T.len[w][lane] = Lc;
  int mx = Lc;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const int y = __shfl_xor(mx, o, 64);
    mx = mx > y ? mx : y;
  }
  const int steps = mx < kCkTab ? mx : kCkTab;
  int32_t off = 0;
  for (int j = 0; j < steps; j++) {
    const unsigned long long M = __ballot(j < Lc);
    if (lane == (j & 63)) {
      T.mask[w][j] = M;
      T.off[w][j] = off;
    }
    off += __popcll(M);
  }
  if (lane == 0) T.off[w][steps] = off;
  __syncthreads();
  wave_max = mx;
  return L;
}

// the wave's index in the workgroup (a scalar)
__device__ __forceinline__ int ck_wave() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// the first checkpoint entry of the calling wave's group of tracks (a scalar)
__device__ __forceinline__ int64_t ck_group_base(const int32_t* hit_off)
{
  const int64_t g0 = ((int64_t)blockIdx.x * kBlock) + 64 * ck_wave();
  return hit_off[g0];
}

// Where the calling lane's hit j (0 <= j < its track length) keeps its
// checkpoint, in float4 units from the group's first entry: part q (of five)
// at idx + q * stride.
struct CkSlot {
  int64_t idx;
  int64_t stride;
};

__device__ __forceinline__ CkSlot ck_slot(const CkTables& T, int64_t j)
{
  const int lane = threadIdx.x & 63, w = ck_wave();
  if (j < kCkTab) {
    // the set bits of the mask below this lane
    const unsigned long long M = T.mask[w][j];
    const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(M >> 32),
                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)M, 0u));
    const int32_t e0 = T.off[w][j];
    return CkSlot{5 * (int64_t)e0 + r, (int64_t)(T.off[w][j + 1] - e0)};
  }
  int64_t off = T.off[w][kCkTab], act = 0;
  int rank = 0;
  for (int k = 0; k < 64; k++) {
    const int64_t Lk = T.len[w][k];
    off += (Lk < j ? Lk : j) - (Lk < kCkTab ? Lk : kCkTab);
    act += Lk > j ? 1 : 0;
    rank += (k < lane && Lk > j) ? 1 : 0;
  }
  return CkSlot{5 * off + rank, act};
}

}  // namespace tpcca
