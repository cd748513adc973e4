// Kalman-filter device functions of the tracker and the refit (readings R7
// propagation, R8 Jacobian, R9 update).  Included inside the namespace of a
// kernel build; every expression keeps the operand order of the readings so
// that the contraction-free (deterministic) build rounds exactly as the CPU
// reference does.
#pragma once

// 1/6, 3/40 and 3/20 rounded to binary32
constexpr float kSixth = 0x1.555556p-3f;
constexpr float k3_40 = 0x1.333334p-4f;
constexpr float k3_20 = 0x1.333334p-3f;

struct KSt {
  float p[5];
  float c[15];
};

__device__ __forceinline__ constexpr int ci(int i, int j)
{
  return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
}

// R7 + R8 (see the design notes for the exact operation order); ds_out
// receives the step's signed transverse arc length.
__device__ __forceinline__ bool kprop_ds(KSt& s, float x1, float x2, float kB, float smax,
                                         float& ds_out)
{
  const float one = 1.0f;
  const float dx = x2 - x1;
  const float snp = s.p[2], tgl = s.p[3], qpt = s.p[4];
  const float cc = kB * qpt;
  const float s2 = snp + cc * dx;
  // defined only for |snp| < 1 at both ends of the step (after an update
  // the incoming state may lie outside)
  if (!(fabsf(snp) < smax) || !(fabsf(s2) < smax)) return false;
  const float c1 = sqrtf((one - snp) * (one + snp));
  const float c2 = sqrtf((one - s2) * (one + s2));
  const float f = (snp + s2) / (c1 + c2);
  const float dy = dx * f;
  const float L = sqrtf(dx * dx + dy * dy);
  const float lc = L * cc;
  const float u2 = (lc * lc) * 0.25f;
  const float g = one + u2 * (kSixth + u2 * k3_40);
  const float sg = dx < 0.0f ? -one : one;
  const float ds = (sg * L) * g;
  ds_out = ds;
  const float h = (one + f * f) * 0.5f;
  const float ic1 = one / c1, ic2 = one / c2;
  const float dfs = h * (ic1 + ic2);
  const float dfq = (h * (dx * ic2)) * kB;
  const float dg = kSixth + u2 * k3_20;
  const float dyl = dy / L;
  const float hlc = 0.5f * lc;
  const float Lg = L * dg;
  const float a = dx * dfs;
  const float dLs = dyl * a;
  const float du2s = hlc * (dLs * cc);
  const float d = tgl * (sg * (dLs * g + Lg * du2s));
  const float bq = dx * dfq;
  const float dLq = dyl * bq;
  const float du2q = hlc * (dLq * cc + L * kB);
  const float gq = tgl * (sg * (dLq * g + Lg * du2q));
  const float e = ds;
  const float hq = kB * dx;
  s.p[0] = s.p[0] + dy;
  s.p[1] = s.p[1] + tgl * ds;
  s.p[2] = s2;
  float B0[5], B1[5], B2[5];
#pragma unroll
  for (int j = 0; j < 5; j++) {
    B0[j] = (s.c[ci(0, j)] + a * s.c[ci(2, j)]) + bq * s.c[ci(4, j)];
    B1[j] = ((s.c[ci(1, j)] + d * s.c[ci(2, j)]) + e * s.c[ci(3, j)]) + gq * s.c[ci(4, j)];
    B2[j] = s.c[ci(2, j)] + hq * s.c[ci(4, j)];
  }
  const float n30 = (s.c[ci(3, 0)] + a * s.c[ci(3, 2)]) + bq * s.c[ci(3, 4)];
  const float n31 = ((s.c[ci(3, 1)] + d * s.c[ci(3, 2)]) + e * s.c[ci(3, 3)]) + gq * s.c[ci(3, 4)];
  const float n32 = s.c[ci(3, 2)] + hq * s.c[ci(3, 4)];
  const float n40 = (s.c[ci(4, 0)] + a * s.c[ci(4, 2)]) + bq * s.c[ci(4, 4)];
  const float n41 = ((s.c[ci(4, 1)] + d * s.c[ci(4, 2)]) + e * s.c[ci(4, 3)]) + gq * s.c[ci(4, 4)];
  const float n42 = s.c[ci(4, 2)] + hq * s.c[ci(4, 4)];
  s.c[0] = (B0[0] + a * B0[2]) + bq * B0[4];
  s.c[1] = (B1[0] + a * B1[2]) + bq * B1[4];
  s.c[2] = ((B1[1] + d * B1[2]) + e * B1[3]) + gq * B1[4];
  s.c[3] = (B2[0] + a * B2[2]) + bq * B2[4];
  s.c[4] = ((B2[1] + d * B2[2]) + e * B2[3]) + gq * B2[4];
  s.c[5] = B2[2] + hq * B2[4];
  s.c[6] = n30;
  s.c[7] = n31;
  s.c[8] = n32;
  s.c[10] = n40;
  s.c[11] = n41;
  s.c[12] = n42;
  return true;
}

__device__ __forceinline__ bool kprop(KSt& s, float x1, float x2, float kB, float smax)
{
  float ds;
  return kprop_ds(s, x1, x2, kB, smax, ds);
}

struct Innov {
  float S00, S11, si00, si01, si11;
};

__device__ __forceinline__ Innov innov(const KSt& s, float vy, float vz)
{
  Innov q;
  const float S00 = s.c[0] + vy, S01 = s.c[1], S11 = s.c[2] + vz;
  const float det = S00 * S11 - S01 * S01;
  q.S00 = S00;
  q.S11 = S11;
  q.si00 = S11 / det;
  q.si01 = -(S01 / det);
  q.si11 = S00 / det;
  return q;
}

__device__ __forceinline__ float chi2_of(const Innov& q, float r0, float r1)
{
  return r0 * (q.si00 * r0 + q.si01 * r1) + r1 * (q.si01 * r0 + q.si11 * r1);
}

// R9
__device__ __forceinline__ float kupdate_q(KSt& s, const Innov& q, float my, float mz)
{
  const float r0 = my - s.p[0], r1 = mz - s.p[1];
  const float chi2 = chi2_of(q, r0, r1);
  float k0[5], k1[5], hc0[5], hc1[5];
#pragma unroll
  for (int i = 0; i < 5; i++) {
    k0[i] = s.c[ci(i, 0)] * q.si00 + s.c[ci(i, 1)] * q.si01;
    k1[i] = s.c[ci(i, 0)] * q.si01 + s.c[ci(i, 1)] * q.si11;
    hc0[i] = s.c[ci(0, i)];
    hc1[i] = s.c[ci(1, i)];
  }
#pragma unroll
  for (int i = 0; i < 5; i++) s.p[i] = s.p[i] + (k0[i] * r0 + k1[i] * r1);
#pragma unroll
  for (int i = 0; i < 5; i++)
#pragma unroll
    for (int j = 0; j <= i; j++)
      s.c[ci(i, j)] = s.c[ci(i, j)] - (k0[i] * hc0[j] + k1[i] * hc1[j]);
  return chi2;
}

__device__ __forceinline__ float kupdate(KSt& s, float my, float mz, float vy, float vz)
{
  return kupdate_q(s, innov(s, vy, vz), my, mz);
}

__device__ __forceinline__ void kinit_cov(KSt& s, float vy, float vz)
{
#pragma unroll
  for (int j = 0; j < 15; j++) s.c[j] = 0.0f;
  s.c[0] = vy;
  s.c[2] = vz;
  s.c[5] = 1.0f;
  s.c[9] = 1.0f;
  s.c[14] = 100.0f;
}

