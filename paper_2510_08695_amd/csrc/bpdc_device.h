// Device helpers shared by every BP+DC kernel of libbpdc (gfx950).
//
// This header is compiled into the library's own kernels and is also
// prepended to the source of the code-specialised lane kernel that the
// runtime compiles with hipRTC, so it must stay self-contained (no includes).
#pragma once

#ifndef BPDC_DEVICE_H
#define BPDC_DEVICE_H

namespace bpdc_dev {

typedef unsigned int u32;
typedef unsigned long long u64;

// Saturation of a message or posterior to [-lsat, lsat] (one v_med3_f32).
__device__ __forceinline__ float sat(float x, float lsat) {
  return __builtin_amdgcn_fmed3f(x, -lsat, lsat);
}

// SplitMix64 output function (Steele, Lea, Flood, OOPSLA 2014): advance by
// the golden-ratio increment, then two xor-shift-multiply rounds and a final
// xor-shift.  Used only for the random choice among tied DC candidates.
__device__ __forceinline__ u64 splitmix64(u64 x) {
  u64 z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Counter-based draw for (seed, global shot index, degeneracy-matrix row):
// a function of its arguments only, so the choice does not depend on the
// order in which rows or shots are processed (Sec. III.A).
__device__ __forceinline__ u64 tie_hash(u64 seed, u64 shot, u64 row) {
  return splitmix64(splitmix64(shot * 0x1000000ull + row) ^ seed);
}

// floor(h * k / 2^64): index in [0, k) from a 64-bit draw.
__device__ __forceinline__ u32 scale_draw(u64 h, u32 k) {
  return (u32)__umul64hi(h, (u64)k);
}

// Hard decision e = [L <= 0] as the sign bit of (bits(L) - 1): +0 maps to
// 0xFFFFFFFF (decision 1), positive values and +inf to sign 0, negative
// values keep sign 1.  Posteriors are never -0 (they start from a prior LLR
// that is not -0 and exact cancellations round to +0).
__device__ __forceinline__ u32 hard_decision_bit31(float L) {
  return __float_as_uint(L) - 1u;
}

// Degeneracy cutting for one row of D: among the row's columns (given in
// ascending order) keep those whose saturated posterior is within the
// relative tolerance of the row maximum, and pick one of them either by the
// hash of (seed, shot, row) or as the lowest column.  `vals` holds the
// saturated posteriors of the row's columns.
template <int MAXDEG>
__device__ __forceinline__ int dc_pick(const int* cols, const float* vals, int deg, float tie_eps,
                                       int tie_lowest, u64 seed, u64 shot, u64 row) {
  float lmax = vals[0];
  for (int k = 1; k < deg; ++k) lmax = fmaxf(lmax, vals[k]);
  const float scale = fmaxf(1.0f, fabsf(lmax));
  const float thr = lmax - tie_eps * scale;
  int nt = 0;
  for (int k = 0; k < deg; ++k) nt += (vals[k] >= thr) ? 1 : 0;
  int want = 0;
  if (!tie_lowest && nt > 1) want = (int)scale_draw(tie_hash(seed, shot, row), (u32)nt);
  int pick = cols[0];
  int seen = 0;
  for (int k = 0; k < deg; ++k) {
    if (vals[k] >= thr) {
      if (seen == want) pick = cols[k];
      ++seen;
    }
  }
  return pick;
}

// Degeneracy-cutting diagnostic (Appendix B): the spread of the posterior
// error probabilities p = 1 / (1 + e^L) over a row of D (largest minus
// smallest; p falls as L grows, so it is p(min L) - p(max L)), as a bin
// floor(100 spread) in 0..100.  e^L by the hardware exp2 (about 1 ulp).
template <int MAXD>
__device__ __forceinline__ int spread_bin(const float* vals, int deg) {
  float lo = vals[0], hi = vals[0];
  for (int k = 1; k < MAXD; ++k)
    if (k < deg) {
      lo = fminf(lo, vals[k]);
      hi = fmaxf(hi, vals[k]);
    }
  const float lg = 1.44269504088896341f;
  const float plo = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(lo * lg));
  const float phi = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(hi * lg));
  const int bin = (int)((plo - phi) * 100.0f);
  return bin < 0 ? 0 : (bin > 100 ? 100 : bin);
}

// Product-sum rule (Sec. II.C) in float32, written from the identities
//   tanh(x/2) = (1 - e) / (1 + e),   e = exp(-x) = 2^(-x log2 e),
//   2 atanh(p) = ln((1 + p) / (1 - p)) = ln 2 * log2((1 + p) / (1 - p)),
// with the hardware exp2 / log2 / reciprocal (about 1 ulp each), and below
// the points where those forms cancel (x < 1/2, p < 1/4) the odd Taylor
// series of tanh(x/2) and of 2 atanh(p), whose first omitted terms are below
// 1e-8 relative there.  Accurate to a few ulp, about 15 instructions each;
// every GPU product-sum decoder uses these two functions.
__device__ __forceinline__ float tanh_half(float x) {  // x >= 0
  const float y = 0.5f * x, y2 = y * y;
  float s = fmaf(y2, 62.0f / 2835.0f, -17.0f / 315.0f);
  s = fmaf(s, y2, 2.0f / 15.0f);
  s = fmaf(s, y2, -1.0f / 3.0f);
  s = fmaf(s, y2, 1.0f);
  const float series = y * s;
  const float e = __builtin_amdgcn_exp2f(-fminf(x, 64.0f) * 1.44269504088896341f);
  const float direct = (1.0f - e) * __builtin_amdgcn_rcpf(1.0f + e);
  return x < 0.5f ? series : direct;
}
__device__ __forceinline__ float atanh2(float p) {  // 2 atanh(p), 0 <= p <= 1 (+inf at 1)
  const float p2 = p * p;
  float s = fmaf(p2, 1.0f / 11.0f, 1.0f / 9.0f);
  s = fmaf(s, p2, 1.0f / 7.0f);
  s = fmaf(s, p2, 1.0f / 5.0f);
  s = fmaf(s, p2, 1.0f / 3.0f);
  s = fmaf(s, p2, 1.0f);
  const float series = 2.0f * p * s;
  const float direct = __builtin_amdgcn_logf((1.0f + p) * __builtin_amdgcn_rcpf(1.0f - p)) * 0.693147180559945309f;
  return p < 0.25f ? series : direct;
}

}  // namespace bpdc_dev

#endif  // BPDC_DEVICE_H
