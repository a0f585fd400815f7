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
// spread_bin_of takes the row's smallest and largest saturated posterior,
// spread_bin the row's values.
__device__ __forceinline__ int spread_bin_of(float lo, float hi) {
  const float lg = 1.44269504088896341f;
  const float plo = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(lo * lg));
  const float phi = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(hi * lg));
  const int bin = (int)((plo - phi) * 100.0f);
  return bin < 0 ? 0 : (bin > 100 ? 100 : bin);
}

template <int MAXD>
__device__ __forceinline__ int spread_bin(const float* vals, int deg) {
  float lo = vals[0], hi = vals[0];
  for (int k = 1; k < MAXD; ++k)
    if (k < deg) {
      lo = fminf(lo, vals[k]);
      hi = fmaxf(hi, vals[k]);
    }
  return spread_bin_of(lo, hi);
}

// Product-sum rule (Sec. II.C) in the log domain: with
//   phi(x) = -ln tanh(x / 2) = ln((e^x + 1) / (e^x - 1))   (x >= 0),
// an involution with phi(0) = +inf and phi(+inf) = 0, the message
// 2 atanh(prod tanh(|q| / 2)) equals phi(sum phi(|q|)).  Unlike the product of
// tanh values, which rounds to 1 long before the messages saturate, both sums
// and phi keep their relative precision at every magnitude.  float32 phi from
// the hardware exp2 / log2 / reciprocal (about 1 ulp each), in three ranges:
//   x < 1/2:   -ln(x/2) + y^2/3 - 7y^4/90 + 62y^6/2835 - 127y^8/18900 (y = x/2;
//              the Taylor series of -ln(tanh(y)/y), Bernoulli-number coefficients);
//   1/2 <= x < 2:  ln((1 + e) / (1 - e)),  e = e^-x  (1 - e >= 0.39: no cancellation);
//   x >= 2:    2 atanh(e) = 2e (1 + e^2/3 + e^4/5 + e^6/7 + e^8/9)  (e <= 0.136).
// Every GPU product-sum decoder uses this function; a cut column sends +inf
// (prior probability 0), whose phi is 0.
__device__ __forceinline__ float phi(float x) {  // x >= 0 or +inf
  const float y = 0.5f * x, y2 = y * y;
  float ps = fmaf(y2, -127.0f / 18900.0f, 62.0f / 2835.0f);
  ps = fmaf(ps, y2, -7.0f / 90.0f);
  ps = fmaf(ps, y2, 1.0f / 3.0f);
  ps = ps * y2;
  // e = e^-x = 2^-(x log2 e): t = x log2 e rounded, with its rounding error d
  // (fma) and the constant's own (x times log2 e - its float value), and
  // 2^-d = 1 - d ln 2 to first order (|d| < 2^-17), so the exponent's rounding
  // does not scale with x; beyond x = 128 (+inf included) e underflows to 0
  const float xc = fminf(x, 128.0f);
  const float t = xc * 1.44269504088896341f;
  const float d = fmaf(xc, 1.44269504088896341f, -t) + xc * 1.9259629911e-8f;
  const float e = __builtin_amdgcn_exp2f(-t) * fmaf(-d, 0.693147180559945309f, 1.0f);
  const float e2 = e * e;
  float pl = fmaf(e2, 1.0f / 9.0f, 1.0f / 7.0f);
  pl = fmaf(pl, e2, 1.0f / 5.0f);
  pl = fmaf(pl, e2, 1.0f / 3.0f);
  pl = fmaf(pl, e2, 1.0f);
  const float large = 2.0f * e * pl;
  const float arg = (x < 0.5f) ? y : (1.0f + e) * __builtin_amdgcn_rcpf(1.0f - e);
  const float lg = __builtin_amdgcn_logf(arg) * 0.693147180559945309f;  // ln(arg)
  return (x < 0.5f) ? ps - lg : ((x < 2.0f) ? lg : large);
}

// q of a product-sum edge: sat(L - r), except +inf from a cut column (L = +inf).
__device__ __forceinline__ float ps_q(float L, float r, float lsat) {
  const float x = L - r;
  return (x == __builtin_huge_valf()) ? x : sat(x, lsat);
}

}  // namespace bpdc_dev

#endif  // BPDC_DEVICE_H
