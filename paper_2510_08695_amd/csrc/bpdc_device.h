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

}  // namespace bpdc_dev

#endif  // BPDC_DEVICE_H
