// Plain BP+DC decoder: one kernel launch per BP phase per iteration, all
// per-edge messages in HBM in edge-major layout [E][B] (consecutive shots are
// consecutive addresses, so every access is coalesced).  Shots that finished
// a pass are skipped by a per-shot state check; DC is its own kernel.  No
// persistence, no LDS residency, no graph capture: the straightforward GPU
// decoder that the fused kernels are measured against.  Arithmetic order is
// the same as every other decoder of the library (flooding schedule, scaled
// min-sum, Sec. II.C; degeneracy cutting, Sec. III.A), so its results are
// bit-identical to theirs.
#include "internal.h"
// after the HIP runtime header: bpdc_device.h itself includes nothing
#include "bpdc_device.h"

namespace bpdc {
namespace {

using bpdc_dev::u32;
using bpdc_dev::u64;

enum : unsigned char { ST_PASS1 = 0, ST_DONE1 = 1, ST_NEED_DC = 2, ST_PASS2 = 3, ST_DONE2 = 4 };

struct PlainWs {
  float* q;          // [E][B]
  float* r;          // [E][B]
  float* L;          // [n][B]
  float* lam2;       // [n][B] prior of the second pass (+inf on cut columns)
  unsigned char* st; // [B]
  unsigned char* conv;  // [B]
  short* it;         // [B][2]
  u32* mark;         // [ceil(n/32)][B] nominees of one soft-DC application
};

__host__ __device__ inline size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

PlainWs carve(const DevCode& c, int64_t B, void* ws) {
  char* p = (char*)ws;
  PlainWs w;
  w.q = (float*)p; p += align_up(sizeof(float) * (size_t)c.E * B);
  w.r = (float*)p; p += align_up(sizeof(float) * (size_t)c.E * B);
  w.L = (float*)p; p += align_up(sizeof(float) * (size_t)c.n * B);
  w.lam2 = (float*)p; p += align_up(sizeof(float) * (size_t)c.n * B);
  w.st = (unsigned char*)p; p += align_up((size_t)B);
  w.conv = (unsigned char*)p; p += align_up((size_t)B);
  w.it = (short*)p; p += align_up(sizeof(short) * 2 * (size_t)B);
  w.mark = (u32*)p; p += align_up(sizeof(u32) * (size_t)((c.n + 31) / 32) * B);
  return w;
}

__device__ __forceinline__ u32 syn_bit(const uint64_t* syn, int sw64, int64_t b, int c) {
  return (u32)((syn[b * sw64 + (c >> 6)] >> (c & 63)) & 1ull);
}

__global__ void k_init_state(unsigned char* st, short* it, int64_t B) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  st[b] = ST_PASS1;
  it[2 * b] = 0;
  it[2 * b + 1] = 0;
}

// First-iteration messages of a pass: q_{v->c} = sat(prior_v), +inf on cut
// columns (prior probability 0: never a minimum, phi(+inf) = 0 in a sum).
__global__ void k_init_msgs(DevCode c, PlainWs w, int64_t B, int pass, float lsat) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (b >= B) return;
  if (w.st[b] != (pass ? ST_PASS2 : ST_PASS1)) return;
  const float lam = pass ? w.lam2[(size_t)v * B + b] : c.lam[v];
  const float q0 = (lam == __builtin_huge_valf()) ? lam : bpdc_dev::sat(lam, lsat);
  for (int k = c.h_col_ptr[v]; k < c.h_col_ptr[v + 1]; ++k) w.q[(size_t)c.h_col_edge[k] * B + b] = q0;
}

// Check half, product-sum rule (Sec. II.C): r_{c->v} = sign * alpha *
// 2 atanh(product over the other edges of tanh(|q| / 2)), evaluated in the
// log domain as phi(sum over the other edges of phi(|q|)), the sum taken left
// to right in row order; the magnitude saturates at lsat (an empty sum gives
// phi(0) = +inf).  Sign as for min-sum.  At most 32 edges per check (plan
// creation refuses product-sum on longer rows).  phi is bpdc_device.h's
// float32 form, shared with the lane and group kernels.
__device__ void check_product_sum(const DevCode& c, const PlainWs& w, int64_t B, int64_t b, int e0, int e1,
                                  u32 neg, float alpha, float lsat) {
  float ph[32];
  for (int e = e0; e < e1; ++e) {
    const float q = w.q[(size_t)e * B + b];
    neg ^= (q < 0.0f) ? 1u : 0u;
    ph[e - e0] = bpdc_dev::phi(fabsf(q));
  }
  for (int e = e0; e < e1; ++e) {
    // phi of the sum of the other edges' phi, left to right in row order
    float sum = 0.0f;
    for (int o = e0; o < e1; ++o)
      if (o != e) sum = sum + ph[o - e0];
    float mag = bpdc_dev::phi(sum);
    if (!(mag < lsat)) mag = lsat;
    const float val = alpha * mag;
    const float q = w.q[(size_t)e * B + b];
    const bool negative = (neg ^ ((q < 0.0f) ? 1u : 0u)) != 0u;
    w.r[(size_t)e * B + b] = negative ? -val : val;
  }
}

// Check half: r_{c->v} = sign * alpha * (min over the other |q|), sign =
// s_c xor the other signs.  Minimum and second minimum start at lsat (a
// minimum over no inputs is lsat) and are tracked with strict '<'.
__global__ void k_check(DevCode c, PlainWs w, const uint64_t* syn, int sw64, int64_t B, int pass,
                        float alpha, float lsat, int rule) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int chk = blockIdx.y;
  if (b >= B) return;
  if (w.st[b] != (pass ? ST_PASS2 : ST_PASS1)) return;
  const int e0 = c.h_row_ptr[chk], e1 = c.h_row_ptr[chk + 1];
  u32 neg = syn_bit(syn, sw64, b, chk);
  if (rule) {
    check_product_sum(c, w, B, b, e0, e1, neg, alpha, lsat);
    return;
  }
  float m1 = lsat, m2 = lsat;
  int amin = -1;
  for (int e = e0; e < e1; ++e) {
    const float q = w.q[(size_t)e * B + b];
    const float a = fabsf(q);
    neg ^= (q < 0.0f) ? 1u : 0u;
    if (a < m1) {
      m2 = m1;
      m1 = a;
      amin = e;
    } else if (a < m2) {
      m2 = a;
    }
  }
  const float v1 = alpha * m1, v2 = alpha * m2;
  for (int e = e0; e < e1; ++e) {
    const float q = w.q[(size_t)e * B + b];
    const float val = (e == amin) ? v2 : v1;
    const bool negative = (neg ^ ((q < 0.0f) ? 1u : 0u)) != 0u;
    w.r[(size_t)e * B + b] = negative ? -val : val;
  }
}

// Variable half: L_v = prior + sum of r (ascending check order), q = sat(L - r).
// The first pass reads its per-shot prior from lam2 when soft DC shifts it.
__global__ void k_var(DevCode c, PlainWs w, int64_t B, int pass, float lsat, int soft) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (b >= B) return;
  if (w.st[b] != (pass ? ST_PASS2 : ST_PASS1)) return;
  const float lam = (pass || soft) ? w.lam2[(size_t)v * B + b] : c.lam[v];
  const int k0 = c.h_col_ptr[v], k1 = c.h_col_ptr[v + 1];
  if (lam == __builtin_huge_valf()) {  // cut column: prior probability 0 (LLR +inf)
    for (int k = k0; k < k1; ++k) w.q[(size_t)c.h_col_edge[k] * B + b] = __builtin_huge_valf();
    w.L[(size_t)v * B + b] = lam;
    return;
  }
  float L = lam;
  for (int k = k0; k < k1; ++k) L = L + w.r[(size_t)c.h_col_edge[k] * B + b];
  for (int k = k0; k < k1; ++k) {
    const size_t e = (size_t)c.h_col_edge[k] * B + b;
    w.q[e] = bpdc_dev::sat(L - w.r[e], lsat);
  }
  w.L[(size_t)v * B + b] = L;
}

// Hard decision e = [L <= 0] and stop test H e = s; pass bookkeeping.
__global__ void k_stop(DevCode c, PlainWs w, const uint64_t* syn, int sw64, int64_t B, int pass,
                       int t, int T, int stop) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (w.st[b] != (pass ? ST_PASS2 : ST_PASS1)) return;
  bool ok = true;
  for (int chk = 0; chk < c.m && ok; ++chk) {
    u32 par = syn_bit(syn, sw64, b, chk);
    for (int e = c.h_row_ptr[chk]; e < c.h_row_ptr[chk + 1]; ++e)
      par ^= (w.L[(size_t)c.h_col[e] * B + b] <= 0.0f) ? 1u : 0u;
    ok = (par == 0u);
  }
  w.conv[b] = ok ? 1 : 0;
  if ((stop && ok) || t >= T) {
    w.conv[b] = ok ? 1 : 0;
    w.it[2 * b + pass] = (short)t;
    w.st[b] = pass ? ST_DONE2 : (ok ? ST_DONE1 : ST_NEED_DC);
  }
}

// First-pass prior of every shot for soft DC: the channel prior.
__global__ void k_init_soft(DevCode c, PlainWs w, int64_t B) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y;
  if (b >= B) return;
  w.lam2[(size_t)v * B + b] = c.lam[v];
}

// Intermittent soft DC (application j of the first pass), one thread per shot
// still in its first pass with H e != s: every row of D nominates as in DC
// (row h hashed as j * rows(D) + h) and each nominee's prior LLR rises by
// `shift` once, however many rows nominate it.
__global__ void k_soft(DevCode c, PlainWs w, int64_t B, int64_t shot_offset, float lsat, float tie_eps,
                       int tie_lowest, u64 seed, u64 j, float shift) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (w.st[b] != ST_PASS1 || w.conv[b]) return;
  const int nw = (c.n + 31) >> 5;
  for (int i = 0; i < nw; ++i) w.mark[(size_t)i * B + b] = 0u;
  for (int h = 0; h < c.md; ++h) {
    const int e0 = c.d_row_ptr[h], deg = c.d_row_ptr[h + 1] - e0;
    if (deg == 0) continue;
    int cols[32];
    float vals[32];
    for (int k = 0; k < deg; ++k) {
      cols[k] = c.d_col[e0 + k];
      vals[k] = bpdc_dev::sat(w.L[(size_t)cols[k] * B + b], lsat);
    }
    const int pick = bpdc_dev::dc_pick<32>(cols, vals, deg, tie_eps, tie_lowest, seed, (u64)(shot_offset + b),
                                           j * (u64)c.md + (u64)h);
    w.mark[(size_t)(pick >> 5) * B + b] |= 1u << (pick & 31);
  }
  for (int v = 0; v < c.n; ++v)
    if ((w.mark[(size_t)(v >> 5) * B + b] >> (v & 31)) & 1u) {
      const size_t i = (size_t)v * B + b;
      w.lam2[i] = w.lam2[i] + shift;
    }
}

// Degeneracy cutting, one thread per shot whose first pass failed.
__global__ void k_dc(DevCode c, PlainWs w, int64_t B, int64_t shot_offset, float lsat, float tie_eps,
                     int tie_lowest, u64 seed, int posterior, unsigned long long* dcstats) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (w.st[b] != ST_NEED_DC) return;
  // second-pass prior of every column (cut columns overwritten below)
  for (int v = 0; v < c.n; ++v)
    w.lam2[(size_t)v * B + b] = posterior ? bpdc_dev::sat(w.L[(size_t)v * B + b], lsat) : c.lam[v];
  for (int h = 0; h < c.md; ++h) {
    const int e0 = c.d_row_ptr[h], deg = c.d_row_ptr[h + 1] - e0;
    if (deg == 0) continue;
    int cols[32];
    float vals[32];
    for (int k = 0; k < deg; ++k) {
      cols[k] = c.d_col[e0 + k];
      vals[k] = bpdc_dev::sat(w.L[(size_t)cols[k] * B + b], lsat);
    }
    const int pick = bpdc_dev::dc_pick<32>(cols, vals, deg, tie_eps, tie_lowest, seed,
                                           (u64)(shot_offset + b), (u64)h);
    w.lam2[(size_t)pick * B + b] = __builtin_huge_valf();
    if (dcstats) atomicAdd(&dcstats[bpdc_dev::spread_bin<32>(vals, deg)], 1ull);
  }
  if (dcstats) {  // DC diagnostics: shots that ran DC, cut size
    int ncut = 0;
    for (int v = 0; v < c.n; ++v) ncut += w.lam2[(size_t)v * B + b] == __builtin_huge_valf() ? 1 : 0;
    atomicAdd(&dcstats[101], 1ull);
    atomicAdd(&dcstats[102 + ncut], 1ull);
  }
  w.st[b] = ST_PASS2;
}

__global__ void k_output(DevCode c, PlainWs w, int64_t B, float lsat, uint64_t* corr,
                         uint8_t* flags, float* post, uint64_t* cut, int16_t* iters) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int nw = (c.n + 63) >> 6;
  const bool dc = w.st[b] == ST_DONE2;
  for (int wd = 0; wd < nw; ++wd) {
    u64 e = 0, k = 0;
    for (int j = 0; j < 64; ++j) {
      const int v = wd * 64 + j;
      if (v >= c.n) break;
      const float L = w.L[(size_t)v * B + b];
      if (L <= 0.0f) e |= 1ull << j;
      if (dc && w.lam2[(size_t)v * B + b] == __builtin_huge_valf()) k |= 1ull << j;
    }
    corr[b * nw + wd] = e;
    if (cut) cut[b * nw + wd] = k;
  }
  flags[b] = (uint8_t)((w.conv[b] ? 1 : 0) | (dc ? 2 : 0));
  if (iters) {
    iters[2 * b] = w.it[2 * b];
    iters[2 * b + 1] = w.it[2 * b + 1];
  }
  if (post) {
    for (int v = 0; v < c.n; ++v) {
      const float L = w.L[(size_t)v * B + b];
      post[b * c.n + v] = (L == __builtin_huge_valf()) ? L : bpdc_dev::sat(L, lsat);
    }
  }
}

// The product-sum function phi of bpdc_device.h on an array (accuracy tests).
__global__ void k_eval_phi(const float* x, int64_t n, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = bpdc_dev::phi(x[i]);
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, size_t count) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

}  // namespace

hipError_t eval_phi(const float* x, int64_t n, float* out, hipStream_t stream) {
  (void)hipGetLastError();
  if (n > 0) hipLaunchKernelGGL(k_eval_phi, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, x, n, out);
  return hipGetLastError();
}

hipError_t fill_u64(uint64_t* p, uint64_t v, size_t count, hipStream_t stream) {
  if (count == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((count + 255) / 256);
  hipLaunchKernelGGL(k_fill_u64, dim3(blocks), dim3(256), 0, stream, p, v, count);
  return hipGetLastError();
}

size_t plain_workspace_bytes(const DevCode& c, int64_t B) {
  return align_up(sizeof(float) * (size_t)c.E * B) * 2 + align_up(sizeof(float) * (size_t)c.n * B) * 2 +
         align_up((size_t)B) * 2 + align_up(sizeof(short) * 2 * (size_t)B) +
         align_up(sizeof(u32) * (size_t)((c.n + 31) / 32) * B);
}

hipError_t plain_decode(const DevCode& c, const KParams& p, const DecodeIO& io, void* ws,
                        hipStream_t stream) {
  const int64_t B = io.B;
  if (B == 0) return hipSuccess;
  (void)hipGetLastError();  // report only this decode's errors
  PlainWs w = carve(c, B, ws);
  const int sw64 = (c.m + 63) >> 6;
  const dim3 blk(256);
  const unsigned gx = (unsigned)((B + 255) / 256);
  hipLaunchKernelGGL(k_init_state, dim3(gx), blk, 0, stream, w.st, w.it, B);
  const int soft = p.soft_period > 0;
  if (soft) hipLaunchKernelGGL(k_init_soft, dim3(gx, c.n), blk, 0, stream, c, w, B);
  for (int pass = 0; pass < 2; ++pass) {
    const int T = pass ? p.T2 : p.T1;
    if (pass == 1)
      hipLaunchKernelGGL(k_dc, dim3(gx), blk, 0, stream, c, w, B, io.shot_offset, p.lsat, p.tie_eps,
                         p.tie_lowest, (u64)p.seed, p.second_pass_posterior, (unsigned long long*)io.dcstats);
    hipLaunchKernelGGL(k_init_msgs, dim3(gx, c.n), blk, 0, stream, c, w, B, pass, p.lsat);
    for (int t = 1; t <= T; ++t) {
      hipLaunchKernelGGL(k_check, dim3(gx, c.m), blk, 0, stream, c, w, io.syn, sw64, B, pass, p.alpha,
                         p.lsat, p.rule);
      hipLaunchKernelGGL(k_var, dim3(gx, c.n), blk, 0, stream, c, w, B, pass, p.lsat, soft);
      hipLaunchKernelGGL(k_stop, dim3(gx), blk, 0, stream, c, w, io.syn, sw64, B, pass, t, T, p.stop);
      if (soft && pass == 0 && t % p.soft_period == 0 && t < T)
        hipLaunchKernelGGL(k_soft, dim3(gx), blk, 0, stream, c, w, B, io.shot_offset, p.lsat, p.tie_eps,
                           p.tie_lowest, (u64)p.seed, (u64)(t / p.soft_period), p.soft_shift);
    }
  }
  hipLaunchKernelGGL(k_output, dim3(gx), blk, 0, stream, c, w, B, p.lsat, io.corr, io.flags, io.post,
                     io.cut, io.iters);
  return hipGetLastError();
}

}  // namespace bpdc
