// Fused persistent BP -> DC -> BP kernel, one shot per lane (gfx950, wave64).
//
// This source is compiled at plan-creation time with hipRTC, after the
// device helpers (bpdc_device.h) and a generated specification of one code:
// sizes (NB_*), and NB_SWEEP(), a straight-line sweep over the code's Tanner
// graph with every index a literal.  Everything a lane needs for its shot
// therefore lives in registers at fixed places:
//
//   per check c : A1[c], A2[c]  alpha * (smallest, second smallest |q|)
//                 a field of W[] holding, per incident edge, the sign of the
//                 check-to-variable message r and a one-hot argmin bit;
//                 r = sign * (edge is argmin ? A2 : A1) (scaled min-sum,
//                 the check rule of Sec. II.C);
//   per column  : the cut bit C[], and the posterior L written to LDS
//                 (sL, [column][65 lanes]) every sweep for DC and output.
//
// One sweep visits every column v once: L_v = lambda_v + sum_c r_{c->v}
// (ascending check order), the hard decision and the stop-test parity of
// each check (H e = s, Sec. II.C), then q_{v->c} = sat(L_v - r_{c->v}) and
// its contribution to the next check state of c (min, second min, argmin,
// sign parity).  A check's new state is completed ("finalised") at its last
// edge in the sweep, so one sweep is the variable half of iteration t and the
// check half of iteration t + 1 (flooding schedule).  The very first sweep of
// a pass starts from an all-zero check state, which makes L = lambda and
// q = sat(lambda), the first-iteration messages.
//
// Lanes are independent shots; a lane whose pass ends (converged, or T
// iterations) is handled by the whole wave: degeneracy cutting (Sec. III.A,
// one D row per lane, nominees OR-ed into an LDS bitmask), or output of the
// packed correction with one ballot per 64 columns; then the lane takes the
// next shot from a global counter.  The kernel is persistent: a wave exits
// when the counter is past the batch and all its lanes are idle.

struct LaneArgs {
  const unsigned long long* syn;  // [B][NB_SW64]
  long long B;
  long long shot_offset;
  unsigned long long* corr;       // [B][NB_NW64]
  unsigned char* flags;           // [B]
  float* post;                    // [B][NB_N] or null
  unsigned long long* cut;        // [B][NB_NW64] or null
  short* iters;                   // [B][2] or null
  const float* lam;               // [NB_N] prior LLRs
  const int* d_row_ptr;           // [NB_MD + 1]
  const int* d_col;               // [NB_DNNZ]
  unsigned long long* queue;      // next shot counter (zeroed before launch)
  float alpha;
  float lsat;
  float tie_eps;
  int T1;
  int T2;
  int stop;
  int tie_lowest;
  int pad_;
  unsigned long long seed;
};

#define NB_STRIDE 65  // LDS row stride (floats) of the [column][lane] posterior array

namespace bpdc_lane {
using bpdc_dev::u32;
using bpdc_dev::u64;

// min(|q|, m) as one VOP3 instruction with an abs source modifier.
__device__ __forceinline__ float absmin(float q, float m) {
  float r;
  asm("v_min_f32_e64 %0, |%1|, %2" : "=v"(r) : "v"(q), "v"(m));
  return r;
}

// Bitwise select (mask & a) | (~mask & b) as one v_bfi_b32 (the compiler
// otherwise splits it into compares and selects when mask is 0 / -1).
__device__ __forceinline__ u32 bfi(u32 mask, u32 a, u32 b) {
  u32 r;
  asm("v_bfi_b32 %0, %1, %2, %3" : "=v"(r) : "v"(mask), "v"(a), "v"(b));
  return r;
}

// r for the edge slot whose one-hot argmin bit is `op` and whose sign bit is
// `sp` in the check field word w: magnitude A2 if the edge holds the
// minimum, else A1; sign from the field.
__device__ __forceinline__ float dec(float a1, float a2, u32 w, const int op, const int sp,
                                     u32 signmask) {
  const u32 mask = (u32)__builtin_amdgcn_sbfe((int)w, op, 1);
  const u32 mag = bfi(mask, __float_as_uint(a2), __float_as_uint(a1));
  return __uint_as_float(bfi(signmask, w << (31 - sp), mag));
}

// A cut column has prior probability 0: its posterior is +inf, so its
// messages saturate at +lsat and its hard decision is 0 (Algorithm 2).
__device__ __forceinline__ float cutsel(float L, u32 cw, const int b, u32 infbits) {
  const u32 mask = (u32)__builtin_amdgcn_sbfe((int)cw, b, 1);
  return __uint_as_float(bfi(mask, infbits, __float_as_uint(L)));
}
}  // namespace bpdc_lane

// Accumulate q into the next state of check c (slot bit b): first slot / later slots.
#define NB_ACC0(c, q, ev, b)                                   \
  {                                                            \
    const float a_ = fabsf(q);                                 \
    m1_##c = bpdc_lane::absmin(q, LS);                         \
    m2_##c = LS;                                               \
    am_##c = (a_ < LS) ? (1u << (b)) : 0u;                     \
    sb_##c = __float_as_uint(q) >> 31;                         \
    ep_##c = (ev);                                             \
  }
#define NB_ACC(c, q, ev, b)                                    \
  {                                                            \
    const float a_ = fabsf(q);                                 \
    am_##c = (a_ < m1_##c) ? (1u << (b)) : am_##c;             \
    m2_##c = __builtin_amdgcn_fmed3f(a_, m1_##c, m2_##c);      \
    m1_##c = bpdc_lane::absmin(q, m1_##c);                     \
    sb_##c = __builtin_amdgcn_alignbit(sb_##c, __float_as_uint(q), 31); \
    ep_##c ^= (ev);                                            \
  }
// Complete check c (degree d, field at bit `off` of W[cw]): r signs =
// s_c xor parity of all q signs xor own sign; stop-test parity into U.
#define NB_FIN(c, cw, off, d)                                               \
  {                                                                         \
    const u32 sc_ = __builtin_amdgcn_ubfe(S[(c) >> 5], (c) & 31, 1);        \
    const u32 rs_ = ((u32)__builtin_popcount(sb_##c) ^ sc_) & 1u;          \
    const u32 rm_ = (0u - rs_) & ((1u << (d)) - 1u);                        \
    const u32 f_ = (am_##c << (d)) | (sb_##c ^ rm_);                        \
    const u32 fm_ = ((1u << (2 * (d))) - 1u) << (off);                      \
    W[cw] = (W[cw] & ~fm_) | (f_ << (off));                                 \
    A1[c] = alpha * m1_##c;                                                 \
    A2[c] = alpha * m2_##c;                                                 \
    U |= ep_##c ^ (sc_ << 31);                                              \
  }
#define NB_DEC(c, cw, op, sp) bpdc_lane::dec(A1[c], A2[c], W[cw], op, sp, SIGNMASK)
#define NB_CUT(L, v) L = bpdc_lane::cutsel(L, C[(v) >> 5], (v) & 31, INFBITS)
#define NB_STORE(v, L) myL[(v) * NB_STRIDE] = (L)
#define NB_Q(L, r) bpdc_dev::sat((L) - (r), LS)

#if NB_POSTERIOR
#define NB_LAM(v) (pass ? myLam2[(v) * NB_STRIDE] : lamp[v])
#else
#define NB_LAM(v) (lamp[v])
#endif


extern "C" __global__ void __launch_bounds__(64, 1) bpdc_lane_kernel(LaneArgs a) {
  using namespace bpdc_lane;
  __shared__ float sL[NB_N * NB_STRIDE];
#if NB_POSTERIOR
  __shared__ float sLam2[NB_N * NB_STRIDE];
#endif
  __shared__ int sDptr[NB_MD + 1];
  __shared__ short sDcol[NB_DNNZ];
  __shared__ u32 sCut[NB_NC32];
  __shared__ float sLam[NB_N];

  const int lane = threadIdx.x;
  for (int i = lane; i <= NB_MD; i += 64) sDptr[i] = a.d_row_ptr[i];
  for (int i = lane; i < NB_DNNZ; i += 64) sDcol[i] = (short)a.d_col[i];
  for (int i = lane; i < NB_N; i += 64) sLam[i] = a.lam[i];
  __syncthreads();

  float* myL = sL + lane;
#if NB_POSTERIOR
  float* myLam2 = sLam2 + lane;
#endif
  const u32 SIGNMASK = 0x80000000u, INFBITS = 0x7F800000u;
  const float LS = a.lsat;
  const float alpha = a.alpha;
  const u64 below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  float A1[NB_M], A2[NB_M];
  u32 W[NB_NWC], S[NB_SW32], C[NB_NC32];
  long long shot = -1;
  int t = 0, pass = 0, it1 = 0;
  bool want = true, dead = false;

  for (;;) {
    // ---- take new shots for idle lanes --------------------------------------------
    const u64 need = __ballot(want && !dead);
    if (need) {
      const int leader = __ffsll((long long)need) - 1;
      unsigned long long base = 0;
      if (lane == leader) base = atomicAdd(a.queue, (unsigned long long)__popcll(need));
      base = __shfl(base, leader);
      if (want && !dead) {
        const long long my = (long long)base + __popcll(need & below);
        if (my < a.B) {
          shot = my;
          const unsigned long long* sp = a.syn + my * NB_SW64;
#pragma unroll
          for (int w = 0; w < NB_SW32; ++w) {
            const unsigned long long x = sp[w >> 1];
            S[w] = (w & 1) ? (u32)(x >> 32) : (u32)x;
          }
#pragma unroll
          for (int c = 0; c < NB_M; ++c) { A1[c] = 0.0f; A2[c] = 0.0f; }
#pragma unroll
          for (int w = 0; w < NB_NWC; ++w) W[w] = 0u;
#pragma unroll
          for (int w = 0; w < NB_NC32; ++w) C[w] = 0u;
          t = 0;
          pass = 0;
          it1 = 0;
        } else {
          dead = true;
          shot = -1;
        }
        want = false;
      }
    }
    if (__ballot(shot >= 0) == 0) break;

    // ---- one sweep: variable half of iteration t, check half of iteration t+1 -----
    // Priors are read from LDS (a broadcast read per column) through an offset
    // the compiler cannot prove constant, so that they are not hoisted out of
    // the loop into n registers.
    int zoff;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zoff));
    const float* lamp = sLam + zoff;
    u32 U = 0u;
    NB_SWEEP();

    const bool conv = (U >> 31) == 0u;
    const int T = pass ? a.T2 : a.T1;
    const bool done = (shot >= 0) && ((t >= 1 && a.stop && conv) || t >= T);
    const bool to_dc = done && pass == 0 && !conv;
    const bool finish = done && !to_dc;

    if (__ballot(done)) {
      // ---- degeneracy cutting for each lane whose first pass failed -------------------
      u64 dcm = __ballot(to_dc);
      while (dcm) {
        const int src = __ffsll((long long)dcm) - 1;
        dcm &= dcm - 1;
        const long long sshot = __shfl(shot, src);
        for (int w = lane; w < NB_NC32; w += 64) sCut[w] = 0u;
        __syncthreads();
        for (int h = lane; h < NB_MD; h += 64) {
          const int b0 = sDptr[h], deg = sDptr[h + 1] - b0;
          int cols[NB_DMAXROW];
          float vals[NB_DMAXROW];
          for (int k = 0; k < deg; ++k) {
            cols[k] = sDcol[b0 + k];
            vals[k] = bpdc_dev::sat(sL[cols[k] * NB_STRIDE + src], LS);
          }
          if (deg > 0) {
            const int pick = bpdc_dev::dc_pick<NB_DMAXROW>(cols, vals, deg, a.tie_eps, a.tie_lowest,
                                                           a.seed, (u64)(a.shot_offset + sshot), (u64)h);
            atomicOr(&sCut[pick >> 5], 1u << (pick & 31));
          }
        }
        __syncthreads();
#if NB_POSTERIOR
        for (int v = lane; v < NB_N; v += 64) {
          const bool cv = (sCut[v >> 5] >> (v & 31)) & 1u;
          sLam2[v * NB_STRIDE + src] = cv ? __builtin_huge_valf() : bpdc_dev::sat(sL[v * NB_STRIDE + src], LS);
        }
#endif
        if (lane == src) {
#pragma unroll
          for (int w = 0; w < NB_NC32; ++w) C[w] = sCut[w];
        }
        __syncthreads();
      }
      // ---- output of finished shots ---------------------------------------------------
      u64 fm = __ballot(finish);
      while (fm) {
        const int src = __ffsll((long long)fm) - 1;
        fm &= fm - 1;
        const long long sshot = __shfl(shot, src);
#pragma unroll
        for (int w = 0; w < NB_NW64; ++w) {
          const int v = w * 64 + lane;
          const bool e = (v < NB_N) && (sL[v * NB_STRIDE + src] <= 0.0f);
          const u64 word = __ballot(e);
          if (lane == 0) a.corr[sshot * NB_NW64 + w] = word;
        }
        const int spass = __shfl(pass, src);
        const bool sconv = __shfl((int)conv, src) != 0;
        const int st = __shfl(t, src);
        const int sit1 = __shfl(it1, src);
        if (lane == 0) {
          a.flags[sshot] = (unsigned char)((sconv ? 1 : 0) | (spass ? 2 : 0));
          if (a.iters) {
            a.iters[2 * sshot] = (short)(spass ? sit1 : st);
            a.iters[2 * sshot + 1] = (short)(spass ? st : 0);
          }
        }
        if (a.cut) {
#pragma unroll
          for (int w = 0; w < NB_NW64; ++w) {
            const u32 lo = (2 * w < NB_NC32) ? __shfl(C[(2 * w < NB_NC32) ? 2 * w : 0], src) : 0u;
            const u32 hi = (2 * w + 1 < NB_NC32) ? __shfl(C[(2 * w + 1 < NB_NC32) ? 2 * w + 1 : 0], src) : 0u;
            if (lane == 0) a.cut[sshot * NB_NW64 + w] = spass ? (((u64)hi << 32) | lo) : 0ull;
          }
        }
        if (a.post) {
          for (int v = lane; v < NB_N; v += 64) {
            const float x = sL[v * NB_STRIDE + src];
            a.post[sshot * NB_N + v] = (x == __builtin_huge_valf()) ? x : bpdc_dev::sat(x, LS);
          }
        }
      }
      if (to_dc) {
#pragma unroll
        for (int c = 0; c < NB_M; ++c) { A1[c] = 0.0f; A2[c] = 0.0f; }
#pragma unroll
        for (int w = 0; w < NB_NWC; ++w) W[w] = 0u;
        it1 = t;
        pass = 1;
        t = -1;
      }
      if (finish) {
        shot = -1;
        want = true;
      }
    }
    t += 1;
  }
}
