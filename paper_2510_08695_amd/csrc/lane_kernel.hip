// Fused persistent BP -> DC -> BP kernel, one shot per lane or per pair of
// lanes (gfx950, wave64).
//
// This source is compiled at plan-creation time with hipRTC, after the
// device helpers (bpdc_device.h) and a generated specification of one code:
// sizes (NB_*), lookup tables, and NB_SWEEP(), a straight-line sweep over the
// code's Tanner graph with every index a literal.  Everything a lane needs
// for its shot therefore lives in registers at fixed places:
//
//   per check ("slot") s : A1[s], A2[s] = alpha * (smallest, second smallest
//                 |q|); a field of W[] holding, per incident edge, the sign of
//                 the check-to-variable message r and a one-hot argmin bit;
//                 r = sign * (edge is argmin ? A2 : A1) (scaled min-sum);
//   per column ("row") i : the cut bit C[], and the posterior L written to
//                 LDS (sL, [row][65 lanes]) every sweep for DC and output.
//
// A shot is decoded by a group of NB_G adjacent lanes (1, 2 or 4): lane k of
// the group holds the images under an automorphism of the code of lane 0's
// checks and columns, and the edges that cross between lanes are exchanged
// with DPP quad permutations (see lane_spec.cpp).
//
// One sweep visits every row once: L = lambda + sum of r (ascending check
// order), the hard decision and the stop-test parity of each check (H e = s,
// Sec. II.C), then q = sat(L - r) and its contribution to the next check
// state (min, second min, argmin, sign parity).  A check's new state is
// completed ("finalised") at its last edge in the sweep, so one sweep is the
// variable half of iteration t and the check half of iteration t + 1
// (flooding schedule).  The first sweep of a pass starts from an all-zero
// check state, which makes L = lambda and q = sat(lambda), the first-iteration
// messages.
//
// A shot whose pass ends (converged, or T iterations) is handled by the whole
// wave: degeneracy cutting (Sec. III.A, one D row per lane, nominees OR-ed
// into LDS bitmasks), or output of the packed correction with one ballot per
// 64 columns; then its lane(s) take the next shot from a global counter.  The
// kernel is persistent: a wave exits when the counter is past the batch and
// all its lanes are idle.

struct LaneArgs {
  const unsigned* synp;           // [B][NB_G][NB_SPW] syndrome bits of each lane's slots (bpdc_lane_prepare)
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
  float lam_uniform;              // the prior LLR when all priors are equal
  int T1;
  int T2;
  int stop;
  int tie_lowest;
  unsigned long long seed;
  float a1_init;                  // alpha * lambda: check state after a first iteration (equal priors)
  float a2_init1;                 // alpha * lsat: its second minimum for a check of degree 1
  int skip0;                      // start first passes from that state (equal priors, 0 < lambda < lsat)
  unsigned long long* dcstats;    // DC diagnostics (NB_NSTAT words, accumulated) or null
  int soft_period;                // intermittent soft DC every soft_period first-pass iterations (NB_SOFT)
  float soft_shift;               // prior-LLR increase of each soft nominee (NB_SOFT)
};

// Posteriors in LDS as [column][shot slot of the wave], one slot per lane
// group (lane k's columns are lane 0's shifted by NB_LOFFk, so all lanes of a
// group store with the same offsets).  The odd strides keep column-wise reads
// free of bank conflicts.
#define NB_LSTR (64 / NB_G + 1)
// DC diagnostics (Appendix B): [0, 101) histogram of the spread of the
// first-pass posterior error probabilities over each row of D on shots that
// run DC, bin floor(100 spread); [101] number of such shots; [102, 103 + n)
// histogram of the cut size.
#define NB_NSTAT (103 + NB_N)
#ifndef NB_CHUNK
#define NB_CHUNK 16   // largest number of shots a wave claims at once
#endif

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
__device__ __forceinline__ float dec(float a1, float a2, u32 w, const int op, const int sp, u32 signmask) {
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

// Exchange with lane (lane xor J) of the same group of four: one DPP quad
// permutation (quad_perm [1,0,3,2], [2,3,0,1], [3,2,1,0]).  Every source
// lane of a quad permutation is valid and the sweep runs with all lanes
// enabled, so bound_ctrl (zero for invalid sources) never applies; it lets
// the compiler fold the permutation into the consuming VOP2 instruction
// (v_add_f32_dpp, v_sub_f32_dpp, v_xor_b32_dpp) instead of a separate move.
template <int J>
__device__ __forceinline__ u32 xchgu(u32 x) {
  constexpr int ctrl = J == 1 ? 0xB1 : (J == 2 ? 0x4E : 0x1B);
  return (u32)__builtin_amdgcn_mov_dpp((int)x, ctrl, 0xF, 0xF, true);
}
template <int J>
__device__ __forceinline__ float xchgf(float x) {
  return __uint_as_float(xchgu<J>(__float_as_uint(x)));
}

// Product-sum check output from the leave-one-out sum of phi(|q|): phi of the
// sum, saturated (an empty sum gives phi(0) = +inf, which becomes lsat),
// scaled, with the sign bit `neg`.
__device__ __forceinline__ float ps_r(float sum, u32 neg, float alpha, float lsat) {
  float mag = bpdc_dev::phi(sum);
  mag = (mag < lsat) ? mag : lsat;
  return __uint_as_float(__float_as_uint(alpha * mag) ^ (neg << 31));
}

// x of lane `src` (uniform across the wave) into scalar registers.
__device__ __forceinline__ long long readlane64(long long x, int src) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)x, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)((unsigned long long)x >> 32), src);
  return (long long)(((unsigned long long)hi << 32) | lo);
}
}  // namespace bpdc_lane

// Accumulate q into the next state of slot s (bit b): first event / later events.
#define NB_ACC0(s, q, b)                                       \
  {                                                            \
    const float a_ = fabsf(q);                                 \
    m1_##s = bpdc_lane::absmin(q, LS);                         \
    m2_##s = LS;                                               \
    am_##s = (a_ < LS) ? (1u << (b)) : 0u;                     \
    sb_##s = __float_as_uint(q) >> 31;                         \
  }
#define NB_ACC(s, q, b)                                        \
  {                                                            \
    const float a_ = fabsf(q);                                 \
    am_##s = (a_ < m1_##s) ? (1u << (b)) : am_##s;             \
    m2_##s = __builtin_amdgcn_fmed3f(a_, m1_##s, m2_##s);      \
    m1_##s = bpdc_lane::absmin(q, m1_##s);                     \
    sb_##s = __builtin_amdgcn_alignbit(sb_##s, __float_as_uint(q), 31); \
  }
// Stop-test parity of slot s: xor of its columns' hard decisions (bit 31 of
// ev), starting from the check's syndrome bit.
#define NB_EP0(s, ev) ep_##s = (ev) ^ (S[(s) >> 5] << (31 - ((s) & 31)))
#define NB_EP(s, ev) ep_##s ^= (ev)
// Product-sum rule (NB_PS, one lane per shot), in the log domain: an edge's
// register R[k] takes phi(|q|) once its column is swept, and the sign of q
// goes to bit b of the check's sign word; at the check's last edge NB_PSR
// forms each new r = sign * alpha * min(phi(sum of the other edges' values), lsat).
#define NB_PSACC0(s, k, b, q)                                  \
  {                                                            \
    R[k] = bpdc_dev::phi(fabsf(q));                            \
    sb_##s = (__float_as_uint(q) >> 31) << (b);                \
  }
#define NB_PSACC(s, k, b, q)                                   \
  {                                                            \
    R[k] = bpdc_dev::phi(fabsf(q));                            \
    sb_##s |= (__float_as_uint(q) >> 31) << (b);               \
  }
#define NB_PSR(sum, neg) bpdc_lane::ps_r((sum), (neg), alpha, LS)
// Complete slot s (degree d, field at bit `off` of W[cw]): r signs =
// s_c xor parity of all q signs xor own sign; stop-test parity into U.  Only
// bit 31 of ev, ep and U is meaningful: ep starts as the check's syndrome bit
// (placed at bit 31) xor its first column's hard decision.
#define NB_FIN(s, cw, off, d)                                               \
  {                                                                         \
    /* bit 0 of popcount + (S >> s) = parity of the q signs xor s_c */      \
    const u32 rs_ = (u32)__builtin_popcount(sb_##s) + (S[(s) >> 5] >> ((s) & 31)); \
    const u32 rm_ = (0u - (rs_ & 1u)) & ((1u << (d)) - 1u);                 \
    const u32 f_ = (am_##s << (d)) | (sb_##s ^ rm_);                        \
    const u32 fm_ = ((1u << (2 * (d))) - 1u) << (off);                      \
    W[cw] = (W[cw] & ~fm_) | (f_ << (off));                                 \
    A1[s] = alpha * m1_##s;                                                 \
    A2[s] = alpha * m2_##s;                                                 \
    U |= ep_##s;                                                            \
  }
#define NB_DEC(s, cw, op, sp) bpdc_lane::dec(A1[s], A2[s], W[cw], op, sp, SIGNMASK)
#define NB_CUT(L, i) L = bpdc_lane::cutsel(L, C[(i) >> 5], (i) & 31, INFBITS)
#define NB_STORE(v, L) myL[(v) * NB_LSTR] = (L)
// q = L - r without the clamp to [-lsat, lsat]: q enters the check state only
// through its sign bit and through min / median operations against minima
// that start at lsat, and clamping changes neither (|q| >= lsat leaves every
// minimum, argmin and second minimum as they are; the sign is kept).
#define NB_Q(L, r) ((L) - (r))
#define NB_XF0(x) (x)
#define NB_XF1(x) bpdc_lane::xchgf<1>(x)
#define NB_XF2(x) bpdc_lane::xchgf<2>(x)
#define NB_XF3(x) bpdc_lane::xchgf<3>(x)
#define NB_XU1(x) bpdc_lane::xchgu<1>(x)
#define NB_XU2(x) bpdc_lane::xchgu<2>(x)
#define NB_XU3(x) bpdc_lane::xchgu<3>(x)
// a on the lanes of a group whose index is in the bit mask, else b: one
// v_bfi_b32 with a per-lane mask register (kept in a vector register so that
// the conditions do not occupy scalar register pairs)
#define NB_SEL(mask, a, b) __uint_as_float(bpdc_lane::bfi(rolemask[mask], __float_as_uint(a), __float_as_uint(b)))

#if NB_UNIFORM_PRIOR
#define NB_LAM1(i) LAMU
#else
#define NB_LAM1(i) lamrow[i]
#endif
#if NB_SOFT
// soft DC: every pass reads the shot's own prior (shifted by soft DC in the
// first pass; the second pass's channel or posterior prior after DC)
#define NB_LAM(i, v) myLam2[(v) * NB_LSTR]
#elif NB_POSTERIOR
#define NB_LAM(i, v) (pass ? myLam2[(v) * NB_LSTR] : NB_LAM1(i))
#else
#define NB_LAM(i, v) NB_LAM1(i)
#endif

#ifdef NB_WAVES_PER_EU
#define NB_KATTR __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(NB_WAVES_PER_EU, NB_WAVES_PER_EU)))
#else
#define NB_KATTR __launch_bounds__(64, 1)
#endif
extern "C" __global__ void NB_KATTR bpdc_lane_kernel(LaneArgs a) {
  using namespace bpdc_lane;
  __shared__ float sL[NB_N * NB_LSTR];
#if NB_POSTERIOR || NB_SOFT
  __shared__ float sLam2[NB_N * NB_LSTR];  // per-shot prior: posterior second pass, or soft DC
#endif
  __shared__ short sDcolP[NB_MD * NB_DMAXROW];  // D rows, padded to the largest degree
#if !NB_DUNIFORM
  __shared__ unsigned char sDdeg[NB_MD];
#endif
  __shared__ u32 sCut[NB_G][NB_RC32];
  __shared__ short sColRow[NB_N];
  __shared__ u32 sSyn[NB_CHUNK][NB_G * NB_SPW];  // staged syndrome words of the reservoir
  __shared__ u32 sStat[NB_NSTAT];                 // this wave's DC diagnostics (when requested)
#if !NB_UNIFORM_PRIOR
  __shared__ float sLamRow[NB_G][NB_ROWS];
#endif

  const int lane = threadIdx.x;
  const int role = lane & (NB_G - 1);  // this lane's index in its shot's group
  const int first = lane & ~(NB_G - 1);
  for (int h = lane; h < NB_MD; h += 64) {
    const int b0 = a.d_row_ptr[h], deg = a.d_row_ptr[h + 1] - b0;
    for (int k = 0; k < NB_DMAXROW; ++k) sDcolP[h * NB_DMAXROW + k] = (short)(k < deg ? a.d_col[b0 + k] : 0);
#if !NB_DUNIFORM
    sDdeg[h] = (unsigned char)deg;
#endif
  }
  for (int i = lane; i < NB_N; i += 64) sColRow[i] = nb_col_row[i];
  for (int i = lane; i < NB_NSTAT; i += 64) sStat[i] = 0u;
#if !NB_UNIFORM_PRIOR
  for (int i = lane; i < NB_G * NB_ROWS; i += 64)
    sLamRow[i / NB_ROWS][i % NB_ROWS] = a.lam[nb_row_col[i / NB_ROWS][i % NB_ROWS]];
#endif
  __syncthreads();

  const int sid = lane / NB_G;  // this lane's shot slot in sL
  const int loff = role == 1 ? NB_LOFF1 : (role == 2 ? NB_LOFF2 : (role == 3 ? NB_LOFF3 : 0));
  // rolemask[m]: all ones on the lanes whose role is in the bit set m
  u32 rolemask[16];
#pragma unroll
  for (int m = 0; m < 16; ++m) asm("v_mov_b32 %0, %1" : "=v"(rolemask[m]) : "v"(0u - ((m >> role) & 1u)));
  float* myL = sL + sid + loff * NB_LSTR;
#if NB_POSTERIOR || NB_SOFT
  float* myLam2 = sLam2 + sid + loff * NB_LSTR;
#endif
  const float LS = a.lsat;
  const float alpha = a.alpha;
  // the uniform prior in a vector register (an asm copy the compiler cannot
  // fold back into a scalar operand): the first addition of a column then
  // takes an exchanged message as a DPP operand, which needs both sources in
  // vector registers
  float LAMU;
  asm volatile("v_mov_b32 %0, %1" : "=v"(LAMU) : "s"(a.lam_uniform));
  const float A1I = a.a1_init, A2I1 = a.a2_init1;
  const u32 SIGNMASK = 0x80000000u, INFBITS = 0x7F800000u;
  // lanes below the first lane of this lane's pair (for numbering new shots)
  const u64 below = (first == 0) ? 0ull : (~0ull >> (64 - first));
  const u64 leaders = NB_G == 4 ? 0x1111111111111111ull : (NB_G == 2 ? 0x5555555555555555ull : ~0ull);

#if NB_PS
  float R[NB_NR];  // per edge: r, or phi(|q|) once its column is swept
#else
  float A1[NB_SLOTS], A2[NB_SLOTS];
  u32 W[NB_NWC];
#endif
  u32 S[NB_SPW], C[NB_RC32];
  long long shot = -1;
  int t = 0, pass = 0, it1 = 0;
  bool want = true, dead = false;
  // the wave's reservoir of claimed shots (wave-uniform)
  long long rlo = 0, rhi = 0, sbase = 0, seen = 0;
  bool exhausted = false;

  for (;;) {
    // ---- take new shots for idle lanes (pairs) -----------------------------------------
    // Shots come from the wave's reservoir [rlo, rhi), a chunk of consecutive
    // shot indices claimed with one atomic, whose syndromes were staged in LDS
    // when it was claimed: a refill waits neither for the counter nor for
    // HBM.  The chunk shrinks as the batch runs out (a fraction of what was
    // left at the wave's last claim), so that few claimed shots are still
    // waiting when other waves already idle.
    long long nshot = -1;  // shot taken by this lane's group in this refill
    u32 nS[NB_SPW];
#pragma unroll
    for (int w = 0; w < NB_SPW; ++w) nS[w] = 0u;
    u64 need = __ballot(want && !dead) & leaders;
    while (need) {
      if (rlo == rhi) {
        if (exhausted) {
          if (want) {
            dead = true;
            shot = -1;
            want = false;
          }
          break;
        }
        const long long left = a.B - seen;
        long long c = left / (2 * (long long)gridDim.x);
        c = c < 1 ? 1 : (c > NB_CHUNK ? NB_CHUNK : c);
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(a.queue, (unsigned long long)c);
        // uniform across the wave: read from lane 0 into scalar registers
        const long long b0 = (long long)(((unsigned long long)__builtin_amdgcn_readfirstlane((int)(base >> 32)) << 32) |
                                         (unsigned)__builtin_amdgcn_readfirstlane((int)base));
        seen = b0 + c;
        if (b0 >= a.B) {
          exhausted = true;
          continue;
        }
        rlo = b0;
        rhi = b0 + c < a.B ? b0 + c : a.B;
        for (int i = lane; i < (rhi - rlo) * (NB_G * NB_SPW); i += 64)
          sSyn[i / (NB_G * NB_SPW)][i % (NB_G * NB_SPW)] = a.synp[rlo * (NB_G * NB_SPW) + i];
        __syncthreads();
        sbase = rlo;
      }
      const long long avail = rhi - rlo;
      if ((need >> first) & 1ull) {
        const long long rank = __popcll(need & below);
        if (rank < avail) {
          nshot = rlo + rank;
#pragma unroll
          for (int w = 0; w < NB_SPW; ++w) nS[w] = sSyn[nshot - sbase][role * NB_SPW + w];
          want = false;
        }
      }
      const long long cnt = __popcll(need);
      rlo += cnt < avail ? cnt : avail;
      need = __ballot(want && !dead) & leaders;
    }
    // the new shots' initial state, merged with selects rather than under a
    // branch, so that the state keeps its registers
    const bool fresh = nshot >= 0;
    if (__ballot(fresh)) {
#if NB_PS
#pragma unroll
      for (int k = 0; k < NB_NR; ++k) R[k] = fresh ? 0.0f : R[k];
      const int tn = 0;
#else
      float A1n[NB_SLOTS], A2n[NB_SLOTS];
      u32 Wn[NB_NWC];
      int tn;
#if NB_UNIFORM_PRIOR
      if (a.skip0) {
        // the first iteration's check half, written directly
#pragma unroll
        for (int s = 0; s < NB_SLOTS; ++s) { A1n[s] = A1[s]; A2n[s] = A2[s]; }
        NB_INIT1(Wn, A1n, A2n, nS);
        tn = 1;
      } else
#endif
      {
#pragma unroll
        for (int s = 0; s < NB_SLOTS; ++s) { A1n[s] = 0.0f; A2n[s] = 0.0f; }
#pragma unroll
        for (int w = 0; w < NB_NWC; ++w) Wn[w] = 0u;
        tn = 0;
      }
#pragma unroll
      for (int s = 0; s < NB_SLOTS; ++s) {
        A1[s] = fresh ? A1n[s] : A1[s];
        A2[s] = fresh ? A2n[s] : A2[s];
      }
#pragma unroll
      for (int w = 0; w < NB_NWC; ++w) W[w] = fresh ? Wn[w] : W[w];
#endif
#pragma unroll
      for (int w = 0; w < NB_SPW; ++w) S[w] = fresh ? nS[w] : S[w];
#pragma unroll
      for (int w = 0; w < NB_RC32; ++w) C[w] = fresh ? 0u : C[w];
      shot = fresh ? nshot : shot;
      t = fresh ? tn : t;
      pass = fresh ? 0 : pass;
      it1 = fresh ? 0 : it1;
    }
    if (__ballot(shot >= 0) == 0) break;
#if NB_SOFT
    // new shots start their first pass from the channel prior
    {
      u64 fm = __ballot(fresh) & leaders;
      while (fm) {
        const int src = __ffsll((long long)fm) - 1;
        const int ssid = src / NB_G;
        fm &= fm - 1;
        for (int u = lane; u < NB_N; u += 64) sLam2[u * NB_LSTR + ssid] = a.lam[u];
      }
      __syncthreads();
    }
#endif

    // ---- one sweep: variable half of iteration t, check half of iteration t+1 -----
#if !NB_UNIFORM_PRIOR
    // priors read from LDS through an offset the compiler cannot prove
    // constant, so that they are not hoisted out of the loop into registers
    int zoff;
    asm volatile("v_mov_b32 %0, 0" : "=v"(zoff));
    const float* lamrow = &sLamRow[role][0] + zoff;
#endif
    u32 U = 0u;
    NB_SWEEP();
#if NB_G >= 2
    U |= NB_XU1(U);
#endif
#if NB_G == 4
    U |= NB_XU2(U);
#endif

    const bool conv = (U >> 31) == 0u;
    const int T = pass ? a.T2 : a.T1;
    const bool done = (shot >= 0) && ((t >= 1 && a.stop && conv) || t >= T);
    const bool to_dc = done && pass == 0 && !conv;
    const bool finish = done && !to_dc;

    if (__ballot(done)) {
      // ---- degeneracy cutting for each shot whose first pass failed -------------------
      u64 dcm = __ballot(to_dc) & leaders;
      while (dcm) {
        const int src = __ffsll((long long)dcm) - 1;
        const int ssid = src / NB_G;
        dcm &= dcm - 1;
        const long long sshot = readlane64(shot, src);
        for (int w = lane; w < NB_G * NB_RC32; w += 64) sCut[w / NB_RC32][w % NB_RC32] = 0u;
        // nominees of rows lane, lane + 64, ...: all loads first, then the picks
        constexpr int kRowIt = (NB_MD + 63) / 64;
        int pick[kRowIt];
#pragma unroll
        for (int it = 0; it < kRowIt; ++it) {
          const int h = lane + 64 * it;
          pick[it] = -1;
          if (h < NB_MD) {
            int cols[NB_DMAXROW];
            float vals[NB_DMAXROW];
#pragma unroll
            for (int k = 0; k < NB_DMAXROW; ++k) {
              cols[k] = sDcolP[h * NB_DMAXROW + k];
              vals[k] = bpdc_dev::sat(sL[cols[k] * NB_LSTR + ssid], LS);
            }
#if NB_DUNIFORM
            const int deg = NB_DMAXROW;
#else
            const int deg = sDdeg[h];
#endif
            if (deg > 0) {
              pick[it] = bpdc_dev::dc_pick<NB_DMAXROW>(cols, vals, deg, a.tie_eps, a.tie_lowest, a.seed,
                                                       (u64)(a.shot_offset + sshot), (u64)h);
              if (a.dcstats) atomicAdd(&sStat[bpdc_dev::spread_bin<NB_DMAXROW>(vals, deg)], 1u);
            }
          }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kRowIt; ++it) {
          if (pick[it] >= 0) {
            const int pr = sColRow[pick[it]];
            atomicOr(&sCut[pr & 3][(pr >> 2) >> 5], 1u << ((pr >> 2) & 31));
          }
        }
        __syncthreads();
        if (a.dcstats && lane == 0) {
          int ncut = 0;
          for (int w = 0; w < NB_G * NB_RC32; ++w) ncut += __popc(sCut[w / NB_RC32][w % NB_RC32]);
          sStat[101] += 1u;
          sStat[102 + ncut] += 1u;
        }
#if NB_POSTERIOR
        for (int u = lane; u < NB_N; u += 64) {
          const int cr = sColRow[u];
          const int r = cr >> 2, hb = cr & 3;
          const bool cv = (sCut[hb][r >> 5] >> (r & 31)) & 1u;
          const float x = sL[u * NB_LSTR + ssid];
          sLam2[u * NB_LSTR + ssid] = cv ? __builtin_huge_valf() : bpdc_dev::sat(x, LS);
        }
#elif NB_SOFT
        // channel second pass: the unshifted prior (cut columns are +inf through C)
        for (int u = lane; u < NB_N; u += 64) sLam2[u * NB_LSTR + ssid] = a.lam[u];
#endif
        if (first == src) {
#pragma unroll
          for (int w = 0; w < NB_RC32; ++w) C[w] = sCut[role][w];
        }
        __syncthreads();
      }
      // ---- output of finished shots ---------------------------------------------------
      u64 fm = __ballot(finish) & leaders;
      while (fm) {
        const int src = __ffsll((long long)fm) - 1;
        const int ssid = src / NB_G;
        fm &= fm - 1;
        const long long sshot = readlane64(shot, src);
        const int spass = __builtin_amdgcn_readlane(pass, src);
        const bool sconv = __builtin_amdgcn_readlane((int)conv, src) != 0;
        const int st = __builtin_amdgcn_readlane(t, src);
        const int sit1 = __builtin_amdgcn_readlane(it1, src);
        float xs[NB_NW64];
#pragma unroll
        for (int w = 0; w < NB_NW64; ++w) {
          const int u = w * 64 + lane;
          xs[w] = (u < NB_N) ? sL[(u < NB_N ? u : 0) * NB_LSTR + ssid] : 1.0f;
        }
#pragma unroll
        for (int w = 0; w < NB_NW64; ++w) {
          const float x = xs[w];
          const u64 word = __ballot(x <= 0.0f);
          const u64 cword = __ballot(spass && x == __builtin_huge_valf());
          if (lane == 0) {
            a.corr[sshot * NB_NW64 + w] = word;
            if (a.cut) a.cut[sshot * NB_NW64 + w] = cword;
          }
        }
        if (lane == 0) {
          a.flags[sshot] = (unsigned char)((sconv ? 1 : 0) | (spass ? 2 : 0));
          if (a.iters) {
            a.iters[2 * sshot] = (short)(spass ? sit1 : st);
            a.iters[2 * sshot + 1] = (short)(spass ? st : 0);
          }
        }
        if (a.post) {
          for (int u = lane; u < NB_N; u += 64) {
            const float x = sL[u * NB_LSTR + ssid];
            a.post[sshot * NB_N + u] = (x == __builtin_huge_valf()) ? x : bpdc_dev::sat(x, LS);
          }
        }
      }
      // second pass from a zero check state (selects, as for new shots)
#if NB_PS
#pragma unroll
      for (int k = 0; k < NB_NR; ++k) R[k] = to_dc ? 0.0f : R[k];
#else
#pragma unroll
      for (int s = 0; s < NB_SLOTS; ++s) {
        A1[s] = to_dc ? 0.0f : A1[s];
        A2[s] = to_dc ? 0.0f : A2[s];
      }
#pragma unroll
      for (int w = 0; w < NB_NWC; ++w) W[w] = to_dc ? 0u : W[w];
#endif
      it1 = to_dc ? t : it1;
      pass = to_dc ? 1 : pass;
      t = to_dc ? -1 : t;
      shot = finish ? -1 : shot;
      want = want || finish;
    }
#if NB_SOFT
    // ---- intermittent soft DC: at t = K, 2K, ... of a first pass with H e != s
    // the rows of D nominate on this iteration's posteriors (the j-th
    // application hashes row h as j * rows(D) + h) and the nominees' priors
    // rise by soft_shift; the next sweep reads them ---------------------------------
    {
      const bool softnow = (shot >= 0) && !done && pass == 0 && !conv && t >= 1 && (t % a.soft_period) == 0;
      u64 sm = __ballot(softnow) & leaders;
      while (sm) {
        const int src = __ffsll((long long)sm) - 1;
        const int ssid = src / NB_G;
        sm &= sm - 1;
        const long long sshot = readlane64(shot, src);
        const int st = __builtin_amdgcn_readlane(t, src);
        const u64 rbase = (u64)(st / a.soft_period) * (u64)NB_MD;
        for (int w = lane; w < NB_G * NB_RC32; w += 64) sCut[w / NB_RC32][w % NB_RC32] = 0u;
        constexpr int kRowIt = (NB_MD + 63) / 64;
        int pick[kRowIt];
#pragma unroll
        for (int it = 0; it < kRowIt; ++it) {
          const int h = lane + 64 * it;
          pick[it] = -1;
          if (h < NB_MD) {
            int cols[NB_DMAXROW];
            float vals[NB_DMAXROW];
#pragma unroll
            for (int k = 0; k < NB_DMAXROW; ++k) {
              cols[k] = sDcolP[h * NB_DMAXROW + k];
              vals[k] = bpdc_dev::sat(sL[cols[k] * NB_LSTR + ssid], LS);
            }
#if NB_DUNIFORM
            const int deg = NB_DMAXROW;
#else
            const int deg = sDdeg[h];
#endif
            if (deg > 0)
              pick[it] = bpdc_dev::dc_pick<NB_DMAXROW>(cols, vals, deg, a.tie_eps, a.tie_lowest, a.seed,
                                                       (u64)(a.shot_offset + sshot), rbase + (u64)h);
          }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < kRowIt; ++it) {
          if (pick[it] >= 0) {
            const int pr = sColRow[pick[it]];
            atomicOr(&sCut[pr & 3][(pr >> 2) >> 5], 1u << ((pr >> 2) & 31));
          }
        }
        __syncthreads();
        for (int u = lane; u < NB_N; u += 64) {
          const int cr = sColRow[u];
          const int r = cr >> 2, hb = cr & 3;
          if ((sCut[hb][r >> 5] >> (r & 31)) & 1u) sLam2[u * NB_LSTR + ssid] = sLam2[u * NB_LSTR + ssid] + a.soft_shift;
        }
        __syncthreads();
      }
    }
#endif
    t += 1;
  }
  if (a.dcstats) {
    __syncthreads();
    for (int i = lane; i < NB_NSTAT; i += 64)
      if (sStat[i]) atomicAdd(&a.dcstats[i], (unsigned long long)sStat[i]);
  }
}

// Syndrome words of every shot in the order the lane kernel reads them
// (NB_PREP): [B][NB_G][NB_SPW], one thread per shot.
extern "C" __global__ void __launch_bounds__(256) bpdc_lane_prepare(const unsigned long long* syn, long long B,
                                                                    unsigned* synp) {
  const long long b = (long long)blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  unsigned s32[2 * NB_SW64];
#pragma unroll
  for (int x = 0; x < NB_SW64; ++x) {
    const unsigned long long v = syn[b * NB_SW64 + x];
    s32[2 * x] = (unsigned)v;
    s32[2 * x + 1] = (unsigned)(v >> 32);
  }
  unsigned out[NB_G * NB_SPW];
  NB_PREP(s32, out);
#pragma unroll
  for (int x = 0; x < NB_G * NB_SPW; ++x) synp[b * (NB_G * NB_SPW) + x] = out[x];
}
