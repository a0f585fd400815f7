// Weighted min-sum BP+DC with learned per-edge scales, and its adjoint.
//
// Forward: the decoder of the other kernels with r_e = sign * (w_e * min of
// the other |q|) and a separate scale vector per pass (before / after
// degeneracy cutting), always T iterations per pass (unrolled, no early
// stop).  Every K iterations the state of each check is stored as a
// checkpoint: the smallest and second smallest |q| over its row, their
// positions, the signs of its q and the parity of those signs with the
// syndrome bit (12 bytes per check).  That state determines every r of the
// iteration, so a checkpoint restarts the decoder exactly.
//
// Backward: for each shot and pass, from the last checkpoint segment to the
// first, the check states of the segment's iterations are recomputed from its
// checkpoint and then walked in reverse:
//   L_v = prior_v + sum_e r_e,   q_e = sat(L_v - r_e)      (linear, 0 where saturated)
//   r_e = sigma_e * w_e * |q_e*|  with e* the edge holding the minimum over
//         the other edges of the check (the second minimum for the argmin
//         edge), sigma_e the sign (syndrome bit times the other signs, locally
//         constant):  dr_e/dw_e = sigma_e |q_e*|,  dr_e/dq_e* = sigma_e w_e sgn(q_e*),
// so a check passes gradient back to two of its edges only: the argmin (from
// every other edge) and the second argmin (from the argmin edge).  The cut set
// is held fixed (a function of the first pass, not differentiated), and with
// the channel prior the second pass depends on the first only through the
// cut, so each pass's gradient comes from its own posteriors (a shot without
// DC reports its first-pass posteriors in both rows, so its first pass takes
// the gradient of both).
//
// Layout: one wave decodes one shot at a time (no workgroup barrier inside
// the decode: the lanes of a wave step together, and LDS traffic within a
// wave is ordered by a wavefront fence); a workgroup holds several waves,
// which share the code's index tables and both scale vectors, staged in LDS
// once.  Per wave, the messages live in one per-edge array updated in place
// (the check phase turns a row's q into its r, the variable phase a column's
// r into its q: every edge belongs to one row and one column).  Lanes own
// checks c = lane + 64 k in the check phase and columns v = lane + 64 k in
// the variable phase.  Weight gradients are summed per workgroup in LDS
// (float atomics) and added to the output once per workgroup.
#include <algorithm>
#include <cstdlib>

#include "internal.h"
// after the HIP runtime header: bpdc_device.h itself includes nothing
#include "bpdc_device.h"

namespace bpdc {

namespace {

using bpdc_dev::u32;
using bpdc_dev::u64;

constexpr u32 kNone = 31u;  // position field of a check state: no such edge

// Device-side view of a code (global memory).
struct WCode {
  int n, m, md, E, dnnz;
  const int32_t* rp;    // H CSR row pointer [m + 1]
  const int32_t* col;   // H CSR columns [E]
  const int32_t* cp;    // CSC column pointer [n + 1]
  const int32_t* ce;    // CSC -> CSR edge ids [E] (ascending rows)
  const int32_t* erow;  // row of each CSR edge [E]
  const int32_t* drp;   // D CSR row pointer [md + 1]
  const int32_t* dcol;  // D CSR columns [dnnz]
  const float* lam;     // prior LLRs [n]
};

// The code's tables and the scales of both passes in LDS (shared by the waves
// of a workgroup).
struct WTab {
  int32_t* rp;   // [m + 1]
  int32_t* cp;   // [n + 1]
  int32_t* ce;   // [E]
  int32_t* col;  // [E] (forward: stop test)
  int32_t* drp;  // [md + 1] (forward: DC)
  int32_t* dcol; // [dnnz] (forward: DC)
  float* w;      // [2][E]
  float* lam;    // [n]
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// Bytes of the shared tables; `forward` adds the stop-test and DC tables.
__host__ __device__ inline size_t wtab_bytes(int n, int m, int md, int E, int dnnz, bool forward) {
  size_t b = align16((size_t)(m + 1) * 4) + align16((size_t)(n + 1) * 4) + align16((size_t)E * 4) +
             align16((size_t)2 * E * 4) + align16((size_t)n * 4);
  if (forward) b += align16((size_t)E * 4) + align16((size_t)(md + 1) * 4) + align16((size_t)std::max(dnnz, 1) * 4);
  return b;
}

__device__ WTab carve_tab(unsigned char* base, const WCode& C, bool forward) {
  WTab t;
  unsigned char* p = base;
  auto take = [&](size_t bytes) {
    unsigned char* q = p;
    p += align16(bytes);
    return q;
  };
  t.rp = (int32_t*)take((size_t)(C.m + 1) * 4);
  t.cp = (int32_t*)take((size_t)(C.n + 1) * 4);
  t.ce = (int32_t*)take((size_t)C.E * 4);
  t.w = (float*)take((size_t)2 * C.E * 4);
  t.lam = (float*)take((size_t)C.n * 4);
  if (forward) {
    t.col = (int32_t*)take((size_t)C.E * 4);
    t.drp = (int32_t*)take((size_t)(C.md + 1) * 4);
    t.dcol = (int32_t*)take((size_t)std::max(C.dnnz, 1) * 4);
  } else {
    t.col = t.drp = t.dcol = nullptr;
  }
  return t;
}

// All threads of the workgroup copy the tables, then one workgroup barrier
// (before any per-wave work, reached by every thread).
__device__ void load_tab(const WTab& t, const WCode& C, const float* w, bool forward) {
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = tid; i <= C.m; i += nt) t.rp[i] = C.rp[i];
  for (int i = tid; i <= C.n; i += nt) t.cp[i] = C.cp[i];
  for (int k = tid; k < C.E; k += nt) t.ce[k] = C.ce[k];
  for (int i = tid; i < 2 * C.E; i += nt) t.w[i] = w[i];
  for (int i = tid; i < C.n; i += nt) t.lam[i] = C.lam[i];
  if (forward) {
    for (int i = tid; i < C.E; i += nt) t.col[i] = C.col[i];
    for (int i = tid; i <= C.md; i += nt) t.drp[i] = C.drp[i];
    for (int i = tid; i < C.dnnz; i += nt) t.dcol[i] = C.dcol[i];
  }
  __syncthreads();
}

// Order the LDS accesses of one wave (its lanes execute in lockstep; the
// fences keep the compiler from moving LDS operations across the point).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// State of one check in one iteration (computed from the q of the previous
// iteration): |q| minima and the bits
//   [0, 5) position of the minimum in the row (kNone: every |q| >= lsat),
//   [5, 10) position of the second minimum (kNone: none below lsat),
//   [10] parity of the syndrome bit and the q signs, [11, 32) q sign bits.
struct __align__(16) CState {
  float m1, m2;
  u32 bits, pad;
};

__device__ __forceinline__ u32 cs_a1(u32 bits) { return bits & 31u; }
__device__ __forceinline__ u32 cs_a2(u32 bits) { return (bits >> 5) & 31u; }
__device__ __forceinline__ u32 cs_neg(u32 bits) { return (bits >> 10) & 1u; }
__device__ __forceinline__ u32 cs_qsign(u32 bits, int k) { return (bits >> (11 + k)) & 1u; }

// r of the edge at row position k of a check (scale w): w * (min2 on the
// argmin edge, min1 elsewhere), negative iff the parity of the syndrome bit
// and the other signs is odd.
__device__ __forceinline__ float cs_r(const CState& s, int k, float w) {
  const float mag = ((u32)k == cs_a1(s.bits)) ? s.m2 : s.m1;
  const float val = w * mag;
  return (cs_neg(s.bits) ^ cs_qsign(s.bits, k)) ? -val : val;
}

// Check state from the q of a row (strict '<' in row order: the first
// minimum wins; minima start at lsat).  RDM bounds the row degree: the row's
// loads are issued together.
template <int RDM>
__device__ __forceinline__ CState check_state(const float* msg, int e0, int deg, u32 sbit, float lsat) {
  float q[RDM];
#pragma unroll
  for (int k = 0; k < RDM; ++k)
    if (k < deg) q[k] = msg[e0 + k];
  float m1 = lsat, m2 = lsat;
  u32 a1 = kNone, a2 = kNone, neg = sbit, qs = 0u;
#pragma unroll
  for (int k = 0; k < RDM; ++k)
    if (k < deg) {
      const float a = fabsf(q[k]);
      const u32 sg = (q[k] < 0.0f) ? 1u : 0u;
      neg ^= sg;
      qs |= sg << k;
      if (a < m1) {
        m2 = m1;
        a2 = a1;
        m1 = a;
        a1 = (u32)k;
      } else if (a < m2) {
        m2 = a;
        a2 = (u32)k;
      }
    }
  CState s;
  s.m1 = m1;
  s.m2 = m2;
  s.bits = a1 | (a2 << 5) | (neg << 10) | (qs << 11);
  s.pad = 0u;
  return s;
}

// The r of every edge of a row from its state, in place of the row's messages.
template <int RDM>
__device__ __forceinline__ void write_r(float* msg, const float* wp, int e0, int deg, const CState& st) {
  float w[RDM];
#pragma unroll
  for (int k = 0; k < RDM; ++k)
    if (k < deg) w[k] = wp[e0 + k];
#pragma unroll
  for (int k = 0; k < RDM; ++k)
    if (k < deg) msg[e0 + k] = cs_r(st, k, w[k]);
}

struct WArgs {
  WCode C;
  const uint64_t* syn;
  int64_t B;
  int64_t shot_offset;
  int K, nck1, nck2;
  const float* w;          // [2][E]
  float* post;             // [2][B][n] (forward)
  uint64_t* cut;           // [B][ceil(n/64)] (forward: out; backward: in)
  uint8_t* flags;          // [B] (forward: out; backward: in)
  float* ck_m1;            // checkpoints: three planes [pass-major shot-slot][m] (see ck_index)
  float* ck_m2;
  u32* ck_bits;
  const float* gpost;      // [2][B][n] (backward)
  float* gw;               // [2][E] (backward, accumulated)
  size_t wave_bytes;       // per-wave LDS
  size_t tab_bytes;        // shared LDS (tables; backward: + weight-gradient sums)
  KParams p;
};

// Row of checkpoint j of shot b in pass `pass` in the checkpoint planes.
__device__ __forceinline__ size_t ck_index(const WArgs& a, int pass, int64_t b, int j) {
  return pass ? ((size_t)a.B * a.nck1 + (size_t)b * a.nck2 + j) : ((size_t)b * a.nck1 + j);
}

// DC nomination of one row of D (bpdc_device.h's rule, streamed from the
// tables): the row maximum of the saturated posteriors, the tie threshold,
// the number of ties, then the chosen tie in ascending column order.
__device__ int wms_dc_pick(const int32_t* dcol, int e0, int deg, const float* L, float lsat, float tie_eps,
                           int tie_lowest, u64 seed, u64 shot, u64 row) {
  float lmax = bpdc_dev::sat(L[dcol[e0]], lsat);
  for (int k = 1; k < deg; ++k) lmax = fmaxf(lmax, bpdc_dev::sat(L[dcol[e0 + k]], lsat));
  const float scale = fmaxf(1.0f, fabsf(lmax));
  const float thr = lmax - tie_eps * scale;
  int nt = 0;
  for (int k = 0; k < deg; ++k) nt += (bpdc_dev::sat(L[dcol[e0 + k]], lsat) >= thr) ? 1 : 0;
  int want = 0;
  if (!tie_lowest && nt > 1) want = (int)bpdc_dev::scale_draw(bpdc_dev::tie_hash(seed, shot, row), (u32)nt);
  int seen = 0;
  for (int k = 0; k < deg; ++k) {
    const int c = dcol[e0 + k];
    if (bpdc_dev::sat(L[c], lsat) >= thr) {
      if (seen == want) return c;
      ++seen;
    }
  }
  return dcol[e0];
}

// CDM, RDM: bounds on the column and row degrees (a column's or row's edge ids
// and messages stay in registers, and its loads are issued together).
template <int CDM, int RDM>
__global__ void __launch_bounds__(512) k_wms_forward(WArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const WCode& C = a.C;
  const WTab tb = carve_tab(smem, C, true);
  load_tab(tb, C, a.w, true);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int n = C.n, m = C.m, E = C.E;
  const int nwc = (n + 31) >> 5, swc = (m + 31) >> 5;
  const int sw64 = (m + 63) >> 6, nw64 = (n + 63) >> 6;
  unsigned char* mine = smem + a.tab_bytes + (size_t)wave * a.wave_bytes;
  float* msg = (float*)mine;                              // [E]
  float* L = msg + E;                                     // [n]
  u32* cutw = (u32*)(L + n);                              // [nwc]
  u32* synw = cutw + nwc;                                 // [swc]
  const float LS = a.p.lsat, INF = __builtin_huge_valf();
  const int K = a.K;

  for (int64_t b = (int64_t)blockIdx.x * nwaves + wave; b < a.B; b += (int64_t)gridDim.x * nwaves) {
    for (int i = lane; i < swc; i += 64) {
      const uint64_t x = a.syn[b * sw64 + (i >> 1)];
      synw[i] = (i & 1) ? (u32)(x >> 32) : (u32)x;
    }
    for (int i = lane; i < nwc; i += 64) cutw[i] = 0u;
    wave_sync();
    bool conv = false;
    int pass = 0;
    for (; pass < 2; ++pass) {
      const int T = pass ? a.p.T2 : a.p.T1;
      const float* wp = tb.w + (size_t)pass * E;
      // first-iteration q: the prior, +lsat on cut columns
      for (int v = lane; v < n; v += 64) {
        const bool cv = (cutw[v >> 5] >> (v & 31)) & 1u;
        const float q0 = cv ? LS : bpdc_dev::sat(tb.lam[v], LS);
        for (int k = tb.cp[v]; k < tb.cp[v + 1]; ++k) msg[tb.ce[k]] = q0;
      }
      wave_sync();
      for (int t = 1; t <= T; ++t) {
        const bool save = ((t - 1) % K) == 0;
        const int j = (t - 1) / K;
        // check phase: r of every edge of the row (in place of its q)
        for (int c = lane; c < m; c += 64) {
          const int e0 = tb.rp[c], deg = tb.rp[c + 1] - e0;
          const CState s = check_state<RDM>(msg, e0, deg, (synw[c >> 5] >> (c & 31)) & 1u, LS);
          if (save) {
            const size_t row = ck_index(a, pass, b, j) * (size_t)m + c;
            a.ck_m1[row] = s.m1;
            a.ck_m2[row] = s.m2;
            a.ck_bits[row] = s.bits;
          }
          write_r<RDM>(msg, wp, e0, deg, s);
        }
        wave_sync();
        // variable phase: L = prior + sum r (ascending rows), q = sat(L - r)
        for (int v = lane; v < n; v += 64) {
          const int k0 = tb.cp[v], deg = tb.cp[v + 1] - k0;
          const bool cv = (cutw[v >> 5] >> (v & 31)) & 1u;
          int ee[CDM];
          float rr[CDM];
#pragma unroll
          for (int j = 0; j < CDM; ++j)
            if (j < deg) {
              ee[j] = tb.ce[k0 + j];
              rr[j] = msg[ee[j]];
            }
          float Lv = tb.lam[v];
#pragma unroll
          for (int j = 0; j < CDM; ++j)
            if (j < deg) Lv = Lv + rr[j];
#pragma unroll
          for (int j = 0; j < CDM; ++j)
            if (j < deg) msg[ee[j]] = cv ? LS : bpdc_dev::sat(Lv - rr[j], LS);
          L[v] = cv ? INF : Lv;
        }
        wave_sync();
      }
      float* pp = a.post + ((size_t)pass * a.B + b) * n;
      for (int v = lane; v < n; v += 64) pp[v] = (L[v] == INF) ? INF : bpdc_dev::sat(L[v], LS);
      // stop test H e = s with e = [L <= 0]
      int bad = 0;
      for (int c = lane; c < m; c += 64) {
        u32 par = (synw[c >> 5] >> (c & 31)) & 1u;
        for (int e = tb.rp[c]; e < tb.rp[c + 1]; ++e) par ^= (L[tb.col[e]] <= 0.0f) ? 1u : 0u;
        bad |= (int)par;
      }
      conv = __ballot(bad) == 0ull;
      if (pass == 1 || conv) break;
      // degeneracy cutting on the first-pass posteriors
      for (int h = lane; h < C.md; h += 64) {
        const int e0 = tb.drp[h], deg = tb.drp[h + 1] - e0;
        if (deg == 0) continue;
        const int pick = wms_dc_pick(tb.dcol, e0, deg, L, LS, a.p.tie_eps, a.p.tie_lowest, a.p.seed,
                                     (u64)(a.shot_offset + b), (u64)h);
        atomicOr(&cutw[pick >> 5], 1u << (pick & 31));
      }
      wave_sync();
    }
    const bool dc = pass == 1;
    if (!dc) {  // second-pass rows of shots without DC are copies of the first pass
      const float* p0 = a.post + (size_t)b * n;
      float* p1 = a.post + ((size_t)a.B + b) * n;
      for (int v = lane; v < n; v += 64) p1[v] = p0[v];
    }
    for (int i = lane; i < nw64; i += 64) {
      const u32 lo = cutw[2 * i];
      const u32 hi = (2 * i + 1 < nwc) ? cutw[2 * i + 1] : 0u;
      a.cut[b * nw64 + i] = dc ? (((u64)hi << 32) | lo) : 0ull;
    }
    if (lane == 0) a.flags[b] = (uint8_t)((conv ? 1 : 0) | (dc ? 2 : 0));
    wave_sync();
  }
}

__device__ __forceinline__ float sgn_of(float mag, u32 sign) {
  // sign of a q from its magnitude (a minimum over the row) and sign bit: 0 at q = 0
  return mag == 0.0f ? 0.0f : (sign ? -1.0f : 1.0f);
}

// At most 128 VGPRs: four waves per SIMD, as many as the per-wave LDS state
// lets stay resident anyway.  SEG: checkpoints every K > 1 iterations (each
// segment recomputed from its checkpoint); without, one checkpoint per
// iteration, read back directly, the next one's loads issued before the
// current iteration is reversed (codes of at most 128 checks: two rows per
// lane in registers).
template <int CDM, int RDM, bool SEG>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) k_wms_backward(WArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const WCode& C = a.C;
  const WTab tb = carve_tab(smem, C, false);
  const int n = C.n, m = C.m, E = C.E;
  float* gws = (float*)(smem + wtab_bytes(n, m, C.md, E, C.dnnz, false));  // [2][E] weight-gradient sums
  for (int i = threadIdx.x; i < 2 * E; i += blockDim.x) gws[i] = 0.0f;
  load_tab(tb, C, a.w, false);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  const int nwc = (n + 31) >> 5, swc = (m + 31) >> 5;
  const int sw64 = (m + 63) >> 6, nw64 = (n + 63) >> 6;
  const int K = a.K;
  unsigned char* mine = smem + a.tab_bytes + (size_t)wave * a.wave_bytes;
  // check states of the segment's iterations, [K][m] planes; only the lane that
  // owns a row reads or writes its entries
  float* cm1 = (float*)mine;
  float* cm2 = cm1 + (size_t)K * m;
  u32* cbits = (u32*)(cm2 + (size_t)K * m);
  float* msg = (float*)(cbits + (size_t)K * m);            // [E] messages: q or r (in place)
  float* grad = msg + E;                                   // [E] dLoss/dq, then dLoss/dr, in place
  u32* cutw = (u32*)(grad + E);                            // [nwc]
  u32* synw = cutw + nwc;                                  // [swc]
  const float LS = a.p.lsat;
  auto cs_at = [&](int j, int c) {
    CState st;
    const size_t i = (size_t)j * m + c;
    st.m1 = cm1[i];
    st.m2 = cm2[i];
    st.bits = cbits[i];
    st.pad = 0u;
    return st;
  };

  for (int64_t b = (int64_t)blockIdx.x * nwaves + wave; b < a.B; b += (int64_t)gridDim.x * nwaves) {
    for (int i = lane; i < swc; i += 64) {
      const uint64_t x = a.syn[b * sw64 + (i >> 1)];
      synw[i] = (i & 1) ? (u32)(x >> 32) : (u32)x;
    }
    const bool dc = (a.flags[b] & 2) != 0;
    for (int pass = dc ? 1 : 0; pass >= 0; --pass) {
      for (int i = lane; i < nwc; i += 64) {
        const uint64_t x = a.cut[b * nw64 + (i >> 1)];
        cutw[i] = pass == 0 ? 0u : ((i & 1) ? (u32)(x >> 32) : (u32)x);
      }
      for (int e = lane; e < E; e += 64) grad[e] = 0.0f;
      const int T = pass ? a.p.T2 : a.p.T1;
      const int nck = pass ? a.nck2 : a.nck1;
      const float* wp = tb.w + (size_t)pass * E;
      float* gwp = gws + (size_t)pass * E;
      const float* gp = a.gpost + ((size_t)pass * a.B + b) * n;
      const float* gp2 = dc ? nullptr : a.gpost + ((size_t)a.B + b) * n;
      const bool pf = !SEG && m <= 128;  // prefetched checkpoints
      float p1[2] = {0.0f, 0.0f}, p2[2] = {0.0f, 0.0f};
      u32 pb[2] = {0u, 0u};
      auto ck_load = [&](int s) {
#pragma unroll
        for (int r = 0; r < 2; ++r) {
          const int c = lane + 64 * r;
          if (c < m) {
            const size_t row = ck_index(a, pass, b, s) * (size_t)m + c;
            p1[r] = a.ck_m1[row];
            p2[r] = a.ck_m2[row];
            pb[r] = a.ck_bits[row];
          }
        }
      };
      if (pf) ck_load(nck - 1);
      for (int s = nck - 1; s >= 0; --s) {
        const int t0 = s * K, len = min(T, t0 + K) - t0;
        // the checkpoint (state of iteration t0 + 1) and its r
        if (pf) {
#pragma unroll
          for (int r = 0; r < 2; ++r) {
            const int c = lane + 64 * r;
            if (c < m) {
              CState st;
              st.m1 = cm1[c] = p1[r];
              st.m2 = cm2[c] = p2[r];
              st.bits = cbits[c] = pb[r];
              const int e0 = tb.rp[c];
              write_r<RDM>(msg, wp, e0, tb.rp[c + 1] - e0, st);
            }
          }
          if (s > 0) ck_load(s - 1);
        } else {
          for (int c = lane; c < m; c += 64) {
            const size_t row = ck_index(a, pass, b, s) * (size_t)m + c;
            CState st;
            st.m1 = cm1[c] = a.ck_m1[row];
            st.m2 = cm2[c] = a.ck_m2[row];
            st.bits = cbits[c] = a.ck_bits[row];
            const int e0 = tb.rp[c];
            write_r<RDM>(msg, wp, e0, tb.rp[c + 1] - e0, st);
          }
        }
        wave_sync();
        // recompute the forward through the segment: states of iterations t0 + 2 .. t0 + len
        if constexpr (SEG)
        for (int j = 1; j < len; ++j) {
          for (int v = lane; v < n; v += 64) {
            const int k0 = tb.cp[v], deg = tb.cp[v + 1] - k0;
            const bool cv = (cutw[v >> 5] >> (v & 31)) & 1u;
            int ee[CDM];
            float rr[CDM];
#pragma unroll
            for (int i = 0; i < CDM; ++i)
              if (i < deg) {
                ee[i] = tb.ce[k0 + i];
                rr[i] = msg[ee[i]];
              }
            float Lv = tb.lam[v];
#pragma unroll
            for (int i = 0; i < CDM; ++i)
              if (i < deg) Lv = Lv + rr[i];
#pragma unroll
            for (int i = 0; i < CDM; ++i)
              if (i < deg) msg[ee[i]] = cv ? LS : bpdc_dev::sat(Lv - rr[i], LS);
          }
          wave_sync();
          for (int c = lane; c < m; c += 64) {
            const int e0 = tb.rp[c], deg = tb.rp[c + 1] - e0;
            const CState st = check_state<RDM>(msg, e0, deg, (synw[c >> 5] >> (c & 31)) & 1u, LS);
            const size_t i = (size_t)j * m + c;
            cm1[i] = st.m1;
            cm2[i] = st.m2;
            cbits[i] = st.bits;
            write_r<RDM>(msg, wp, e0, deg, st);
          }
          wave_sync();
        }
        // reverse sweep over the segment; msg holds the r of the iteration at hand
        for (int j = len - 1; j >= 0; --j) {
          const int t = t0 + j + 1;
          // variable side: dLoss/dr from dLoss/dq (and dLoss/dpost at the last iteration)
          for (int v = lane; v < n; v += 64) {
            const int k0 = tb.cp[v], deg = tb.cp[v + 1] - k0;
            const bool cv = (cutw[v >> 5] >> (v & 31)) & 1u;
            int ee[CDM];
            float rr[CDM], gq[CDM];
#pragma unroll
            for (int i = 0; i < CDM; ++i)
              if (i < deg) {
                ee[i] = tb.ce[k0 + i];
                rr[i] = msg[ee[i]];
                gq[i] = grad[ee[i]];
              }
            float Lv = tb.lam[v];
#pragma unroll
            for (int i = 0; i < CDM; ++i)
              if (i < deg) Lv = Lv + rr[i];
            float gL = 0.0f;
            if (t == T && fabsf(Lv) < LS) gL = gp2 ? gp[v] + gp2[v] : gp[v];
#pragma unroll
            for (int i = 0; i < CDM; ++i)
              if (i < deg && fabsf(Lv - rr[i]) < LS) gL += gq[i];
            // a cut column's messages are constants: no gradient through its edges
#pragma unroll
            for (int i = 0; i < CDM; ++i)
              if (i < deg) grad[ee[i]] = cv ? 0.0f : ((fabsf(Lv - rr[i]) < LS) ? gL - gq[i] : gL);
          }
          wave_sync();
          // check side: dLoss/dw and dLoss/dq of the previous iteration (argmin and
          // second argmin of each row only); then the r of the previous iteration
          for (int c = lane; c < m; c += 64) {
            const CState sc = cs_at(j, c);
            const int e0 = tb.rp[c], deg = tb.rp[c + 1] - e0;
            const u32 a1 = cs_a1(sc.bits), a2 = cs_a2(sc.bits);
            // the row's gradients and scales loaded together (RDM bounds the degree)
            float g[RDM], w[RDM];
#pragma unroll
            for (int k = 0; k < RDM; ++k)
              if (k < deg) {
                g[k] = grad[e0 + k];
                w[k] = wp[e0 + k];
              }
            float g1 = 0.0f, g2 = 0.0f;  // into the argmin's q, into the second argmin's q
#pragma unroll
            for (int k = 0; k < RDM; ++k)
              if (k < deg) {
                grad[e0 + k] = 0.0f;
                const bool isa1 = (u32)k == a1;
                const float mag = isa1 ? sc.m2 : sc.m1;
                const float sg = (cs_neg(sc.bits) ^ cs_qsign(sc.bits, k)) ? -g[k] : g[k];
                if (g[k] != 0.0f) atomicAdd(&gwp[e0 + k], sg * mag);
                // a zero gradient adds +-0 (the sums start at +0: unchanged)
                const float d = sg * w[k];
                g2 = isa1 ? g2 + d : g2;
                g1 = isa1 ? g1 : g1 + d;
              }
            if (a1 != kNone) {
              grad[e0 + a1] = g1 * sgn_of(sc.m1, cs_qsign(sc.bits, a1));
              if (a2 != kNone) grad[e0 + a2] = g2 * sgn_of(sc.m2, cs_qsign(sc.bits, a2));
            }
            if (SEG && j > 0) {
              const CState sp = cs_at(j - 1, c);
#pragma unroll
              for (int k = 0; k < RDM; ++k)
                if (k < deg) msg[e0 + k] = cs_r(sp, k, w[k]);
            }
          }
          wave_sync();
        }
      }
    }
  }
  __syncthreads();  // every wave has left its shot loop
  for (int e = threadIdx.x; e < 2 * E; e += blockDim.x)
    if (gws[e] != 0.0f) atomicAdd(&a.gw[e], gws[e]);
}

WCode wcode(const DevCode& d) {
  WCode c;
  c.n = d.n;
  c.m = d.m;
  c.md = d.md;
  c.E = d.E;
  c.dnnz = d.dnnz;
  c.rp = d.h_row_ptr;
  c.col = d.h_col;
  c.cp = d.h_col_ptr;
  c.ce = d.h_col_edge;
  c.erow = d.h_edge_row;
  c.drp = d.d_row_ptr;
  c.dcol = d.d_col;
  c.lam = d.lam;
  return c;
}

// Compile-time bounds on the column and row degrees of a code's kernels (the
// unrolled per-column and per-row loops run every slot, masked past a short
// column or row): 3 and 6 (BB codes), 4 and 8, else 16 and the row limit.
int wms_degree_class(const DevCode& d) {
  if (d.max_col_deg <= 3 && d.max_row_deg <= 6) return 0;
  if (d.max_col_deg <= 4 && d.max_row_deg <= 8) return 1;
  return 2;
}

size_t fwd_wave_bytes(const DevCode& d) {
  return align16((size_t)(d.E + d.n) * 4 + (size_t)(((d.n + 31) / 32) + ((d.m + 31) / 32)) * 4);
}

size_t bwd_wave_bytes(const DevCode& d, int K) {
  return align16((size_t)3 * K * d.m * 4 + (size_t)2 * d.E * 4 + (size_t)(((d.n + 31) / 32) + ((d.m + 31) / 32)) * 4);
}

size_t fwd_tab_bytes(const DevCode& d) { return wtab_bytes(d.n, d.m, d.md, d.E, d.dnnz, true); }
size_t bwd_tab_bytes(const DevCode& d) { return wtab_bytes(d.n, d.m, d.md, d.E, d.dnnz, false) + align16((size_t)2 * d.E * 4); }

// Waves per workgroup of the weighted kernels (each wave decodes its own
// shots; the workgroup shares one copy of the tables): 8, or fewer when the
// LDS of one workgroup cannot hold them (on BB144, 8 waves measured 1.3x
// faster than 4 for the forward and 1.15x for the adjoint, though fewer waves
// stay resident).  BPDC_WMS_WAVES overrides.
int wms_waves(size_t tab, size_t per_wave, int max_lds) {
  const char* e = getenv("BPDC_WMS_WAVES");
  int w = e ? std::max(1, std::min(8, atoi(e))) : 8;
  while (w > 1 && tab + (size_t)w * per_wave > (size_t)max_lds) --w;
  return w;
}

// Persistent grid: as many workgroups as fit on the device at once, at most
// enough for one shot per wave.
int wms_grid(const void* kernel, int threads, size_t lds, int num_cu, int64_t B) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  const int64_t waves = threads / 64;
  return (int)std::max<int64_t>(1, std::min<int64_t>((B + waves - 1) / waves, (int64_t)nb * num_cu));
}

WArgs wargs(const DevCode& d, const KParams& p, const float* w, const uint64_t* syn, int64_t B, int K, void* ckpt) {
  WArgs a;
  a.C = wcode(d);
  a.syn = syn;
  a.B = B;
  a.shot_offset = 0;
  a.K = K;
  a.nck1 = (p.T1 + K - 1) / K;
  a.nck2 = (p.T2 + K - 1) / K;
  a.w = w;
  a.post = nullptr;
  a.cut = nullptr;
  a.flags = nullptr;
  // three planes of (B nck1 + B nck2) m entries each
  const size_t rows = ((size_t)B * a.nck1 + (size_t)B * a.nck2) * (size_t)d.m;
  a.ck_m1 = (float*)ckpt;
  a.ck_m2 = a.ck_m1 + rows;
  a.ck_bits = (u32*)(a.ck_m2 + rows);
  a.gpost = nullptr;
  a.gw = nullptr;
  a.p = p;
  return a;
}

}  // namespace

size_t wms_ckpt_bytes(const DevCode& d, const KParams& p, int64_t B, int K) {
  const int64_t nck = (p.T1 + K - 1) / K + (p.T2 + K - 1) / K;
  return (size_t)B * (size_t)nck * (size_t)d.m * 12;
}

size_t wms_forward_lds(const DevCode& d) { return fwd_tab_bytes(d) + fwd_wave_bytes(d); }

size_t wms_backward_lds(const DevCode& d, int K) { return bwd_tab_bytes(d) + bwd_wave_bytes(d, K); }

hipError_t wms_forward(const DevCode& d, const KParams& p, const float* w, const uint64_t* syn, int64_t B,
                       int64_t shot_offset, int K, float* post, uint64_t* cut, uint8_t* flags, void* ckpt,
                       int num_cu, int max_lds, hipStream_t stream) {
  WArgs a = wargs(d, p, w, syn, B, K, ckpt);
  a.shot_offset = shot_offset;
  a.post = post;
  a.cut = cut;
  a.flags = flags;
  a.tab_bytes = fwd_tab_bytes(d);
  a.wave_bytes = fwd_wave_bytes(d);
  static const void* const kerns[3] = {(const void*)k_wms_forward<3, 6>, (const void*)k_wms_forward<4, 8>,
                                       (const void*)k_wms_forward<16, kWmsMaxRowDeg>};
  const void* kern = kerns[wms_degree_class(d)];
  if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds) != hipSuccess)
    return hipErrorInvalidValue;
  const int waves = wms_waves(a.tab_bytes, a.wave_bytes, max_lds);
  const size_t lds = a.tab_bytes + (size_t)waves * a.wave_bytes;
  (void)hipGetLastError();
  const int grid = wms_grid(kern, 64 * waves, lds, num_cu, B);
  void* args[] = {&a};
  const hipError_t e = hipLaunchKernel(kern, dim3(grid), dim3(64 * waves), args, lds, stream);
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t wms_backward(const DevCode& d, const KParams& p, const float* w, const uint64_t* syn, int64_t B, int K,
                        const float* gpost, const uint64_t* cut, const uint8_t* flags, const void* ckpt, float* gw,
                        int num_cu, int max_lds, hipStream_t stream) {
  WArgs a = wargs(d, p, w, syn, B, K, const_cast<void*>(ckpt));
  a.cut = const_cast<uint64_t*>(cut);
  a.flags = const_cast<uint8_t*>(flags);
  a.gpost = gpost;
  a.gw = gw;
  a.tab_bytes = bwd_tab_bytes(d);
  a.wave_bytes = bwd_wave_bytes(d, K);
  static const void* const kerns[3][2] = {
      {(const void*)k_wms_backward<3, 6, false>, (const void*)k_wms_backward<3, 6, true>},
      {(const void*)k_wms_backward<4, 8, false>, (const void*)k_wms_backward<4, 8, true>},
      {(const void*)k_wms_backward<16, kWmsMaxRowDeg, false>, (const void*)k_wms_backward<16, kWmsMaxRowDeg, true>}};
  const void* kern = kerns[wms_degree_class(d)][K > 1 ? 1 : 0];
  if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds) != hipSuccess)
    return hipErrorInvalidValue;
  const int waves = wms_waves(a.tab_bytes, a.wave_bytes, max_lds);
  const size_t lds = a.tab_bytes + (size_t)waves * a.wave_bytes;
  (void)hipGetLastError();
  const int grid = wms_grid(kern, 64 * waves, lds, num_cu, B);
  void* args[] = {&a};
  const hipError_t e = hipLaunchKernel(kern, dim3(grid), dim3(64 * waves), args, lds, stream);
  return e != hipSuccess ? e : hipGetLastError();
}

}  // namespace bpdc
