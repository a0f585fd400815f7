// Weighted min-sum BP+DC with learned per-edge scales, and its adjoint.
//
// Forward: the decoder of the other kernels with r_e = sign * (w_e * min of
// the other |q|) and a separate weight vector per pass (before / after
// degeneracy cutting), always T iterations per pass (unrolled, no early
// stop).  The per-edge messages q at iterations 0, K, 2K, ... of each pass
// are stored as checkpoints.  Backward: for each shot and pass, from the last
// checkpoint segment to the first, the K iterations of a segment are
// recomputed from its checkpoint and then run in reverse:
//   L_v = prior_v + sum_e r_e,   q_e = sat(L_v - r_e)      (linear, 0 where saturated)
//   r_e = sigma_e * w_e * |q_e*|  with e* the edge holding the minimum over
//         the other edges of the check (the second minimum for the argmin
//         edge), sigma_e the sign (syndrome bit times the other signs, locally
//         constant):  dr_e/dw_e = sigma_e |q_e*|,  dr_e/dq_e* = sigma_e w_e sgn(q_e*).
// The cut set is held fixed (it is a function of the first pass, not
// differentiated), and with the channel prior the second pass depends on the
// first only through the cut, so each pass's gradient comes from its own
// posteriors.  One workgroup per shot; messages of a segment live in LDS;
// per-edge weight gradients are summed in LDS and added to the output once
// per workgroup.
#include <algorithm>
#include <cstdlib>

#include "internal.h"
// after the HIP runtime header: bpdc_device.h itself includes nothing
#include "bpdc_device.h"

namespace bpdc {

namespace {

using bpdc_dev::u32;
using bpdc_dev::u64;

struct WCode {
  int n, m, md, E;
  const int32_t* rp;      // H CSR row pointer
  const int32_t* col;     // H CSR columns
  const int32_t* cp;      // CSC column pointer
  const int32_t* ce;      // CSC -> CSR edge ids (ascending rows)
  const int32_t* drp;
  const int32_t* dcol;
  const float* lam;
};

// Check half of one iteration for all checks: r from q (weights w).
__device__ void wms_check_phase(const WCode& C, const u32* synw, const float* q, float* r, const float* w,
                                float lsat) {
  for (int c = threadIdx.x; c < C.m; c += blockDim.x) {
    const int e0 = C.rp[c], e1 = C.rp[c + 1];
    u32 neg = (synw[c >> 5] >> (c & 31)) & 1u;
    float m1 = lsat, m2 = lsat;
    int amin = -1;
    for (int e = e0; e < e1; ++e) {
      const float a = fabsf(q[e]);
      neg ^= (q[e] < 0.0f) ? 1u : 0u;
      if (a < m1) {
        m2 = m1;
        m1 = a;
        amin = e;
      } else if (a < m2) {
        m2 = a;
      }
    }
    for (int e = e0; e < e1; ++e) {
      const float val = w[e] * ((e == amin) ? m2 : m1);
      r[e] = (neg ^ ((q[e] < 0.0f) ? 1u : 0u)) ? -val : val;
    }
  }
}

// Variable half: L = prior + sum r (ascending check order), q = sat(L - r).
__device__ void wms_var_phase(const WCode& C, const u32* cutw, const float* r, float* q, float* L, float lsat) {
  const float INF = __builtin_huge_valf();
  for (int v = threadIdx.x; v < C.n; v += blockDim.x) {
    const int k0 = C.cp[v], k1 = C.cp[v + 1];
    if ((cutw[v >> 5] >> (v & 31)) & 1u) {
      for (int k = k0; k < k1; ++k) q[C.ce[k]] = lsat;
      L[v] = INF;
      continue;
    }
    float Lv = C.lam[v];
    for (int k = k0; k < k1; ++k) Lv = Lv + r[C.ce[k]];
    for (int k = k0; k < k1; ++k) {
      const int e = C.ce[k];
      q[e] = bpdc_dev::sat(Lv - r[e], lsat);
    }
    L[v] = Lv;
  }
}

__device__ void wms_init_q(const WCode& C, const u32* cutw, float* q, float lsat) {
  for (int v = threadIdx.x; v < C.n; v += blockDim.x) {
    const bool cut = (cutw[v >> 5] >> (v & 31)) & 1u;
    const float q0 = cut ? lsat : bpdc_dev::sat(C.lam[v], lsat);
    for (int k = C.cp[v]; k < C.cp[v + 1]; ++k) q[C.ce[k]] = q0;
  }
}

__global__ void __launch_bounds__(256) k_wms_forward(WCode C, const float* w, const uint64_t* syn, int64_t B,
                                                     int64_t shot_offset, int K, int nck1, int nck2, float* post,
                                                     uint64_t* cut_out, uint8_t* flags, float* ckpt, KParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sUnsat;
  const int n = C.n, m = C.m, E = C.E;
  float* q = (float*)smem;
  float* r = q + E;
  float* L = r + E;
  u32* cutw = (u32*)(L + n);
  u32* synw = cutw + ((n + 31) >> 5);
  const int sw64 = (m + 63) >> 6, nw64 = (n + 63) >> 6;
  const float LS = P.lsat, INF = __builtin_huge_valf();
  const int nck[2] = {nck1, nck2};
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    for (int i = threadIdx.x; i < ((m + 31) >> 5); i += blockDim.x) {
      const uint64_t x = syn[b * sw64 + (i >> 1)];
      synw[i] = (i & 1) ? (u32)(x >> 32) : (u32)x;
    }
    for (int i = threadIdx.x; i < ((n + 31) >> 5); i += blockDim.x) cutw[i] = 0u;
    __syncthreads();
    bool conv = false;
    int pass = 0;
    for (; pass < 2; ++pass) {
      const int T = pass ? P.T2 : P.T1;
      const float* wp = w + (size_t)pass * E;
      float* ck = ckpt + ((size_t)(pass ? B * nck1 : 0) + (size_t)b * nck[pass]) * E;
      wms_init_q(C, cutw, q, LS);
      __syncthreads();
      for (int t = 1; t <= T; ++t) {
        if ((t - 1) % K == 0)
          for (int e = threadIdx.x; e < E; e += blockDim.x) ck[(size_t)((t - 1) / K) * E + e] = q[e];
        wms_check_phase(C, synw, q, r, wp, LS);
        __syncthreads();
        wms_var_phase(C, cutw, r, q, L, LS);
        __syncthreads();
      }
      float* pp = post + ((size_t)pass * B + b) * n;
      for (int v = threadIdx.x; v < n; v += blockDim.x) pp[v] = (L[v] == INF) ? INF : bpdc_dev::sat(L[v], LS);
      if (threadIdx.x == 0) sUnsat = 0;
      __syncthreads();
      int bad = 0;
      for (int c = threadIdx.x; c < m; c += blockDim.x) {
        u32 par = (synw[c >> 5] >> (c & 31)) & 1u;
        for (int e = C.rp[c]; e < C.rp[c + 1]; ++e) par ^= (L[C.col[e]] <= 0.0f) ? 1u : 0u;
        bad |= (int)par;
      }
      if (bad) atomicOr(&sUnsat, 1);
      __syncthreads();
      conv = sUnsat == 0;
      if (pass == 1 || conv) break;
      // degeneracy cutting on the first-pass posteriors
      for (int h = threadIdx.x; h < C.md; h += blockDim.x) {
        const int e0 = C.drp[h], deg = C.drp[h + 1] - e0;
        if (deg == 0) continue;
        int cols[32];
        float vals[32];
        for (int k = 0; k < deg; ++k) {
          cols[k] = C.dcol[e0 + k];
          vals[k] = bpdc_dev::sat(L[cols[k]], LS);
        }
        const int pick = bpdc_dev::dc_pick<32>(cols, vals, deg, P.tie_eps, P.tie_lowest, P.seed,
                                               (u64)(shot_offset + b), (u64)h);
        atomicOr(&cutw[pick >> 5], 1u << (pick & 31));
      }
      __syncthreads();
    }
    const bool dc = pass == 1;
    if (!dc) {  // second-pass rows of shots without DC are copies of the first pass
      float* p0 = post + (size_t)b * n;
      float* p1 = post + ((size_t)B + b) * n;
      for (int v = threadIdx.x; v < n; v += blockDim.x) p1[v] = p0[v];
    }
    for (int i = threadIdx.x; i < nw64; i += blockDim.x) {
      const u32 lo = cutw[2 * i];
      const u32 hi = (2 * i + 1 < ((n + 31) >> 5)) ? cutw[2 * i + 1] : 0u;
      cut_out[b * nw64 + i] = dc ? (((u64)hi << 32) | lo) : 0ull;
    }
    if (threadIdx.x == 0) flags[b] = (uint8_t)((conv ? 1 : 0) | (dc ? 2 : 0));
    __syncthreads();
  }
}

__device__ __forceinline__ float sgnf(float x) { return (x > 0.0f) ? 1.0f : ((x < 0.0f) ? -1.0f : 0.0f); }

__global__ void __launch_bounds__(256) k_wms_backward(WCode C, const float* w, const uint64_t* syn, int64_t B,
                                                      int K, int nck1, int nck2, const float* gpost,
                                                      const uint64_t* cut_in, const uint8_t* flags,
                                                      const float* ckpt, float* gw_out, KParams P) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int n = C.n, m = C.m, E = C.E;
  float* qs = (float*)smem;          // [(K + 1) * E] messages q(t0 .. t0 + K)
  float* r = qs + (size_t)(K + 1) * E;  // [E] r(t) (recomputed)
  float* gq = r + E;                 // [E] dLoss/dq(t)
  float* gqn = gq + E;               // [E] dLoss/dq(t - 1) being accumulated (the two swap roles)
  float* gr = gqn + E;               // [E] dLoss/dr(t)
  float* gw = gr + E;                // [2 * E] per-workgroup weight gradients
  float* L = gw + 2 * E;             // [n]
  u32* cutw = (u32*)(L + n);
  u32* synw = cutw + ((n + 31) >> 5);
  const int sw64 = (m + 63) >> 6, nw64 = (n + 63) >> 6;
  const float LS = P.lsat;
  const int nck[2] = {nck1, nck2};
  for (int e = threadIdx.x; e < 2 * E; e += blockDim.x) gw[e] = 0.0f;
  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    for (int i = threadIdx.x; i < ((m + 31) >> 5); i += blockDim.x) {
      const uint64_t x = syn[b * sw64 + (i >> 1)];
      synw[i] = (i & 1) ? (u32)(x >> 32) : (u32)x;
    }
    const bool dc = (flags[b] & 2) != 0;
    for (int pass = dc ? 1 : 0; pass >= 0; --pass) {
      for (int i = threadIdx.x; i < ((n + 31) >> 5); i += blockDim.x) {
        const uint64_t x = cut_in[b * nw64 + (i >> 1)];
        cutw[i] = pass == 0 ? 0u : ((i & 1) ? (u32)(x >> 32) : (u32)x);
      }
      for (int e = threadIdx.x; e < E; e += blockDim.x) gq[e] = 0.0f;
      __syncthreads();
      const int T = pass ? P.T2 : P.T1;
      const float* wp = w + (size_t)pass * E;
      const float* ck = ckpt + ((size_t)(pass ? B * nck1 : 0) + (size_t)b * nck[pass]) * E;
      const float* gp = gpost + ((size_t)pass * B + b) * n;
      // a shot without DC reports its first-pass posteriors in both output rows,
      // so pass 0 collects the gradient of both rows
      const float* gp2 = dc ? nullptr : gpost + ((size_t)B + b) * n;
      for (int s = nck[pass] - 1; s >= 0; --s) {
        const int t0 = s * K, t1 = min(T, t0 + K);
        for (int e = threadIdx.x; e < E; e += blockDim.x) qs[e] = ck[(size_t)s * E + e];
        __syncthreads();
        for (int t = t0 + 1; t <= t1; ++t) {  // recompute the segment's messages
          wms_check_phase(C, synw, qs + (size_t)(t - t0 - 1) * E, r, wp, LS);
          __syncthreads();
          wms_var_phase(C, cutw, r, qs + (size_t)(t - t0) * E, L, LS);
          __syncthreads();
        }
        for (int t = t1; t > t0; --t) {
          const float* qp = qs + (size_t)(t - t0 - 1) * E;  // q(t - 1)
          wms_check_phase(C, synw, qp, r, wp, LS);          // r(t)
          __syncthreads();
          // variable side: L(t) = prior + sum r(t); q(t) = sat(L - r)
          for (int v = threadIdx.x; v < n; v += blockDim.x) {
            const int k0 = C.cp[v], k1 = C.cp[v + 1];
            if ((cutw[v >> 5] >> (v & 31)) & 1u) {
              for (int k = k0; k < k1; ++k) gr[C.ce[k]] = 0.0f;
              continue;
            }
            float Lv = C.lam[v];
            for (int k = k0; k < k1; ++k) Lv = Lv + r[C.ce[k]];
            float gL = (t == T && fabsf(Lv) < LS) ? (gp2 ? gp[v] + gp2[v] : gp[v]) : 0.0f;
            for (int k = k0; k < k1; ++k) {
              const int e = C.ce[k];
              if (fabsf(Lv - r[e]) < LS) gL += gq[e];
            }
            for (int k = k0; k < k1; ++k) {
              const int e = C.ce[k];
              gr[e] = (fabsf(Lv - r[e]) < LS) ? gL - gq[e] : gL;
            }
          }
          for (int e = threadIdx.x; e < E; e += blockDim.x) gqn[e] = 0.0f;
          __syncthreads();
          // check side: through w * min |q| and the (locally constant) signs
          for (int c = threadIdx.x; c < m; c += blockDim.x) {
            const int e0 = C.rp[c], e1 = C.rp[c + 1];
            float m1 = LS, m2 = LS;
            int a1 = -1, a2 = -1;
            u32 neg = (synw[c >> 5] >> (c & 31)) & 1u;
            for (int e = e0; e < e1; ++e) {
              neg ^= (qp[e] < 0.0f) ? 1u : 0u;
              const float a = fabsf(qp[e]);
              if (a < m1) {
                m2 = m1;
                a2 = a1;
                m1 = a;
                a1 = e;
              } else if (a < m2) {
                m2 = a;
                a2 = e;
              }
            }
            for (int e = e0; e < e1; ++e) {
              const float g = gr[e];
              if (g == 0.0f) continue;
              const float mag = (e == a1) ? m2 : m1;
              const int src = (e == a1) ? a2 : a1;
              const float sig = (neg ^ ((qp[e] < 0.0f) ? 1u : 0u)) ? -1.0f : 1.0f;
              // edge e belongs to this thread's check only: a plain add
              gw[(size_t)pass * E + e] += g * sig * mag;
              if (src >= 0) gqn[src] += g * sig * wp[e] * sgnf(qp[src]);
            }
          }
          __syncthreads();
          // dLoss/dq(t - 1) becomes the next step's dLoss/dq(t); the old buffer
          // is cleared before it accumulates again
          float* tmp = gq;
          gq = gqn;
          gqn = tmp;
        }
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 2 * E; e += blockDim.x)
    if (gw[e] != 0.0f) atomicAdd(&gw_out[e], gw[e]);
}

WCode wcode(const DevCode& d) {
  WCode c;
  c.n = d.n;
  c.m = d.m;
  c.md = d.md;
  c.E = d.E;
  c.rp = d.h_row_ptr;
  c.col = d.h_col;
  c.cp = d.h_col_ptr;
  c.ce = d.h_col_edge;
  c.drp = d.d_row_ptr;
  c.dcol = d.d_col;
  c.lam = d.lam;
  return c;
}

}  // namespace

size_t wms_forward_lds(const DevCode& d) {
  return (size_t)(2 * d.E + d.n) * 4 + (size_t)(((d.n + 31) / 32) + ((d.m + 31) / 32)) * 4 + 16;
}

size_t wms_backward_lds(const DevCode& d, int K) {
  return (size_t)((K + 1) * d.E + 4 * d.E + 2 * d.E + d.n) * 4 + (size_t)(((d.n + 31) / 32) + ((d.m + 31) / 32)) * 4 +
         16;
}

// Threads per workgroup of the weighted kernels (one workgroup per shot; 64,
// 128 or 256): the forward kernel's small LDS footprint lets one-wave
// workgroups fill the compute units (64, measured fastest on BB144); the
// adjoint keeps K + 1 message vectors per shot and is LDS-bound, so it takes
// two waves per shot (128).  BPDC_WMS_THREADS_FWD / _BWD override.
int wms_threads(bool backward) {
  const char* e = getenv(backward ? "BPDC_WMS_THREADS_BWD" : "BPDC_WMS_THREADS_FWD");
  const int v = e ? atoi(e) : (backward ? 128 : 64);
  return v <= 64 ? 64 : (v <= 128 ? 128 : 256);
}

// Persistent grid: as many workgroups as fit on the device at once, at most B.
int wms_grid(const void* kernel, int threads, size_t lds, int num_cu, int64_t B) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  return (int)std::max<int64_t>(1, std::min<int64_t>(B, (int64_t)nb * num_cu));
}

hipError_t wms_forward(const DevCode& d, const KParams& p, const float* w, const uint64_t* syn, int64_t B,
                       int64_t shot_offset, int K, float* post, uint64_t* cut, uint8_t* flags, float* ckpt,
                       int num_cu, int max_lds, hipStream_t stream) {
  const size_t lds = wms_forward_lds(d);
  if (lds > 65536 &&
      hipFuncSetAttribute((const void*)k_wms_forward, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds) != hipSuccess)
    return hipErrorInvalidValue;
  (void)hipGetLastError();
  const int threads = wms_threads(false);
  const int grid = wms_grid((const void*)k_wms_forward, threads, lds, num_cu, B);
  const int nck1 = (p.T1 + K - 1) / K, nck2 = (p.T2 + K - 1) / K;
  hipLaunchKernelGGL(k_wms_forward, dim3(grid), dim3(threads), lds, stream, wcode(d), w, syn, B, shot_offset, K, nck1,
                     nck2, post, cut, flags, ckpt, p);
  return hipGetLastError();
}

hipError_t wms_backward(const DevCode& d, const KParams& p, const float* w, const uint64_t* syn, int64_t B, int K,
                        const float* gpost, const uint64_t* cut, const uint8_t* flags, const float* ckpt, float* gw,
                        int num_cu, int max_lds, hipStream_t stream) {
  const size_t lds = wms_backward_lds(d, K);
  if (lds > 65536 &&
      hipFuncSetAttribute((const void*)k_wms_backward, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds) != hipSuccess)
    return hipErrorInvalidValue;
  (void)hipGetLastError();
  const int threads = wms_threads(true);
  const int grid = wms_grid((const void*)k_wms_backward, threads, lds, num_cu, B);
  const int nck1 = (p.T1 + K - 1) / K, nck2 = (p.T2 + K - 1) / K;
  hipLaunchKernelGGL(k_wms_backward, dim3(grid), dim3(threads), lds, stream, wcode(d), w, syn, B, K, nck1, nck2, gpost,
                     cut, flags, ckpt, gw, p);
  return hipGetLastError();
}

}  // namespace bpdc
