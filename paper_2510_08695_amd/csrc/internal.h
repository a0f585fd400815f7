// Internal interfaces between the host runtime (runtime.cpp) and the kernels
// of libbpdc.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace bpdc {

// A code resident on the device: Tanner graph H in CSR and CSC form, the
// degeneracy matrix D in CSR form and the prior LLRs (float, rounded once
// from double).  Edge e of H is its CSR position; the CSC lists per column
// the CSR positions of its edges in ascending row order.
// Bytes of control words at the start of the group kernel's LDS.
constexpr int kLdsHead = 32;

struct DevCode {
  int n = 0, m = 0, md = 0, E = 0, dnnz = 0;
  int max_row_deg = 0, max_col_deg = 0, max_drow_deg = 0;
  int32_t* h_row_ptr = nullptr;  // [m+1]
  int32_t* h_col = nullptr;      // [E]
  int32_t* h_col_ptr = nullptr;  // [n+1]
  int32_t* h_col_edge = nullptr; // [E] CSR edge ids, per column ascending row
  int32_t* h_edge_row = nullptr; // [E] row of each edge
  int32_t* d_row_ptr = nullptr;  // [md+1]
  int32_t* d_col = nullptr;      // [dnnz]
  float* lam = nullptr;          // [n]
  // The group kernel's min-sum phases read these two tables as LDS addresses
  // (its layout: kLdsHead bytes of control words, m + 1 check records of 16
  // bytes, then L[n + 1]).
  // The group kernel's min-sum variants keep L in slot order (for codes with
  // rows above 32 edges the columns sorted by descending degree, ties in
  // column order, so that a block of 64 slots mostly holds one degree;
  // otherwise the column order) and index these by slot.
  int32_t* v_ell = nullptr;      // [max_col_deg][n] ((row + kLdsHead / 16) << 10) | position in row, ascending
                                 // rows: >> 6 is the LDS address of the row's record; pad row m
  int32_t* c_ell = nullptr;      // [max_row_deg][m] LDS address of L[slot of the column] at each row
                                 // position (kLdsHead + 16 (m + 1) + 4 slot); pad slot n
  int32_t* v_blk_deg = nullptr;  // [ceil(n/64)] largest column degree of each block of 64 slots
  float* g_lam = nullptr;        // [n] prior of each slot
  int32_t* g_dcol = nullptr;     // [dnnz] d_col as slots (rows keep ascending column order)
  int32_t* g_pos = nullptr;      // [n] slot of each column
};

// Runtime decoder parameters as the kernels see them.
struct KParams {
  int T1, T2;
  float alpha, lsat, tie_eps;
  int second_pass_posterior;
  int stop;
  int tie_lowest;
  unsigned long long seed;
  int rule;  // 0 scaled min-sum, 1 product-sum
  int soft_period;   // intermittent soft DC every soft_period first-pass iterations (0: off)
  float soft_shift;  // prior-LLR increase of each soft nominee
};

// Output / input buffers of one single-code decode.
struct DecodeIO {
  const uint64_t* syn;
  int64_t B;
  int64_t shot_offset;
  uint64_t* corr;
  uint8_t* flags;
  float* post;
  uint64_t* cut;
  int16_t* iters;
  uint64_t* dcstats;  // DC diagnostics (accumulated) or null
};

// Plain decoder: one launch per phase per iteration, edge-major state in HBM.
size_t plain_workspace_bytes(const DevCode& c, int64_t B);
hipError_t plain_decode(const DevCode& c, const KParams& p, const DecodeIO& io, void* ws,
                        hipStream_t stream);

// Launch shape of the group kernel chosen by the autotuner.
struct GroupTile {
  int shots_per_wg = 1;
  int threads = 256;
  int grid = 0;          // persistent workgroups
  size_t lds_bytes = 0;  // dynamic LDS per workgroup
  int info_bytes = 4;    // min-sum check records with 4 (row degree <= 32) or 8 (<= 58) bytes of sign
                         // bits; 0: product-sum (per-edge r, rows of at most 8 edges)
};

// Group decoder (group.hip): persistent fused kernel, one workgroup per shot,
// the shot's state in dynamic LDS; also the multi-code launch.
size_t group_lds_bytes_nm(int n, int m, bool posterior, int info_bytes, int edges);
int group_occupancy(int threads, size_t lds, int info_bytes, int max_lds);
// True when no group kernel uses static LDS (their dynamic block, and so the
// LDS addresses in the code tables, start at 0).
bool group_lds_starts_at_zero();
// Flags value of a multi-code shot whose code index is outside [0, ncodes): the
// shot is skipped and nothing else of it is written.
constexpr uint8_t kFlagBadCode = 0x80;
// n_bad (device word, multi-code only, else null): the shots group_order left out of
// `order`; the kernel decodes the first B - *n_bad entries of the order.
hipError_t group_launch(const void* d_codes, const unsigned* n_bad, const int32_t* code_of_shot,
                        const int32_t* order, const KParams& p, const uint64_t* syn, const int64_t* syn_off, uint64_t* corr,
                        const int64_t* corr_off, uint8_t* flags, float* post, uint64_t* cut,
                        int16_t* iters, int64_t B, int64_t shot_offset, int threads, int grid,
                        size_t lds, int info_bytes, unsigned long long* queue, hipStream_t stream,
                        unsigned long long* dcstats = nullptr, int claim_n = 0);
// (claim_n: a single-code launch's column count, which sets how many
// consecutive shots a workgroup claims at once; 0 or a multi-code launch: one)
// hist and base hold ncodes + 1 entries each; hist[ncodes] counts the shots with an
// out-of-range code index, which get flags kFlagBadCode and no place in `order`.
hipError_t group_order(const int32_t* code_of_shot, int64_t B, const int32_t* code_by_rank, int ncodes,
                       unsigned* hist, unsigned* base, int32_t* order, uint8_t* flags, hipStream_t stream);

// Mirror of the device code descriptor used by group.hip.
struct GCodeHost {
  int n, m, md;
  int posterior;
  const int32_t* h_row_ptr;
  const int32_t* h_col;
  const int32_t* h_col_ptr;
  const int32_t* h_col_edge;
  const int32_t* h_edge_row;
  const int32_t* d_row_ptr;
  const int32_t* d_col;
  const float* lam;
  const int32_t* v_ell;
  const int32_t* c_ell;
  const int32_t* v_blk_deg;
  int max_col_deg, max_row_deg;
  const float* g_lam;
  const int32_t* g_dcol;
  const int32_t* g_pos;
};

// Weighted min-sum forward (checkpointed) and adjoint (wms.hip).  Rows of at
// most kWmsMaxRowDeg edges (the sign bits of a 12-byte check state).
constexpr int kWmsMaxRowDeg = 21;
size_t wms_ckpt_bytes(const DevCode& d, const KParams& p, int64_t B, int K);
size_t wms_forward_lds(const DevCode& d);
size_t wms_backward_lds(const DevCode& d, int K);
hipError_t wms_forward(const DevCode& d, const KParams& p, const float* w, const uint64_t* syn, int64_t B,
                       int64_t shot_offset, int K, float* post, uint64_t* cut, uint8_t* flags, void* ckpt,
                       int num_cu, int max_lds, hipStream_t stream);
hipError_t wms_backward(const DevCode& d, const KParams& p, const float* w, const uint64_t* syn, int64_t B, int K,
                        const float* gpost, const uint64_t* cut, const uint8_t* flags, const void* ckpt, float* gw,
                        int num_cu, int max_lds, hipStream_t stream);

// bpdc_device.h's product-sum function phi on n floats (accuracy tests).
hipError_t eval_phi(const float* x, int64_t n, float* out, hipStream_t stream);

// Small fill kernel (graph-capture safe replacement for hipMemsetAsync).
hipError_t fill_u64(uint64_t* p, uint64_t v, size_t count, hipStream_t stream);

// Device address of `device`'s copy of the static scratch of bpdc_decode_noalloc
// (noalloc.hip); call with that device current.  Looked up once per device.
hipError_t noalloc_scratch(int device, void** ptr);

}  // namespace bpdc
