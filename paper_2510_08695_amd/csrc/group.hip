// Fused persistent BP -> DC -> BP kernel with one workgroup per shot and the
// shot's whole state in LDS: any code size up to the LDS of one workgroup,
// any mix of codes in one launch.
//
// A workgroup takes the next shot from a global counter (a single-code
// launch of a small code: the next few consecutive shots, whose outputs then
// share cache lines written from one L2; shots of a mixed batch are first
// grouped by code, largest codes first, so that long shots start early and
// consecutive shots of a workgroup share the code's index arrays in cache).
// Per iteration (flooding schedule, Sec. II.C) it runs
//   variable phase: one thread per column: L_v = prior + sum r (ascending
//                  check order), +inf on cut columns (Algorithm 2);
//   check phase  : one thread per check: q = L_v - r_old for each edge (its
//                  clamp to lsat would change nothing here),
//                  new (alpha*min1, alpha*min2, argmin, r-sign bits), and the
//                  parity of [L <= 0] over the check against the syndrome bit
//                  (the stop test H e = s of this iteration);
// with a workgroup barrier after each.  The code's adjacency is read from
// padded column-major tables (one coalesced load per edge).  After a failed
// first pass it runs degeneracy cutting (Sec. III.A) with one thread per row
// of D and the second pass, then writes the packed correction.  The
// arithmetic order is that of every other decoder of the library, so results
// are bit-identical.
#include <algorithm>

#include "internal.h"
// after the HIP runtime header: bpdc_device.h itself includes nothing
#include "bpdc_device.h"

namespace bpdc {

// Device-side description of one code of a (multi-code) plan.
struct GCode {
  int n, m, md;
  int posterior;  // unused per code (plan-wide), kept for alignment
  const int32_t* h_row_ptr;
  const int32_t* h_col;
  const int32_t* h_col_ptr;
  const int32_t* h_col_edge;
  const int32_t* h_edge_row;
  const int32_t* d_row_ptr;
  const int32_t* d_col;
  const float* lam;
  // Min-sum keeps L in slot order: for codes with rows above 32 edges the
  // columns sorted by descending degree (ties in column order), otherwise the
  // column order.
  const int32_t* v_ell;  // [max_col_deg][n]: per slot, ((check + kRec0) << 10) | position in the check's
                         // row, ascending checks; padded with check m (a dummy whose messages are -0)
  const int32_t* c_ell;  // [max_row_deg][m]: LDS address of L at each position of the check's row; padded
                         // with slot n (a dummy whose posterior is +inf)
  const int32_t* v_blk_deg;  // [ceil(n/64)]: largest column degree of each block of 64 slots
  int max_col_deg, max_row_deg;
  const float* g_lam;     // [n] prior of each slot
  const int32_t* g_dcol;  // rows of D as slots (each row in ascending column order)
  const int32_t* g_pos;   // [n] slot of each column
};

namespace {

using bpdc_dev::u32;
using bpdc_dev::u64;

// Check c's record sits at LDS address 16 (c + kRec0) (after the control
// words); the column-table entries and the narrow records' argmin name it as
// ((c + kRec0) << 10) | position.
constexpr int kRec0 = kLdsHead / 16;

struct GArgs {
  const GCode* codes;
  const int32_t* code_of_shot;  // null: every shot is code 0
  const int32_t* order;         // null: identity processing order
  const uint64_t* syn;
  const int64_t* syn_off;       // null: b * ceil(m/64)
  uint64_t* corr;
  const int64_t* corr_off;      // null: b * ceil(n/64)
  uint8_t* flags;
  float* post;                  // single-code only (may be null)
  uint64_t* cut;                // single-code only (may be null)
  int16_t* iters;
  int64_t B;
  int64_t shot_offset;
  unsigned long long* queue;
  const unsigned* n_bad;        // multi-code: shots with an out-of-range code index (kept out of `order`)
  unsigned long long* dcstats;  // DC diagnostics (spread bins, DC shots, cut sizes) or null
  int claim;                    // consecutive shots per claim from the queue
  KParams p;
};

// Per-check state, one 16-byte record (one LDS access): alpha*min1,
// alpha*min2, the r-sign bit of every edge of the row and the argmin position.
// Narrow rows (at most 32 edges): 32 sign bits, row position k at bit 31 - k
// (the check phase shifts each q's sign in from the bottom), and, in its own
// word, the argmin edge as a column-table entry (((check + kRec0) << 10) | position), so
// that a column compares its entry with it directly; wide rows (at most 58):
// 64 sign bits, position k at bit k, whose top six hold the argmin position.
// old_sign: the sign bit of position k of a sign word, at bit 31;
// push_sign / finish_signs: the sign word of q over positions 0 .. K-1 built
// one position at a time.
template <bool Wide>
struct CheckRec;
template <>
struct __align__(16) CheckRec<false> {
  float a1, a2;
  u32 sgn, amin;
  using Word = u32;
  static constexpr Word kSignMask = 0xffffffffu;
  __device__ __forceinline__ int argmin() const { return (int)(amin & 63u); }
  __device__ __forceinline__ Word signs() const { return sgn; }
  __device__ __forceinline__ void set(float x1, float x2, Word s, int am, int check) {
    a1 = x1; a2 = x2; sgn = s; amin = ((u32)check << 10) | (u32)am;
  }
  // r of the edge with column-table entry `ent` (the magnitude is +0 or
  // positive, alpha >= 0, or -0 on the dummy check, whose sign bits are 0,
  // so the sign is or-ed in)
  __device__ __forceinline__ float r_of(u32 ent) const {
    const float mag = (amin == ent) ? a2 : a1;
    return __uint_as_float(__float_as_uint(mag) | ((sgn << (ent & 31u)) & 0x80000000u));
  }
  static __device__ __forceinline__ u32 old_sign(Word io, int k) { return (io << k) & 0x80000000u; }
  static __device__ __forceinline__ Word push_sign(Word sb, float q, int) {
    return __builtin_amdgcn_alignbit(sb, __float_as_uint(q), 31);  // (sb << 1) | sign(q)
  }
  // (K = 0: no position was pushed and sb is 0; the shift count is taken mod 32)
  static __device__ __forceinline__ Word finish_signs(Word sb, int K) { return sb << ((32 - K) & 31); }
};
template <>
struct __align__(16) CheckRec<true> {
  float a1, a2;
  u32 lo, hi;
  using Word = u64;
  static constexpr Word kSignMask = ((u64)1 << 58) - 1u;
  __device__ __forceinline__ int argmin() const { return (int)(hi >> 26); }
  __device__ __forceinline__ Word signs() const { return ((u64)hi << 32) | lo; }
  __device__ __forceinline__ void set(float x1, float x2, Word s, int am, int) {
    a1 = x1; a2 = x2; lo = (u32)s; hi = (u32)(s >> 32) | ((u32)am << 26);
  }
  __device__ __forceinline__ float r_of(u32 ent) const {
    const int k = (int)(ent & 63u);
    const float mag = (argmin() == k) ? a2 : a1;
    const u32 bit = ((k < 32 ? lo : hi) >> (k & 31)) & 1u;
    return __uint_as_float(__float_as_uint(mag) | (bit << 31));
  }
  static __device__ __forceinline__ u32 old_sign(Word io, int k) { return ((u32)(io >> k) & 1u) << 31; }
  static __device__ __forceinline__ Word push_sign(Word sb, float q, int k) {
    return sb | ((Word)(__float_as_uint(q) >> 31) << k);
  }
  static __device__ __forceinline__ Word finish_signs(Word sb, int) { return sb; }
};

__device__ __forceinline__ int popc_word(u32 x) { return __builtin_popcount(x); }
__device__ __forceinline__ int popc_word(u64 x) { return __builtin_popcountll(x); }

// Load through a global-address-space pointer (the code tables are reached
// through a table in device memory, so the compiler cannot infer it).
__device__ __forceinline__ int gload(const int32_t* p, unsigned i) {
  return ((const __attribute__((address_space(1))) int32_t*)p)[i];
}
// The object at LDS address `addr`.  The group kernels use no static LDS, so
// their dynamic block starts at address 0 (the host checks the static size
// before the first launch) and an address from the code tables is used as is.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ const __attribute__((address_space(3))) T* lds_at(u32 addr) {
  return (const __attribute__((address_space(3))) T*)(uintptr_t)addr;
}

// A code table as a buffer resource (raw, 32-bit words), so that a load
// takes its address as a scalar part (the table slice) plus the thread's
// 32-bit byte offset, with no vector address arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t table_rsrc(const int32_t* p) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ u32 vtab_at(__amdgpu_buffer_rsrc_t t, u32 scalar_off, u32 byte_off) {
  // (readfirstlane: the offset is uniform; it keeps the compiler from a
  // per-value loop where register pressure has moved it to a vector register)
  return (u32)__builtin_amdgcn_raw_buffer_load_b32(t, byte_off, __builtin_amdgcn_readfirstlane(scalar_off), 0);
}

// L + the r of K consecutive slots (from k0) of a column's entries, all loads
// issued before the sums, in slot (ascending check) order.
template <int K, class Rec>
__device__ __forceinline__ float col_sum(float Lv, __amdgpu_buffer_rsrc_t vt, u32 n4, u32 vo, int k0) {
  u32 ent[K];
#pragma unroll
  for (int j = 0; j < K; ++j) ent[j] = vtab_at(vt, (u32)(k0 + j) * n4, vo);
  Rec sr[K];
  // ((check + kRec0) << 10) >> 6: the LDS address of the check's record
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const u32x4 w = *lds_at<u32x4>(ent[j] >> 6);
    __builtin_memcpy(&sr[j], &w, sizeof(Rec));
  }
#pragma unroll
  for (int j = 0; j < K; ++j) Lv = Lv + sr[j].r_of(ent[j]);
  return Lv;
}

// Where the pipelined variable phase takes a column's prior from: the code's
// prior table (first pass, channel prior); the same table with +inf on the
// shot's cut columns (second pass, channel prior: Algorithm 2's frozen
// columns); the shot's prior array in LDS (soft DC, posterior prior, whose
// cut columns already hold +inf).
enum PriorSrc { kPriorTable, kPriorTableCut, kPriorLds };

// The K table entries of column v and its prior.
template <int K, int Src>
__device__ __forceinline__ void col_fetch(u32 (&e)[K], float& lam, __amdgpu_buffer_rsrc_t vt,
                                          __amdgpu_buffer_rsrc_t lt, const float* lam2, u32 n4, int v) {
  const u32 vo = (u32)v << 2;
  if constexpr (Src == kPriorLds) lam = lam2[v];
  else lam = __uint_as_float(vtab_at(lt, 0u, vo));
#pragma unroll
  for (int j = 0; j < K; ++j) e[j] = vtab_at(vt, (u32)j * n4, vo);
}

// L + the r of a column's K fetched entries, in slot (ascending check) order.
// A cut column's L starts at +inf and stays there (+inf + r = +inf: r is
// finite).
template <int K, class Rec>
__device__ __forceinline__ float col_add(float Lv, const u32 (&e)[K]) {
  Rec sr[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const u32x4 w = *lds_at<u32x4>(e[j] >> 6);
    __builtin_memcpy(&sr[j], &w, sizeof(Rec));
  }
#pragma unroll
  for (int j = 0; j < K; ++j) Lv = Lv + sr[j].r_of(e[j]);
  return Lv;
}

// A column's prior, +inf if it is this thread's i-th column and cut (bit i of
// cutbits; sign-extended to a mask that selects the bits of +inf).
template <int Src>
__device__ __forceinline__ float col_prior(float lam, u32 cutbits, int i) {
  if constexpr (Src != kPriorTableCut) return lam;
  const u32 msk = (u32)((int)(cutbits << (31 - i)) >> 31);
  return __uint_as_float((msk & 0x7f800000u) | (~msk & __float_as_uint(lam)));
}

// Variable phase over the run of slots [s0, s1), whose columns all have K
// table entries: thread tid takes slots s0 + tid, s0 + tid + nt, ...; the next
// slot's entries and prior are loaded while this slot's check records are read
// and summed (the same sums in the same order).  Two register sets take turns,
// so nothing is copied between slots, and the prefetch index is clamped to
// the run's last slot, so every load is in bounds.  i counts the thread's
// slots over the whole phase (the cut bit of each); the count after the run
// is returned.
template <int K, class Rec, int Src>
__device__ __forceinline__ int var_run(float* L, const float* lam2, int s0, int s1, int tid, int nt, u32 cutbits,
                                       int i, __amdgpu_buffer_rsrc_t vt, __amdgpu_buffer_rsrc_t lt, u32 n4) {
  int v = s0 + tid;
  if (v >= s1) return i;
  const int last = s1 - 1;
  u32 ea[K], eb[K];
  float la, lb;
  col_fetch<K, Src>(ea, la, vt, lt, lam2, n4, v);
  for (;;) {
    col_fetch<K, Src>(eb, lb, vt, lt, lam2, n4, min(v + nt, last));
    L[v] = col_add<K, Rec>(col_prior<Src>(la, cutbits, i++), ea);
    v += nt;
    if (v >= s1) break;
    col_fetch<K, Src>(ea, la, vt, lt, lam2, n4, min(v + nt, last));
    L[v] = col_add<K, Rec>(col_prior<Src>(lb, cutbits, i++), eb);
    v += nt;
    if (v >= s1) break;
  }
  return i;
}

// Variable phase of a code whose columns have at most K <= 4 entries (K = the
// code's largest column degree, uniform; shorter columns are padded with the
// dummy check, whose r is -0), all slots as one run.  (Runs of one degree
// each, without padding, were measured slower: every run starts with its
// loads exposed.)
template <class Rec, int Src>
__device__ __forceinline__ void var_phase(int K, int n, float* L, const float* lam2, int tid, int nt, u32 cutbits,
                                          __amdgpu_buffer_rsrc_t vt, __amdgpu_buffer_rsrc_t lt, u32 n4) {
  switch (K) {
    case 4: var_run<4, Rec, Src>(L, lam2, 0, n, tid, nt, cutbits, 0, vt, lt, n4); break;
    case 3: var_run<3, Rec, Src>(L, lam2, 0, n, tid, nt, cutbits, 0, vt, lt, n4); break;
    case 2: var_run<2, Rec, Src>(L, lam2, 0, n, tid, nt, cutbits, 0, vt, lt, n4); break;
    case 1: var_run<1, Rec, Src>(L, lam2, 0, n, tid, nt, cutbits, 0, vt, lt, n4); break;
    default: {
      int i = 0;
      for (int v = tid; v < n; v += nt) {  // no column has a check: L = prior
        float lam;
        if constexpr (Src == kPriorLds) lam = lam2[v];
        else lam = __uint_as_float(vtab_at(lt, 0u, (u32)v << 2));
        L[v] = col_prior<Src>(lam, cutbits, i++);
      }
    }
  }
}

// Running state of a check over its row: min1, min2 and argmin of |q|, the
// sign word of q, and (bit `lane`) the parity of the hard decisions [L <= 0].
template <class Rec>
struct RowAcc {
  float m1, m2;
  int amin;
  typename Rec::Word sb;
  u64 pm;
};

// K consecutive row slots (from k0) of a check: q = L - r_old in row order,
// all loads issued before the updates.  r_old is alpha * (min2 on the old
// argmin, min1 elsewhere) with its sign bit (the magnitude is +0 or positive,
// alpha >= 0, or -0 on the dummy check, whose sign bits are 0).  q is not
// clamped to +-lsat: it enters the state only through its sign, which the
// clamp keeps, and through min / median operations against minima that start
// at lsat, which a |q| above lsat leaves as lsat itself would (+inf from a cut
// or dummy column included: r is finite).  A posterior is never -0 (it starts
// from a prior that is not -0 and adds messages; x + y is -0 only when both
// are), so q is never -0 and its sign bit is [q < 0]; the hard-decision parity
// takes one wave-wide compare per edge, the xor on the scalar unit.
template <int K, class Rec>
__device__ __forceinline__ void row_chunk(RowAcc<Rec>& a, const Rec& so, typename Rec::Word io, int am_old, int k0,
                                          __amdgpu_buffer_rsrc_t ct, u32 m4, u32 co) {
  u32 lo[K];
#pragma unroll
  for (int j = 0; j < K; ++j) lo[j] = vtab_at(ct, (u32)(k0 + j) * m4, co);
  float Lj[K];
#pragma unroll
  for (int j = 0; j < K; ++j) Lj[j] = *lds_at<float>(lo[j]);
  int amj = -1;  // position in the chunk of the newest minimum, if any (a constant per slot)
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int k = k0 + j;
    const float Lv = Lj[j];
    a.pm ^= __ballot(Lv <= 0.0f);
    const float mag = (am_old == k) ? so.a2 : so.a1;
    const float r = __uint_as_float(Rec::old_sign(io, k) | __float_as_uint(mag));
    const float q = Lv - r;
    const float aq = fabsf(q);
    const bool lt = aq < a.m1;
    amj = lt ? j : amj;
    a.m2 = __builtin_amdgcn_fmed3f(aq, a.m1, a.m2);
    a.m1 = lt ? aq : a.m1;
    a.sb = Rec::push_sign(a.sb, q, k);
  }
  a.amin = (amj >= 0) ? k0 + amj : a.amin;
}

// A whole row of K <= 8 slots as one chunk from position 0 (the same
// operations as row_chunk): the positions are constants, so the old-argmin
// test and the sign shift take inline constants and the new argmin is kept
// directly.
template <int K, class Rec>
__device__ __forceinline__ void row_whole(RowAcc<Rec>& a, const Rec& so, typename Rec::Word io, int am_old,
                                          __amdgpu_buffer_rsrc_t ct, u32 m4, u32 co) {
  u32 lo[K];
#pragma unroll
  for (int j = 0; j < K; ++j) lo[j] = vtab_at(ct, (u32)j * m4, co);
  float Lj[K];
#pragma unroll
  for (int j = 0; j < K; ++j) Lj[j] = *lds_at<float>(lo[j]);
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const float Lv = Lj[j];
    a.pm ^= __ballot(Lv <= 0.0f);
    const float mag = (am_old == j) ? so.a2 : so.a1;
    const float q = Lv - __uint_as_float(Rec::old_sign(io, j) | __float_as_uint(mag));
    const float aq = fabsf(q);
    const bool lt = aq < a.m1;
    a.amin = lt ? j : a.amin;
    a.m2 = __builtin_amdgcn_fmed3f(aq, a.m1, a.m2);
    a.m1 = lt ? aq : a.m1;
    a.sb = Rec::push_sign(a.sb, q, j);
  }
}
__device__ __forceinline__ float gloadf(const float* p, unsigned i) {
  return ((const __attribute__((address_space(1))) float*)p)[i];
}

// A value the whole wave holds (read from LDS or from memory at a uniform
// address) moved to scalar registers, so that the code description and every
// address derived from it stay scalar.
__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ long long uniform(long long x) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)(unsigned long long)x);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)((unsigned long long)x >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
template <class T>
__device__ __forceinline__ T* uniform(T* p) {
  return (T*)uniform((long long)(uintptr_t)p);
}

// The code description of shot b's code with every field in scalar registers
// (the compiler loads a struct from memory into vector registers unless it can
// prove nothing in the kernel writes that memory).
__device__ __forceinline__ GCode uniform_code(const GCode* codes, int ci) {
  GCode c = codes[ci];
  c.n = uniform(c.n); c.m = uniform(c.m); c.md = uniform(c.md);
  c.h_row_ptr = uniform(c.h_row_ptr); c.h_col = uniform(c.h_col); c.h_col_ptr = uniform(c.h_col_ptr);
  c.h_col_edge = uniform(c.h_col_edge); c.h_edge_row = uniform(c.h_edge_row);
  c.d_row_ptr = uniform(c.d_row_ptr); c.d_col = uniform(c.d_col); c.lam = uniform(c.lam);
  c.v_ell = uniform(c.v_ell); c.c_ell = uniform(c.c_ell); c.v_blk_deg = uniform(c.v_blk_deg);
  c.max_col_deg = uniform(c.max_col_deg); c.max_row_deg = uniform(c.max_row_deg);
  c.g_lam = uniform(c.g_lam);
  return c;
}

// A field of a code description read again where it is used (a volatile
// load, so that it does not occupy registers for the rest of the shot).
template <class T>
__device__ __forceinline__ T code_field(const T* p) {
  return uniform(*(const volatile T*)p);
}

// DC nomination of one row of D (the rule of bpdc_device.h's dc_pick, in the
// same float operations) streamed from the row's column list and the
// posteriors in LDS, with no per-thread arrays: the row maximum of the
// saturated posteriors, the tie threshold, the number of ties, then the
// chosen tie in ascending column order.
__device__ __forceinline__ int dc_pick_row(const int32_t* dcol, int e0, int deg, const float* L, float lsat,
                                           float tie_eps, int tie_lowest, u64 seed, u64 shot, u64 row,
                                           bool want_spread, int& spread) {
  float lmax = bpdc_dev::sat(L[gload(dcol, e0)], lsat), lmin = lmax;
  for (int k = 1; k < deg; ++k) {
    const float x = bpdc_dev::sat(L[gload(dcol, e0 + k)], lsat);
    lmax = fmaxf(lmax, x);
    lmin = fminf(lmin, x);
  }
  if (want_spread) spread = bpdc_dev::spread_bin_of(lmin, lmax);  // DC diagnostics (Appendix B)
  const float scale = fmaxf(1.0f, fabsf(lmax));
  const float thr = lmax - tie_eps * scale;
  int nt = 0;
  for (int k = 0; k < deg; ++k) nt += (bpdc_dev::sat(L[gload(dcol, e0 + k)], lsat) >= thr) ? 1 : 0;
  int want = 0;
  if (!tie_lowest && nt > 1) want = (int)bpdc_dev::scale_draw(bpdc_dev::tie_hash(seed, shot, row), (u32)nt);
  int seen = 0;
  for (int k = 0; k < deg; ++k) {
    const int col = gload(dcol, e0 + k);
    if (bpdc_dev::sat(L[col], lsat) >= thr) {
      if (seen == want) return col;
      ++seen;
    }
  }
  return gload(dcol, e0);
}

// At most 64 VGPRs (eight waves per SIMD): two workgroups of 1024 threads then
// share a compute unit, so one's barriers overlap the other's work (measured
// 1.3-1.5x over the 128-register build, whose single workgroup per CU stalls
// the unit at every barrier; the few spills are outside the inner loops).
// PS: the product-sum rule (Sec. II.C), rows of at most 8 edges: per-edge r
// in LDS instead of check records, in the log domain (phi of the leave-one-out
// sums of phi(|q|), left to right in row order) and the column sums in
// ascending check order, with bpdc_device.h's float32 phi, as in the plain and
// lane kernels.
template <bool Wide, bool PS>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) k_group(GArgs a) {
  // The kernel's LDS is this one block (no static LDS), so smem is LDS address
  // 0 and the code tables can hold absolute LDS byte addresses: 16 bytes of
  // control words, then the shot's state from kLdsHead on.
  extern __shared__ __align__(16) unsigned char smem[];
  long long& sIdx = *(long long*)smem;
  int* sUnsat = (int*)(smem + 8);  // stop-test flag, by iteration parity (read and reset with no barrier between)
  unsigned& sCount = *(unsigned*)(smem + 16);  // DC diagnostics: the shot's cut size
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwaves = nt >> 6;
  const KParams& P = a.p;
  const float LS = P.lsat;
  const float INF = __builtin_huge_valf();
  using Rec = CheckRec<Wide>;
  using W = typename Rec::Word;

  // shots of a mixed batch whose code index is out of range were flagged by the
  // ordering kernels and left out of `order`, which lists the others first
  const long long nshots = a.n_bad ? a.B - (long long)*a.n_bad : a.B;
  for (;;) {
    // claims of a.claim consecutive shots: the outputs of neighbouring shots
    // (small codes: a few words each) are then written from one L2
    if (tid == 0) sIdx = (long long)atomicAdd(a.queue, (unsigned long long)a.claim);
    __syncthreads();
    const long long first = uniform(sIdx);
    __syncthreads();
    if (first >= nshots) break;
    const long long last = first + a.claim < nshots ? first + a.claim : nshots;
    for (long long idx = first; idx < last; ++idx) {
      const long long b = a.order ? (long long)uniform(a.order[idx]) : idx;
      const int ci = a.code_of_shot ? uniform(a.code_of_shot[b]) : 0;
      // min-sum reads its tables as buffer resources built from a scalar code
      // description; product-sum reads them with plain loads, and the scalar
      // copy would only add scalar-register spills there
      const GCode C = PS ? a.codes[ci] : uniform_code(a.codes, ci);
      const int n = C.n, m = C.m;
      const int sw64 = (m + 63) >> 6, nw64 = (n + 63) >> 6;
      // LDS carve for this code; check m and column n are the dummies the
      // padding entries of the adjacency tables point at.  Product-sum keeps
      // the r of every edge (CSR order) where min-sum keeps check records.
      const int E = PS ? C.h_row_ptr[m] : 0;
      unsigned char* state = smem + kLdsHead;
      const __amdgpu_buffer_rsrc_t vt = table_rsrc(C.v_ell), ct = table_rsrc(C.c_ell),
                                   lt = table_rsrc((const int32_t*)(PS ? C.lam : C.g_lam));
      const u32 n4 = (u32)n * 4u, m4 = (u32)m * 4u;
      Rec* S = (Rec*)state;                          // [m + 1] check states (min-sum)
      float* R = (float*)state;                      // [E] per-edge r (product-sum)
      float* L = PS ? (float*)(state + (((size_t)E * 4 + 15) & ~(size_t)15)) : (float*)(S + m + 1);  // [n + 1]
      u32* cutw = (u32*)(L + n + 1);                 // [ceil(n/32)]
      u32* synw = cutw + ((n + 31) >> 5);            // [ceil(m/32)]
      // [n] per-shot prior: the first pass's under soft DC, the second pass's
      // with the posterior prior
      float* lam2 = (float*)(synw + ((m + 31) >> 5));
      const bool soft = P.soft_period > 0;
      // the 64-bit-record variant (rows above 32 edges: circuit-level DEMs, whose
      // column degrees differ from block to block) bounds each wave's column
      // chunks by its block's largest degree; the 32-bit variant keeps the
      // code's (fewer registers live)
      const bool blk_deg = Wide && (nt & 63) == 0;
      // the pipelined variable phase takes narrow-record min-sum codes whose
      // columns have 1 to 4 table entries
      const bool fast_cols = !Wide && !PS && C.max_col_deg <= 4;
      // dummies: a padded column entry adds r = -0 (x + -0 = x for every x), a
      // padded row entry reads L = +inf, so q saturates at lsat: it is never a
      // new minimum, leaves the second minimum (a median with lsat) and the
      // sign parity unchanged
      if (tid == 0) {
        if (!PS) S[m].set(-0.0f, -0.0f, 0, 0, m + kRec0);
        L[n] = INF;
      }

      const uint64_t* sp = a.syn + (a.syn_off ? a.syn_off[b] : b * sw64);
      for (int w = tid; w < ((m + 31) >> 5); w += nt) {
        const uint64_t x = sp[w >> 1];
        synw[w] = (w & 1) ? (u32)(x >> 32) : (u32)x;
      }
      for (int w = tid; w < ((n + 31) >> 5); w += nt) cutw[w] = 0u;
      // the syndrome bits of this thread's checks (check tid + k nt at bit k)
      // in a register when they fit (every code the LDS holds, with 1024
      // threads); otherwise the check phase reads them from LDS
      const bool reg_syn = m <= 32 * nt;
      u32 synbits = 0u;
      if (reg_syn)
        for (int c = tid, k = 0; c < m; c += nt, ++k) synbits |= (u32)((sp[c >> 6] >> (c & 63)) & 1u) << k;

      // iterations of each pass (scalars, not an array indexed by the pass: that
      // would live in per-thread scratch memory)
      int it0 = 0, it1 = 0;
      bool conv = false;
      for (int pass = 0; pass < 2; ++pass) {
        const int T = pass ? P.T2 : P.T1;
        const bool use_lam2 = (pass == 1 && P.second_pass_posterior) || (pass == 0 && soft);
        // the second pass under the channel prior keeps this thread's cut
        // columns as bits of a register (column tid + i nt at bit i), so the
        // pipelined variable phase needs at most 32 columns per thread
        // (slot tid + i nt at bit i: at most 32 slots per thread)
        const bool fast_var = fast_cols && (pass == 0 || use_lam2 || n <= 32 * nt);
        u32 cutbits = 0u;
        if (pass == 1 && fast_var && !use_lam2)
          for (int v = tid, i = 0; v < n; v += nt, ++i) cutbits |= ((cutw[v >> 5] >> (v & 31)) & 1u) << i;
        if (PS)
          for (int e = tid; e < E; e += nt) R[e] = 0.0f;
        else
          for (int c = tid; c < m; c += nt) S[c].set(0.0f, 0.0f, 0, 0, c + kRec0);
        if (pass == 0 && soft)
          for (int v = tid; v < n; v += nt) lam2[v] = (PS ? C.lam : code_field(&a.codes[ci].g_lam))[v];
        __syncthreads();
        int t = 0;
        for (;;) {
          // ---- variable phase: L = prior + sum of r (all zero at t = 0) ----
          // Only the second pass has cut columns (+inf: with the posterior prior
          // lam2 holds them); the first pass's priors are finite.
          const bool cuts = pass == 1;
          if (fast_var) {
            // narrow records, columns of at most 4 entries: the pipelined phase
            const int Kc = C.max_col_deg;
            if (use_lam2) var_phase<Rec, kPriorLds>(Kc, n, L, lam2, tid, nt, 0u, vt, lt, n4);
            else if (cuts) var_phase<Rec, kPriorTableCut>(Kc, n, L, lam2, tid, nt, cutbits, vt, lt, n4);
            else var_phase<Rec, kPriorTable>(Kc, n, L, lam2, tid, nt, 0u, vt, lt, n4);
          } else
          for (int v = tid; v < n; v += nt) {
            const u32 vo = (u32)v << 2;
            float Lv;
            if (use_lam2) Lv = lam2[v];
            else if (cuts && ((cutw[v >> 5] >> (v & 31)) & 1u)) Lv = INF;
            else Lv = __uint_as_float(vtab_at(lt, 0u, vo));
            if (PS && (!cuts || Lv != INF)) {
              for (int k = C.h_col_ptr[v]; k < C.h_col_ptr[v + 1]; ++k) Lv = Lv + R[gload(C.h_col_edge, k)];
            } else if (!PS && (!cuts || Lv != INF)) {
              // entries in chunks of 4 and a last chunk of kend mod 4; padding
              // entries of columns shorter than kend read the dummy check and add
              // -0 (x + -0 = x).  A wave holds 64 consecutive columns (v = tid +
              // k nt with nt a multiple of 64), so it can stop at the largest
              // degree of its block (a wave-uniform bound) instead of the code's
              const int kend = blk_deg ? __builtin_amdgcn_readfirstlane(gload(C.v_blk_deg, v >> 6)) : C.max_col_deg;
              int k0 = 0;
              for (; k0 + 4 <= kend; k0 += 4) Lv = col_sum<4, Rec>(Lv, vt, n4, vo, k0);
              switch (kend - k0) {  // uniform
                case 1: Lv = col_sum<1, Rec>(Lv, vt, n4, vo, k0); break;
                case 2: Lv = col_sum<2, Rec>(Lv, vt, n4, vo, k0); break;
                case 3: Lv = col_sum<3, Rec>(Lv, vt, n4, vo, k0); break;
                default: break;
              }
            }
            L[v] = Lv;
          }
          if (tid == 0) sUnsat[t & 1] = 0;
          __syncthreads();
          // ---- check phase: next check state from q = L - r_old, with the stop
          // test H e = s (e = [L <= 0]) on the way; the new state is not used
          // when the pass ends here ----
          int bad = 0;
          if constexpr (PS) {
            for (int c = tid; c < m; c += nt) {
              const int e0 = gload(C.h_row_ptr, c), deg = gload(C.h_row_ptr, c + 1) - e0;
              const u32 sbit = (synw[c >> 5] >> (c & 31)) & 1u;
              u32 par = sbit, neg = sbit, qn = 0u;
              float ph[8];
  #pragma unroll
              for (int j = 0; j < 8; ++j) {
                ph[j] = 0.0f;
                if (j < deg) {
                  const float Lv = L[gload(C.h_col, e0 + j)];
                  par ^= (Lv <= 0.0f) ? 1u : 0u;
                  const float q = bpdc_dev::ps_q(Lv, R[e0 + j], LS);  // +inf from a cut column
                  const u32 qneg = (q < 0.0f) ? 1u : 0u;
                  neg ^= qneg;
                  qn |= qneg << j;
                  ph[j] = bpdc_dev::phi(fabsf(q));
                }
              }
  #pragma unroll
              for (int j = 0; j < 8; ++j) {
                if (j < deg) {
                  // phi of the sum of the other edges' phi, left to right in row order
                  float sum = 0.0f;
  #pragma unroll
                  for (int o = 0; o < 8; ++o)
                    if (o != j && o < deg) sum = sum + ph[o];
                  float mag = bpdc_dev::phi(sum);
                  if (!(mag < LS)) mag = LS;
                  const float val = P.alpha * mag;
                  R[e0 + j] = (neg ^ ((qn >> j) & 1u)) ? -val : val;
                }
              }
              bad |= (int)par;
            }
          } else
          for (int c = tid, k = 0; c < m; c += nt, ++k) {
            const Rec so = S[c];
            RowAcc<Rec> acc{LS, LS, 0, 0, 0u};
            // the check table holds the LDS address of each entry's L; the
            // code's largest row degree in chunks of 8, then 4, 2, 1 (uniform
            // branches; padding entries of shorter rows read the dummy column,
            // L = +inf, whose q saturates and changes nothing)
            const u32 co = (u32)c << 2;
            const W io = so.signs();
            const int am_old = so.argmin(), K = C.max_row_deg;
            bool whole = false;
            if constexpr (!Wide) {
              whole = K <= 8;
              switch (K) {  // uniform
                case 8: row_whole<8, Rec>(acc, so, io, am_old, ct, m4, co); break;
                case 7: row_whole<7, Rec>(acc, so, io, am_old, ct, m4, co); break;
                case 6: row_whole<6, Rec>(acc, so, io, am_old, ct, m4, co); break;
                case 5: row_whole<5, Rec>(acc, so, io, am_old, ct, m4, co); break;
                case 4: row_whole<4, Rec>(acc, so, io, am_old, ct, m4, co); break;
                case 3: row_whole<3, Rec>(acc, so, io, am_old, ct, m4, co); break;
                case 2: row_whole<2, Rec>(acc, so, io, am_old, ct, m4, co); break;
                case 1: row_whole<1, Rec>(acc, so, io, am_old, ct, m4, co); break;
                default: break;
              }
            }
            if (!whole) {
              int k0 = 0;
              for (; k0 + 8 <= K; k0 += 8) row_chunk<8, Rec>(acc, so, io, am_old, k0, ct, m4, co);
              if ((K - k0) & 4) { row_chunk<4, Rec>(acc, so, io, am_old, k0, ct, m4, co); k0 += 4; }
              if ((K - k0) & 2) { row_chunk<2, Rec>(acc, so, io, am_old, k0, ct, m4, co); k0 += 2; }
              if ((K - k0) & 1) row_chunk<1, Rec>(acc, so, io, am_old, k0, ct, m4, co);
            }
            const W sb = Rec::finish_signs(acc.sb, K);
            const float m1 = acc.m1, m2 = acc.m2;
            const int amin = acc.amin;
            u32 sbit;
            if (reg_syn) sbit = (synbits >> k) & 1u;
            else sbit = (synw[c >> 5] >> (c & 31)) & 1u;
            // stop test on the wave's checks (a prefix of its lanes is active,
            // lane 0 among them): hard-decision parity against the syndrome
            // (a plain store of 1: every writer stores the same value)
            if ((acc.pm ^ __ballot(sbit != 0u)) != 0ull && lane == 0)
              __hip_atomic_store(&sUnsat[t & 1], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            // parity of the q signs and the syndrome bit: bit 0 of their sum
            const u32 rp = ((u32)popc_word(sb) + sbit) & 1u;
            // flip every sign bit on an odd parity: the bits past the row's
            // degree are read only by padding entries, whose q saturates anyway
            const W rb = rp ? (sb ^ Rec::kSignMask) : sb;
            S[c].set(P.alpha * m1, P.alpha * m2, rb, amin, c + kRec0);
          }
          if (PS && __ballot(bad) != 0ull && lane == 0) atomicOr(&sUnsat[t & 1], 1);
          __syncthreads();
          if (t >= 1) {
            const bool ok = sUnsat[t & 1] == 0;
            if ((P.stop && ok) || t >= T) {
              conv = ok;
              if (pass) it1 = t;
              else it0 = t;
              break;
            }
            // intermittent soft DC (application j = t / soft_period of the first
            // pass): the rows of D nominate on this iteration's posteriors (row h
            // hashed as j * rows(D) + h), the nominees' priors rise by soft_shift;
            // cutw (empty during the first pass) collects the nominees
            if (pass == 0 && soft && !ok && t % P.soft_period == 0) {
              const u64 rbase = (u64)(t / P.soft_period) * (u64)C.md;
              for (int h = tid; h < C.md; h += nt) {
                const int e0 = C.d_row_ptr[h], deg = C.d_row_ptr[h + 1] - e0;
                if (deg == 0) continue;
                int unused_bin = 0;
                const int pick = dc_pick_row(PS ? C.d_col : code_field(&a.codes[ci].g_dcol), e0, deg, L, LS, P.tie_eps, P.tie_lowest, P.seed,
                                             (u64)(a.shot_offset + b), rbase + (u64)h, false, unused_bin);
                atomicOr(&cutw[pick >> 5], 1u << (pick & 31));
              }
              __syncthreads();
              for (int v = tid; v < n; v += nt)
                if ((cutw[v >> 5] >> (v & 31)) & 1u) lam2[v] = lam2[v] + P.soft_shift;
              __syncthreads();
              for (int w = tid; w < ((n + 31) >> 5); w += nt) cutw[w] = 0u;
              __syncthreads();
            }
          }
          ++t;
        }
        if (pass == 1 || conv) break;
        // ---- degeneracy cutting (first pass failed) ----
        // With diagnostics on, each row's spread bin goes to a histogram of the
        // shot in LDS over the check-state region (free between the passes),
        // flushed once per shot; a code whose region holds fewer than 101 bins
        // adds to the device histogram directly.
        const bool dcs = a.dcstats != nullptr;
        u32* hist = (u32*)state;
        const bool lds_hist = dcs && (PS ? (size_t)E * 4 : (size_t)(m + 1) * 16) >= 101 * sizeof(u32);
        if (lds_hist) {
          for (int i = tid; i < 101; i += nt) hist[i] = 0u;
          if (tid == 0) sCount = 0u;
          __syncthreads();
        } else if (dcs && tid == 0) {
          sCount = 0u;  // ordered before its use by the barrier after the rows
        }
        for (int h = tid; h < C.md; h += nt) {
          const int e0 = C.d_row_ptr[h], deg = C.d_row_ptr[h + 1] - e0;
          if (deg == 0) continue;
          int bin = 0;
          const int pick = dc_pick_row(PS ? C.d_col : code_field(&a.codes[ci].g_dcol), e0, deg, L, LS, P.tie_eps, P.tie_lowest, P.seed,
                                       (u64)(a.shot_offset + b), (u64)h, dcs, bin);
          atomicOr(&cutw[pick >> 5], 1u << (pick & 31));
          if (lds_hist) atomicAdd(&hist[bin], 1u);
          else if (dcs) atomicAdd(&a.dcstats[bin], 1ull);
        }
        __syncthreads();
        if (dcs) {
          if (lds_hist)
            for (int i = tid; i < 101; i += nt)
              if (hist[i]) atomicAdd(&a.dcstats[i], (unsigned long long)hist[i]);
          unsigned nc = 0;
          for (int w = tid; w < ((n + 31) >> 5); w += nt) nc += (unsigned)__builtin_popcount(cutw[w]);
          if (nc) atomicAdd(&sCount, nc);
        }
        if (P.second_pass_posterior)
          for (int v = tid; v < n; v += nt)
            lam2[v] = ((cutw[v >> 5] >> (v & 31)) & 1u) ? INF : bpdc_dev::sat(L[v], LS);
        __syncthreads();
        if (dcs && tid == 0) {  // the shot ran DC; its cut size
          atomicAdd(&a.dcstats[101], 1ull);
          atomicAdd(&a.dcstats[102 + sCount], 1ull);
        }
      }
      // ---- outputs ----
      const bool dc = it1 > 0;
      uint64_t* cp = a.corr + (a.corr_off ? a.corr_off[b] : b * nw64);
      // (column v's posterior and cut bit sit at its slot: v itself for
      // product-sum)
      const int32_t* gpos = PS ? nullptr : code_field(&a.codes[ci].g_pos);
      for (int w = wave; w < nw64; w += nwaves) {
        const int v = w * 64 + lane;
        const int sv = v < n ? (PS ? v : gload(gpos, (unsigned)v)) : n;
        const u64 word = __ballot(v < n && L[sv] <= 0.0f);
        if (lane == 0) cp[w] = word;
        if (a.cut) {
          const u64 cw = __ballot(dc && v < n && ((cutw[sv >> 5] >> (sv & 31)) & 1u));
          if (lane == 0) a.cut[b * nw64 + w] = cw;
        }
      }
      if (a.post)
        for (int v = tid; v < n; v += nt) {
          const float x = L[PS ? v : gload(gpos, (unsigned)v)];
          a.post[b * n + v] = (x == INF) ? x : bpdc_dev::sat(x, LS);
        }
      if (tid == 0) {
        a.flags[b] = (uint8_t)((conv ? 1 : 0) | (dc ? 2 : 0));
        if (a.iters) {
          a.iters[2 * b] = (int16_t)it0;
          a.iters[2 * b + 1] = (int16_t)it1;
        }
      }
      __syncthreads();
    }
  }
}

// Processing order of a mixed batch: shots grouped by code, codes by
// descending column count (counting sort; order within a code is arbitrary,
// results do not depend on it).  A code index outside [0, ncodes) counts in
// the extra bucket ncodes: such a shot gets the flags value kFlagBadCode here
// and no place in the order, and the decode kernel stops after the others
// (a skip inside its loop would put a thread-0 branch between barriers).
__device__ __forceinline__ int order_bucket(const int32_t* code_of_shot, int64_t i, int ncodes) {
  const int c = code_of_shot[i];
  return ((unsigned)c < (unsigned)ncodes) ? c : ncodes;
}
__global__ void k_order_hist(const int32_t* code_of_shot, int64_t B, int ncodes, unsigned* hist) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) atomicAdd(&hist[order_bucket(code_of_shot, i, ncodes)], 1u);
}
__global__ void k_order_scan(const int32_t* code_by_rank, int ncodes, const unsigned* hist, unsigned* base) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned s = 0;
  for (int r = 0; r < ncodes; ++r) {
    const int c = code_by_rank[r];
    base[c] = s;
    s += hist[c];
  }
}
__global__ void k_order_scatter(const int32_t* code_of_shot, int64_t B, int ncodes, unsigned* base,
                                int32_t* order, uint8_t* flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B) return;
  const int c = order_bucket(code_of_shot, i, ncodes);
  if (c == ncodes) flags[i] = kFlagBadCode;
  else order[atomicAdd(&base[c], 1u)] = (int32_t)i;
}

__global__ void k_zero_u32(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

}  // namespace

size_t group_lds_bytes_nm(int n, int m, bool posterior, int info_bytes, int edges) {
  // check records [m + 1] (16 bytes each, either width) or, for product-sum
  // (info_bytes 0), the per-edge r [edges]; L[n + 1], cut and syndrome words,
  // per-shot prior
  size_t words = (size_t)(n + 1) + ((n + 31) / 32) + ((m + 31) / 32) + (posterior ? n : 0);
  const size_t head = info_bytes == 0 ? (((size_t)edges * 4 + 15) & ~(size_t)15) : (size_t)(m + 1) * 16;
  return kLdsHead + head + words * 4;
}

hipError_t group_launch(const void* d_codes, const unsigned* n_bad, const int32_t* code_of_shot,
                        const int32_t* order, const KParams& p, const uint64_t* syn, const int64_t* syn_off, uint64_t* corr,
                        const int64_t* corr_off, uint8_t* flags, float* post, uint64_t* cut,
                        int16_t* iters, int64_t B, int64_t shot_offset, int threads, int grid,
                        size_t lds, int info_bytes, unsigned long long* queue, hipStream_t stream,
                        unsigned long long* dcstats, int claim_n) {
  GArgs a;
  a.dcstats = dcstats;
  // single-code launches of small codes: up to 8 consecutive shots per claim,
  // about one 128-byte line of corrections (n is the code's column count)
  a.claim = 1;
  if (!code_of_shot && claim_n > 0) {
    const int nw = (claim_n + 63) / 64;
    a.claim = std::max(1, std::min(8, 16 / nw));
  }
  a.codes = (const GCode*)d_codes;
  a.code_of_shot = code_of_shot;
  a.n_bad = n_bad;
  a.order = order;
  a.syn = syn;
  a.syn_off = syn_off;
  a.corr = corr;
  a.corr_off = corr_off;
  a.flags = flags;
  a.post = post;
  a.cut = cut;
  a.iters = iters;
  a.B = B;
  a.shot_offset = shot_offset;
  a.queue = queue;
  a.p = p;
  (void)hipGetLastError();  // report only this launch's errors
  hipError_t e = fill_u64((uint64_t*)queue, 0, 1, stream);
  if (e != hipSuccess) return e;
  if (info_bytes == 8) hipLaunchKernelGGL((k_group<true, false>), dim3(grid), dim3(threads), lds, stream, a);
  else if (info_bytes == 0) hipLaunchKernelGGL((k_group<false, true>), dim3(grid), dim3(threads), lds, stream, a);
  else hipLaunchKernelGGL((k_group<false, false>), dim3(grid), dim3(threads), lds, stream, a);
  return hipGetLastError();
}

// Allow the group kernels up to `max_lds` bytes of dynamic LDS (once per
// process and device), then report how many workgroups of `threads` threads
// and `lds` bytes fit on a compute unit.
int group_occupancy(int threads, size_t lds, int info_bytes, int max_lds) {
  // raise the dynamic-LDS limit of both instantiations once; a refusal leaves
  // the default limit (and its error is cleared so that it is not reported
  // by a later launch check)
  static int raised_to = -1;
  if (raised_to != max_lds) {
    if (hipFuncSetAttribute((const void*)k_group<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            max_lds) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_group<true, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            max_lds) != hipSuccess ||
        hipFuncSetAttribute((const void*)k_group<false, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            max_lds) != hipSuccess)
      (void)hipGetLastError();
    raised_to = max_lds;
  }
  int nb = 0;
  hipError_t e =
      info_bytes == 8   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_group<true, false>, threads, lds)
      : info_bytes == 0 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_group<false, true>, threads, lds)
                        : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_group<false, false>, threads, lds);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

bool group_lds_starts_at_zero() {
  const void* ks[] = {(const void*)k_group<false, false>, (const void*)k_group<true, false>,
                      (const void*)k_group<false, true>};
  for (const void* k : ks) {
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, k) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    if (fa.sharedSizeBytes != 0) return false;
  }
  return true;
}

hipError_t group_order(const int32_t* code_of_shot, int64_t B, const int32_t* code_by_rank, int ncodes,
                       unsigned* hist, unsigned* base, int32_t* order, uint8_t* flags, hipStream_t stream) {
  // hist and base hold ncodes + 1 buckets (the last one: out-of-range code indices)
  hipLaunchKernelGGL(k_zero_u32, dim3((ncodes + 1 + 255) / 256), dim3(256), 0, stream, hist, ncodes + 1);
  const unsigned g = (unsigned)((B + 255) / 256);
  if (B > 0) hipLaunchKernelGGL(k_order_hist, dim3(g), dim3(256), 0, stream, code_of_shot, B, ncodes, hist);
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, stream, code_by_rank, ncodes, hist, base);
  if (B > 0)
    hipLaunchKernelGGL(k_order_scatter, dim3(g), dim3(256), 0, stream, code_of_shot, B, ncodes, base, order, flags);
  return hipGetLastError();
}

}  // namespace bpdc
