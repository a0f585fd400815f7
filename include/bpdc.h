/*
 * bpdc.h -- C ABI of the MI355X (gfx950) BP+DC decoder library, libbpdc.so.
 *
 * BP+DC (degeneracy cutting, arXiv 2510.08695): scaled min-sum belief
 * propagation on the Tanner graph of a parity-check matrix H (H_Z, or a
 * detector check matrix), then -- only for shots whose first pass did not
 * reproduce the syndrome -- every row of a degeneracy matrix D (H_X, or a
 * detector degeneracy matrix) nominates the variable of highest posterior LLR
 * (= lowest posterior error probability) in its support, the nominees are cut
 * (prior probability 0), and BP is run again (Algorithm 1 with the cut of
 * Algorithm 2, Sec. III.A; the detector-error-model form of Sec. IV.B).
 *
 * Conventions for every entry point:
 *  - Every function returns bpdc_status; 0 (BPDC_OK) is success.  Nothing
 *    throws across the ABI.  On a non-OK return, bpdc_last_error() gives a
 *    thread-local message.
 *  - Pointers named h_* are host memory, d_* are device memory on the
 *    current HIP device.  The caller owns every h_* and d_* buffer; the
 *    library owns the handles and its own device copies of H, D and the priors.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work of a call is enqueued on it asynchronously; the only
 *    host-synchronising calls are bpdc_code_create / bpdc_plan_create.
 *  - Bit vectors are packed little-endian: bit j of a vector is bit (j & 63)
 *    of 64-bit word (j >> 6).  Padding bits are ignored on input and written
 *    as 0 on output.
 *  - Results depend only on (code, params, syndrome, seed, shot_offset + index
 *    of the shot), never on the kernel variant, tile shape, batch split or
 *    stream.
 */
#ifndef BPDC_H
#define BPDC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bpdc_status;
enum {
  BPDC_OK = 0,
  BPDC_ERR_INVALID_ARG = 1, /* null pointer, negative size, bad CSR, p outside (0,1), ... */
  BPDC_ERR_UNSUPPORTED = 2, /* degree above the compiled limit, kernel variant not available */
  BPDC_ERR_WORKSPACE = 3,   /* workspace missing or smaller than bpdc_workspace_size() */
  BPDC_ERR_HIP = 4,         /* a HIP runtime call failed (message in bpdc_last_error) */
  BPDC_ERR_OOM = 5          /* device allocation failed */
};

/* Second-pass prior (Sec. III.B): the channel prior p (BB codes) or the
 * first-pass posteriors (surface / toric codes).  Cut variables always get
 * prior probability 0 (Algorithm 2). */
enum { BPDC_PRIOR_CHANNEL = 0, BPDC_PRIOR_POSTERIOR = 1 };

/* Tie-break among DC candidates of equal posterior (Sec. III.A: "selected at
 * random"): a counter-based SplitMix64 hash of (seed, shot, row), or the
 * lowest column index. */
enum { BPDC_TIE_HASH = 0, BPDC_TIE_LOWEST_INDEX = 1 };

/* Check-node rule of BP (Sec. II.C names both): scaled min-sum,
 * r = alpha * min over the other |q|, or product-sum,
 * r = alpha * 2 atanh(prod over the other tanh(|q| / 2)) (alpha = 1 for the
 * plain rule), each saturated at llr_sat and signed by the syndrome bit and
 * the other signs.  Product-sum is evaluated in the log domain,
 * r = alpha * phi(sum over the other phi(|q|)) with phi(x) = -ln tanh(x / 2),
 * the same function without the rounding of a product of tanh values to 1;
 * a cut column (prior probability 0) sends +inf, i.e. phi = 0.  Product-sum runs on the plain kernel family, on the lane
 * family for codes of at most 96 edges (one lane per shot) and on the group
 * family for rows of at most 8 edges; not in the multi-code launch or
 * weighted decoding. */
enum { BPDC_RULE_MIN_SUM = 0, BPDC_RULE_PRODUCT_SUM = 1 };

/* Kernel family of a plan. */
enum {
  BPDC_KERNEL_AUTO = 0,  /* autotuner picks among the fused variants */
  BPDC_KERNEL_PLAIN = 1, /* one launch per BP phase per iteration, messages in HBM */
  BPDC_KERNEL_LANE = 2,  /* fused persistent BP->DC->BP, one shot per lane, code-specialised */
  BPDC_KERNEL_GROUP = 3  /* fused persistent BP->DC->BP, shots per workgroup, state in LDS */
};

/* Binary matrix in CSR form (host memory): 0-based column indices, sorted and
 * unique within each row.  row_ptr has rows + 1 entries. */
typedef struct {
  int32_t rows, cols;
  const int32_t* row_ptr;
  const int32_t* col_idx;
} bpdc_csr;

/* Decoder parameters (the paper leaves the min-sum scale, the saturation and
 * the tie tolerance open; these are the knobs). */
typedef struct {
  int32_t max_iter[2];       /* T before DC, T after DC (each >= 1) */
  float alpha;               /* min-sum scale: r = alpha * min |q| (finite, >= 0) */
  int32_t second_pass_prior; /* BPDC_PRIOR_* */
  int32_t stop_on_converge;  /* 1: stop a pass once H e = s (Sec. II.C); 0: run all iterations */
  float llr_sat;             /* messages and reported posteriors saturate at +-llr_sat (> 0, finite) */
  float tie_eps;             /* DC tie set: L_i >= L_max - tie_eps * max(1, |L_max|) (>= 0) */
  int32_t tie_break;         /* BPDC_TIE_* */
  uint64_t seed;             /* tie-break hash seed */
  int32_t rule;              /* BPDC_RULE_* */
  /* Intermittent soft DC (the extension Sec. V proposes; 0 = off): every
   * soft_period iterations of the first pass (t = K, 2K, ... < T1), on every
   * shot whose H e != s, each row of D nominates as in DC on the saturated
   * posteriors of that iteration (the j-th application hashes row h as
   * j * rows(D) + h), and every nominee's prior LLR rises by soft_shift
   * (>= 0, finite), i.e. its prior error odds p / (1 - p) shrink by the factor
   * e^-soft_shift; messages carry on.  The DC after a failed first pass and
   * the second pass are unchanged (the channel second-pass prior is the
   * unshifted one).  All three kernel families with min-sum (the lane family
   * as its own code-specialised variant), the group and plain families with
   * product-sum; weighted decoding returns BPDC_ERR_UNSUPPORTED. */
  int32_t soft_period;
  float soft_shift;
} bpdc_params;

typedef struct bpdc_code_s* bpdc_code; /* immutable after creation */
typedef struct bpdc_plan_s* bpdc_plan; /* launch configuration for one or more codes */

/* Load a decoding problem: Tanner graph H (m x n), degeneracy matrix D
 * (m' x n, same n) and per-column prior error probabilities h_priors[n], each
 * in (0, 1).  These are Algorithm 1's inputs (Sec. III.A): H = H_Z, whose
 * syndrome is decoded, D = H_X, whose rows nominate the columns to cut, and the
 * channel error probability p of each column (code capacity, Sec. II.C); for
 * a detector error model (Sec. IV.B) H is the detector check matrix, D the
 * detector degeneracy matrix and p the probability of each fault mechanism.  The prior LLRs log((1-p)/p) are evaluated in double and rounded
 * once to float.  Copies everything to the current device; synchronous.
 * Row degree of H is limited to 64, column degree of H to 16, row degree of D
 * to 32 (BPDC_ERR_UNSUPPORTED otherwise); the group kernel family runs rows
 * of up to 58 edges (product-sum: 8), the plain family product-sum rows of
 * up to 32. */
bpdc_status bpdc_code_create(const bpdc_csr* H, const bpdc_csr* D, const double* h_priors,
                             bpdc_code* out);
bpdc_status bpdc_code_destroy(bpdc_code code);
/* Sizes of a code: n columns, m rows of H, m' rows of D, E edges of H. */
bpdc_status bpdc_code_info(bpdc_code code, int32_t* n, int32_t* m, int32_t* md, int32_t* edges);

/* Build a plan for `ncodes` codes (they stay owned by the caller and must
 * outlive the plan); synchronous.  `kernel` is a BPDC_KERNEL_* value.  The
 * plan's autotuner times candidate launch shapes on synthetic shots drawn
 * from each code's own priors and keeps the fastest per shot:
 *  - lane family: lanes per shot (1, 2 or 4, as the code's symmetry allows:
 *    64, 32 or 16 shots per one-wave workgroup) x the largest claim of shots
 *    a wave stages in LDS (8, 16 or 32), each a code-specialised compile
 *    (cached on disk; bpdc_lane_precompile fills the cache);
 *  - group family: threads per workgroup (64 ... 1024, one shot per
 *    workgroup, its state in LDS), ranked on a batch in which every shot
 *    runs min(16, T) iterations per pass without early stop (so that a few
 *    long shots of a short batch cannot turn the time into one shot's
 *    latency);
 *  - AUTO: when both fused families can run a code, both are tuned and the
 *    faster per shot is kept (the group tile chosen as above, timed again
 *    with the plan's iterations); otherwise the one that can (else plain);
 *  - the multi-code launch (more than one code): threads per workgroup timed
 *    on a synthetic mixed batch of every code, ranked the same way.
 * bpdc_plan_describe reports the choices and the timings.
 * BPDC_ERR_UNSUPPORTED if the requested variant cannot run a code. */
bpdc_status bpdc_plan_create(const bpdc_code* codes, int32_t ncodes, const bpdc_params* params,
                             int32_t kernel, bpdc_plan* out);
bpdc_status bpdc_plan_destroy(bpdc_plan plan);
/* The variant and tile a plan chose for code `code`: kernel (BPDC_KERNEL_*),
 * shots per workgroup (lane: 64 / lanes per shot; group: 1; plain: 256, one
 * shot per thread), threads per workgroup. */
bpdc_status bpdc_plan_info(bpdc_plan plan, int32_t code, int32_t* kernel, int32_t* shots_per_wg,
                           int32_t* threads_per_wg);
/* The autotuner's record for code `code` (or, with code = -1, the multi-code
 * launch) as a JSON object written to buf (host, cap bytes, NUL-terminated,
 * truncated to fit): the family and tile kept, why, and every candidate timed
 * with its time per 1000 synthetic shots (group and multi-code candidates on
 * the fixed-iteration batch; under AUTO, one more group entry: the chosen
 * tile with the plan's iterations).  *needed (optional) gets the full length
 * + 1. */
bpdc_status bpdc_plan_describe(bpdc_plan plan, int32_t code, char* buf, size_t cap, size_t* needed);

/* Diagnostics of degeneracy cutting (Appendix B: how flat are the posterior
 * profiles DC picks from; how many columns it cuts).  While a buffer is set,
 * every bpdc_decode of the plan adds, for each shot whose first pass failed,
 * into d_stats (uint64 words on the plan's device, zeroed by the caller,
 * updated with device atomics; the caller owns it):
 *   [0, 101)     histogram over the rows h of D of the spread
 *                Delta(h) = max - min of the first-pass posterior error
 *                probabilities 1 / (1 + e^L) over the support of h, at bin
 *                floor(100 Delta) (bin 100: Delta = 1);
 *   [101]        number of shots that ran DC;
 *   [102, 103+n) histogram of the cut size 0..n.
 * words >= 103 + n of the decoded code (bpdc_decode_multi: of the plan's
 * largest code; checked at decode time).  d_stats = NULL turns it off.  Every
 * kernel family and bpdc_decode_multi; bpdc_graph_capture_multi returns
 * BPDC_ERR_UNSUPPORTED while set (a captured graph would keep the buffer). */
bpdc_status bpdc_plan_set_dc_stats(bpdc_plan plan, uint64_t* d_stats, int64_t words);

/* Device workspace (bytes) that bpdc_decode needs for a batch of B shots of
 * code `code` (bpdc_decode_multi: pass code = -1 and the total batch). */
bpdc_status bpdc_workspace_size(bpdc_plan plan, int32_t code, int64_t B, size_t* bytes);

/* Decode B shots of code `code` (index into the plan's code list): Algorithm 1
 * (Sec. III.A) per shot -- BP_decode on the syndrome (Sec. II.C: flooding
 * updates, hard decision e = [p >= 1/2] of Eq. (3), stop once H e = s), and on
 * shots where it fails, degeneracy cutting over the rows of D and a second
 * BP_decode on the cut graph with the cut columns at prior probability 0
 * (Algorithm 2); the outputs are BP_decode's estimate and posteriors.
 *   d_syn   [B][ceil(m/64)] uint64 packed syndromes (input)
 *   d_corr  [B][ceil(n/64)] uint64 packed corrections e_hat (output; cut columns are 0)
 *   d_flags [B] uint8: bit 0 = H e_hat = s, bit 1 = DC ran (output)
 *   d_post  [B][n] float posterior LLRs of the final pass, saturated, +inf on cut
 *           columns (optional, may be NULL)
 *   d_cut   [B][ceil(n/64)] uint64 cut set, all zero where DC did not run (optional)
 *   d_iters [B][2] int16 iterations executed before / after DC (optional)
 *   shot_offset: global index of shot 0 (tie-break hash counter)
 *   d_ws, ws_bytes: workspace of at least bpdc_workspace_size() bytes. */
bpdc_status bpdc_decode(bpdc_plan plan, int32_t code, const uint64_t* d_syn, int64_t B,
                        int64_t shot_offset, uint64_t* d_corr, uint8_t* d_flags, float* d_post,
                        uint64_t* d_cut, int16_t* d_iters, void* d_ws, size_t ws_bytes,
                        void* stream);

/* bpdc_decode for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops and harnesses that must not call hipMalloc):
 * the same arguments without the workspace, which comes from a static
 * device array of BPDC_NOALLOC_SCRATCH_BYTES bytes inside the library (each
 * GPU the library runs on holds its own copy until the process ends).  The
 * call allocates nothing.  A batch whose workspace (bpdc_workspace_size)
 * exceeds BPDC_NOALLOC_SCRATCH_BYTES is refused with BPDC_ERR_WORKSPACE (a
 * BB[[144,12,12]] plan on the lane family fits about 2e6 shots; the plain
 * family needs about 8 E + 8 n bytes per shot).  Every call on one GPU uses
 * that GPU's one array, whose contents persist from the previous call (the
 * kernels clear what must start at zero), so calls that overlap in time on
 * one GPU (two streams, two threads) race and must be serialised by the
 * caller.  Results equal bpdc_decode's. */
#define BPDC_NOALLOC_SCRATCH_BYTES (32u << 20)
bpdc_status bpdc_decode_noalloc(bpdc_plan plan, int32_t code, const uint64_t* d_syn, int64_t B,
                                int64_t shot_offset, uint64_t* d_corr, uint8_t* d_flags,
                                float* d_post, uint64_t* d_cut, int16_t* d_iters, void* stream);

/* Decode a mixed batch of B shots over all codes of the plan in one persistent
 * launch.  Shot b belongs to code d_code_of_shot[b]; its syndrome starts at
 * word d_syn_off[b] of d_syn and its correction at word d_corr_off[b] of d_corr.
 * d_flags [B], d_iters [B][2] (optional) as in bpdc_decode.  The tie-break
 * counter of shot b is shot_offset + b.  The code indices are read on the
 * device, so they cannot be validated before the launch: a shot whose index
 * lies outside [0, ncodes) is skipped, its flags byte is set to
 * BPDC_FLAG_BAD_CODE and its correction and iteration counts are left
 * unwritten (its syndrome and correction offsets are never read). */
#define BPDC_FLAG_BAD_CODE 0x80
bpdc_status bpdc_decode_multi(bpdc_plan plan, const int32_t* d_code_of_shot, const uint64_t* d_syn,
                              const int64_t* d_syn_off, uint64_t* d_corr, const int64_t* d_corr_off,
                              uint8_t* d_flags, int16_t* d_iters, int64_t B, int64_t shot_offset,
                              void* d_ws, size_t ws_bytes, void* stream);

/* Capture bpdc_decode_multi with fixed buffers into a HIP graph owned by the
 * plan; bpdc_graph_launch replays it on `stream`. */
bpdc_status bpdc_graph_capture_multi(bpdc_plan plan, const int32_t* d_code_of_shot,
                                     const uint64_t* d_syn, const int64_t* d_syn_off,
                                     uint64_t* d_corr, const int64_t* d_corr_off, uint8_t* d_flags,
                                     int16_t* d_iters, int64_t B, int64_t shot_offset, void* d_ws,
                                     size_t ws_bytes, void* stream);
bpdc_status bpdc_graph_launch(bpdc_plan plan, void* stream);

/* Weighted min-sum (learned per-edge scales, one set per pass): the forward
 * runs T1 iterations, DC on shots whose first pass failed, then T2 iterations,
 * with no early stop, and stores check-state checkpoints every `ckpt_every`
 * iterations for the backward (12 bytes per check: both minima of |q| over
 * the row, their positions, the q signs and their parity with the syndrome
 * bit).  ckpt_every = 1 (a checkpoint per iteration: 12 m (T1 + T2) bytes per
 * shot at most) lets the backward read every state back instead of
 * recomputing segments, and is its fastest setting; larger values trade
 * backward time for checkpoint memory.  Rows of H of at most 21 edges, channel second-pass prior, min-sum,
 * no soft DC (BPDC_ERR_UNSUPPORTED otherwise).
 *   d_w      [2][E] float scales in CSR edge order of H (pass 1, pass 2)
 *   d_post   [2][B][n] float posteriors at the end of each pass (pass-2 rows
 *            of shots without DC are copies of pass 1)
 *   d_cut    [B][ceil(n/64)] uint64 cut set (output, held fixed in backward)
 *   d_ckpt   checkpoint buffer of bpdc_wms_ckpt_size() bytes. */
bpdc_status bpdc_wms_ckpt_size(bpdc_plan plan, int32_t code, int64_t B, int32_t ckpt_every,
                               size_t* bytes);
bpdc_status bpdc_wms_forward(bpdc_plan plan, int32_t code, const float* d_w, const uint64_t* d_syn,
                             int64_t B, int64_t shot_offset, int32_t ckpt_every, float* d_post,
                             uint64_t* d_cut, uint8_t* d_flags, void* d_ckpt, size_t ckpt_bytes,
                             void* stream);
/* Adjoint of bpdc_wms_forward: given dLoss/dpost [2][B][n], accumulate
 * dLoss/dw into d_grad_w [2][E] (the caller zeroes it).  The cut is constant
 * (piecewise differentiation through min and sign; saturated messages have
 * zero derivative). */
bpdc_status bpdc_wms_backward(bpdc_plan plan, int32_t code, const float* d_w,
                              const uint64_t* d_syn, int64_t B, int32_t ckpt_every,
                              const float* d_grad_post, const uint64_t* d_cut,
                              const uint8_t* d_flags, const void* d_ckpt, size_t ckpt_bytes,
                              float* d_grad_w, void* stream);

/* Compile, or find in the on-disk kernel cache, the code-specialised lane
 * kernel for (H, D) -- every tile the plan autotuner may time -- without
 * touching a GPU (host-only; hipRTC).  The cache
 * directory is $BPDC_CACHE_DIR, else kcache/ beside libbpdc.so.  posterior =
 * 1 for plans with BPDC_PRIOR_POSTERIOR; uniform_prior = 1 for codes whose
 * priors are all equal (the kernel then takes the prior as one value); rule
 * is the plan's BPDC_RULE_* (product-sum: one lane per shot, at most 96
 * edges); soft = 1 for plans with soft DC (soft_period > 0; min-sum only).
 * BPDC_ERR_UNSUPPORTED if the code is too large for the lane kernel. */
bpdc_status bpdc_lane_precompile(const bpdc_csr* H, const bpdc_csr* D, int32_t posterior,
                                 int32_t uniform_prior, int32_t rule, int32_t soft);

/* The library's float32 phi(x) = ln((e^x + 1) / (e^x - 1)) = -ln tanh(x / 2)
 * (the product-sum rule's function, x >= 0 or +inf) on n floats: d_out[i] =
 * phi(d_x[i]), device arrays, enqueued on `stream`.  For accuracy tests. */
bpdc_status bpdc_eval_phi(const float* d_x, int64_t n, float* d_out, void* stream);

const char* bpdc_status_string(bpdc_status status);
const char* bpdc_last_error(void);
/* Library build identifier (the kernel variants compiled in). */
const char* bpdc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BPDC_H */
