// Plain CPU reference for BP+DC decoding (degeneracy cutting, arXiv 2510.08695).
//
// TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
// checked against.  Only the test suite, the smoke check and the CPU-baseline
// leg of the benchmark load it; the GPU library never includes, links or calls
// it, and it shares no code, header or table with that library.
//
// It follows the paper step by step and favours obviousness over speed:
// messages are stored per edge, every loop walks the CSR / CSC order of the
// matrices, and both precisions come from one template (double: the reference;
// float: the comparator that takes every floating-point decision in the GPU
// kernels' precision).
//
// What it computes (paper sections):
//  * BP_decode(H, s, prior, T) with the flooding schedule: per iteration all
//    variable-to-check messages, then all check-to-variable messages, then the
//    posterior log-likelihood ratios, the hard decision e_v = [p_v >= 1/2]
//    (= [L_v <= 0]) and the stop test H e = s (Sec. II.C, Eq. (3)).
//  * The check rule is scaled min-sum (the paper points to prior work for it
//    and states no scale; the scale is a parameter) or product-sum.
//  * Algorithm 1: BP; if the syndrome is not reproduced, every row of the
//    degeneracy matrix D nominates the variable of lowest posterior error
//    probability (= highest LLR) in its support, ties broken at random; the
//    union of nominees is cut and BP is run again (Sec. III.A).
//  * The cut is taken either as the literal deletion of columns (Algorithm 1)
//    or as prior probability 0 on the cut variables (Algorithm 2); both are
//    implemented so that their equivalence can be tested.
//
// Readings where the paper is silent (each is a parameter or a documented
// convention):
//  * messages and reported posteriors saturate at +-lsat; a check's "minimum
//    over the other inputs" starts from lsat, so a minimum over no inputs is
//    lsat (this makes the two cut forms agree exactly);
//  * the variable-to-check message is q = sat(L_v - r_{c->v});
//  * signs are tested with x < 0;
//  * the stop test runs after every iteration, never before the first;
//  * DC reads the saturated pass-1 posteriors of the last pass-1 iteration;
//    a row's tie set is {i : L_i >= L_max - eps * max(1, |L_max|)}, and the
//    random choice among ties is the SplitMix64 hash (Steele, Lea, Flood,
//    OOPSLA 2014) of (seed, global shot index, row index);
//  * the second pass starts from the channel prior (BB-type codes, Sec.
//    III.B) or from the pass-1 posteriors (surface-type codes), with fresh
//    messages.
//  * intermittent soft DC (the extension Sec. V proposes, off by default):
//    every soft_period iterations of the first pass, while H e != s, every
//    row of D nominates as in DC (on the saturated posteriors of that
//    iteration; the j-th application hashes row h as j * rows(D) + h) and
//    the union of nominees has its prior error odds p / (1 - p) divided by
//    e^soft_shift, i.e. its prior LLR raised by soft_shift; messages carry
//    on.  The final DC and the second pass are unchanged (a channel second
//    pass starts from the unshifted prior).
//
// Parity: pinned by the tests (tree-graph exact marginals and max-marginals,
// single-check closed forms, brute-force maximum-likelihood bounds on tiny
// codes, DC invariants, Algorithm 1 == Algorithm 2).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

extern "C" {

// Mirrored field by field by oracle/oracle.py (ctypes).
struct OracleParams {
  int32_t rule;               // 0 = scaled min-sum, 1 = product-sum
  int32_t max_iter1;          // T before DC
  int32_t max_iter2;          // T after DC
  int32_t second_pass_prior;  // 0 = channel prior, 1 = pass-1 posteriors
  int32_t stop_on_converge;   // 1 = stop when H e = s; 0 = always run T iterations
  int32_t tie_break;          // 0 = hash of (seed, shot, row); 1 = lowest column index
  int32_t dc_form;            // 0 = zero prior on cut variables (Alg. 2); 1 = delete columns (Alg. 1)
  int32_t skip_dc;            // 1 = plain BP only (no DC, no second pass)
  double alpha;               // min-sum scale (used when no per-edge weights are given)
  double llr_sat;             // saturation magnitude (may be +inf)
  double tie_eps;             // relative tie tolerance for DC
  uint64_t seed;              // tie-break seed
  int32_t soft_period;        // intermittent soft DC every soft_period pass-1 iterations (0 = off)
  double soft_shift;          // prior-LLR increase of each soft nominee
};

}  // extern "C"

namespace {

struct Graph {
  int m = 0, n = 0;
  std::vector<int> row_ptr, col_idx;        // CSR; an edge is its CSR position
  std::vector<std::vector<int>> var_edges;  // per column: its edges in ascending row order
};

Graph make_graph(int m, int n, const int* rp, const int* ci) {
  Graph g;
  g.m = m;
  g.n = n;
  g.row_ptr.assign(rp, rp + m + 1);
  g.col_idx.assign(ci, ci + rp[m]);
  g.var_edges.assign(n, {});
  for (int c = 0; c < m; ++c)
    for (int e = rp[c]; e < rp[c + 1]; ++e) g.var_edges[ci[e]].push_back(e);
  return g;
}

// SplitMix64 output function (Steele, Lea, Flood 2014): state advance by the
// golden-ratio increment, then the two xor-shift-multiply finalising rounds.
uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Counter-based tie-break draw for (seed, global shot index, degeneracy-matrix row).
uint64_t tie_hash(uint64_t seed, uint64_t shot, uint64_t row) {
  return splitmix64(splitmix64(shot * 0x1000000ull + row) ^ seed);
}

// floor(h * k / 2^64): a uniform index in [0, k) from a 64-bit draw.
uint64_t scale_draw(uint64_t h, uint64_t k) {
  return (uint64_t)(((unsigned __int128)h * (unsigned __int128)k) >> 64);
}

template <class Real>
Real sat(Real x, Real lsat) {
  return std::min(std::max(x, -lsat), lsat);
}

// phi(x) = ln((e^x + 1) / (e^x - 1)) = -ln tanh(x / 2) for x >= 0, written
// log1p(2 / expm1(x)): phi(0) = +inf, phi(+inf) = 0, and phi is its own
// inverse.  The product-sum message 2 atanh(prod tanh(|q| / 2)) equals
// phi(sum phi(|q|)) (the log of the product is minus the sum of the phi), and
// in this form neither side rounds to 1 near saturation.
template <class Real>
Real phi(Real x) {
  return std::log1p(Real(2) / std::expm1(x));
}

template <class Real>
struct PassOut {
  std::vector<unsigned char> ehat;  // hard decision
  std::vector<Real> L;              // posterior LLR (saturated; +inf on frozen columns)
  bool converged = false;           // H ehat = s at exit
  int iters = 0;                    // iterations executed
  double margin = INFINITY;         // smallest decision margin seen (instrumentation)
};

// Degeneracy cutting: one nominee per row of D (Alg. 1, the loop over rows).
// Row h is hashed as row_base + h (0 for the DC between the passes).
template <class Real>
std::vector<unsigned char> degeneracy_cut(const Graph& D, int n, const std::vector<Real>& L1,
                                          const OracleParams& prm, uint64_t shot, double* margin,
                                          uint64_t row_base = 0) {
  std::vector<unsigned char> cut(n, 0);
  const Real eps = (Real)prm.tie_eps;
  for (int h = 0; h < D.m; ++h) {
    const int b = D.row_ptr[h], f = D.row_ptr[h + 1];
    if (b == f) continue;
    Real lmax = L1[D.col_idx[b]];
    for (int e = b; e < f; ++e) lmax = std::max(lmax, L1[D.col_idx[e]]);
    const Real scale = std::max((Real)1, (Real)std::fabs(lmax));
    const Real thr = lmax - eps * scale;
    std::vector<int> ties;
    for (int e = b; e < f; ++e) {
      const Real x = L1[D.col_idx[e]];
      if (x >= thr) ties.push_back(D.col_idx[e]);
      if (margin && x != lmax) *margin = std::min(*margin, (double)std::fabs(x - thr) / (double)scale);
    }
    int pick = ties[0];
    if (prm.tie_break == 0) pick = ties[scale_draw(tie_hash(prm.seed, shot, row_base + (uint64_t)h), ties.size())];
    cut[pick] = 1;
  }
  return cut;
}

// Intermittent soft DC inside a pass (off when null).
struct SoftDC {
  const Graph* D;
  const OracleParams* prm;
  uint64_t shot;
};

// One run of BP_decode on graph g.  `prior0` is the prior LLR per column,
// `frozen` marks columns held at prior probability 0, `w` holds one scale per
// edge (CSR order) or is null (then every edge uses alpha); `soft` turns on
// intermittent soft DC.
template <class Real>
PassOut<Real> bp_decode(const Graph& g, const unsigned char* s, const std::vector<Real>& prior0,
                        const std::vector<unsigned char>& frozen, const Real* w, Real alpha,
                        int rule, int T, bool stop_on_converge, Real lsat, const SoftDC* soft = nullptr) {
  const int E = g.row_ptr[g.m];
  std::vector<Real> q(E), r(E), L(g.n);
  std::vector<Real> prior = prior0;  // shifted by soft DC
  PassOut<Real> out;
  out.ehat.assign(g.n, 0);
  out.L.assign(g.n, 0);

  // variable-to-check messages of the first iteration: the prior LLR.  A
  // frozen column (prior probability 0) sends +inf: no minimum or sum over a
  // check moves because of it, exactly as if its column were deleted
  for (int v = 0; v < g.n; ++v)
    for (int e : g.var_edges[v]) q[e] = frozen[v] ? (Real)INFINITY : sat(prior[v], lsat);

  auto syndrome_ok = [&]() {
    for (int c = 0; c < g.m; ++c) {
      int par = s[c];
      for (int e = g.row_ptr[c]; e < g.row_ptr[c + 1]; ++e) par ^= out.ehat[g.col_idx[e]];
      if (par) return false;
    }
    return true;
  };

  for (int t = 1; t <= T; ++t) {
    // check-to-variable messages
    for (int c = 0; c < g.m; ++c) {
      const int b = g.row_ptr[c], f = g.row_ptr[c + 1];
      int neg = s[c];
      for (int e = b; e < f; ++e) {
        if (q[e] < 0) neg ^= 1;
        out.margin = std::min(out.margin, (double)std::fabs(q[e]));
      }
      if (rule == 0) {
        Real m1 = lsat, m2 = lsat;  // smallest and second-smallest |q| over the check
        int amin = -1;              // edge holding m1 (first one in CSR order)
        for (int e = b; e < f; ++e) {
          const Real a = std::fabs(q[e]);
          if (a < m1) {
            m2 = m1;
            m1 = a;
            amin = e;
          } else if (a < m2) {
            m2 = a;
          }
        }
        for (int e = b; e < f; ++e) {
          const Real mag = (e == amin) ? m2 : m1;  // min of |q| over the other edges
          const Real val = (w ? w[e] : alpha) * mag;
          const bool negative = neg ^ (q[e] < 0);  // syndrome parity times the other signs
          r[e] = negative ? -val : val;
        }
      } else {
        // product-sum in the log domain: the sum of phi(|q|) over the other edges,
        // left to right in row order, then phi of that sum (an empty sum, or one of
        // zeros from frozen columns, gives +inf: the magnitude is held at lsat)
        for (int e = b; e < f; ++e) {
          Real sum = 0;
          for (int o = b; o < f; ++o)
            if (o != e) sum = sum + phi(std::fabs(q[o]));
          Real mag = phi(sum);
          if (!(mag < lsat)) mag = lsat;
          const Real val = (w ? w[e] : alpha) * mag;
          const bool negative = neg ^ (q[e] < 0);
          r[e] = negative ? -val : val;
        }
      }
    }
    // posteriors, next variable-to-check messages, hard decision
    for (int v = 0; v < g.n; ++v) {
      if (frozen[v]) {
        for (int e : g.var_edges[v]) q[e] = (Real)INFINITY;
        L[v] = INFINITY;
        out.ehat[v] = 0;
        continue;
      }
      Real Lv = prior[v];
      for (int e : g.var_edges[v]) Lv = Lv + r[e];
      L[v] = Lv;
      for (int e : g.var_edges[v]) q[e] = sat(Lv - r[e], lsat);
      out.ehat[v] = (Lv <= 0) ? 1 : 0;
      out.margin = std::min(out.margin, (double)std::fabs(Lv));
    }
    out.iters = t;
    if (stop_on_converge && syndrome_ok()) break;
    if (soft && t % soft->prm->soft_period == 0 && t < T && !syndrome_ok()) {
      std::vector<Real> Ls(g.n);
      for (int v = 0; v < g.n; ++v) Ls[v] = frozen[v] ? (Real)INFINITY : sat(L[v], lsat);
      const uint64_t j = (uint64_t)(t / soft->prm->soft_period);
      const std::vector<unsigned char> nom =
          degeneracy_cut<Real>(*soft->D, g.n, Ls, *soft->prm, soft->shot, &out.margin, j * (uint64_t)soft->D->m);
      for (int v = 0; v < g.n; ++v)
        if (nom[v]) prior[v] = prior[v] + (Real)soft->prm->soft_shift;
    }
  }
  out.converged = syndrome_ok();
  for (int v = 0; v < g.n; ++v) out.L[v] = frozen[v] ? (Real)INFINITY : sat(L[v], lsat);
  return out;
}

template <class Real>
struct ShotOut {
  std::vector<unsigned char> ehat, cut;
  std::vector<Real> L, L1;
  unsigned char flags = 0;
  int iters[2] = {0, 0};
  double margin = INFINITY;
};

template <class Real>
ShotOut<Real> decode_shot(const Graph& H, const Graph& D, const std::vector<Real>& lam,
                          const double* weights, const OracleParams& prm, const unsigned char* s,
                          uint64_t shot) {
  const int n = H.n;
  const int E = H.row_ptr[H.m];
  const Real lsat = (Real)prm.llr_sat, alpha = (Real)prm.alpha;
  std::vector<Real> w1, w2;
  if (weights) {
    w1.assign(weights, weights + E);
    w2.assign(weights + E, weights + 2 * E);
  }
  ShotOut<Real> out;
  std::vector<unsigned char> none(n, 0);
  const SoftDC soft{&D, &prm, shot};
  PassOut<Real> p1 = bp_decode<Real>(H, s, lam, none, weights ? w1.data() : nullptr, alpha, prm.rule,
                                     prm.max_iter1, prm.stop_on_converge != 0, lsat,
                                     prm.soft_period > 0 ? &soft : nullptr);
  out.iters[0] = p1.iters;
  out.L1 = p1.L;
  out.margin = p1.margin;
  out.cut.assign(n, 0);
  if (p1.converged || prm.skip_dc) {
    out.ehat = p1.ehat;
    out.L = p1.L;
    out.flags = p1.converged ? 1 : 0;
    return out;
  }
  out.cut = degeneracy_cut<Real>(D, n, p1.L, prm, shot, &out.margin);

  // prior of the second pass
  std::vector<Real> lam2(n);
  for (int v = 0; v < n; ++v) lam2[v] = (prm.second_pass_prior == 1) ? p1.L[v] : lam[v];

  PassOut<Real> p2;
  if (prm.dc_form == 0) {
    // Algorithm 2: cut variables keep prior probability 0 (LLR +inf) throughout
    p2 = bp_decode<Real>(H, s, lam2, out.cut, weights ? w2.data() : nullptr, alpha, prm.rule,
                         prm.max_iter2, prm.stop_on_converge != 0, lsat);
  } else {
    // Algorithm 1: delete the cut columns, decode the reduced problem, pad with zeros
    std::vector<int> keep, newcol(n, -1);
    for (int v = 0; v < n; ++v)
      if (!out.cut[v]) {
        newcol[v] = (int)keep.size();
        keep.push_back(v);
      }
    std::vector<int> rp(H.m + 1, 0), ci;
    std::vector<Real> wr;
    for (int c = 0; c < H.m; ++c) {
      for (int e = H.row_ptr[c]; e < H.row_ptr[c + 1]; ++e) {
        const int v = H.col_idx[e];
        if (newcol[v] < 0) continue;
        ci.push_back(newcol[v]);
        if (weights) wr.push_back(w2[e]);
      }
      rp[c + 1] = (int)ci.size();
    }
    Graph Hr = make_graph(H.m, (int)keep.size(), rp.data(), ci.data());
    std::vector<Real> lamr(keep.size());
    for (size_t j = 0; j < keep.size(); ++j) lamr[j] = lam2[keep[j]];
    std::vector<unsigned char> none_r(keep.size(), 0);
    PassOut<Real> pr = bp_decode<Real>(Hr, s, lamr, none_r, weights ? wr.data() : nullptr, alpha,
                                       prm.rule, prm.max_iter2, prm.stop_on_converge != 0, lsat);
    p2.ehat.assign(n, 0);
    p2.L.assign(n, (Real)INFINITY);
    for (size_t j = 0; j < keep.size(); ++j) {
      p2.ehat[keep[j]] = pr.ehat[j];
      p2.L[keep[j]] = pr.L[j];
    }
    p2.converged = pr.converged;
    p2.iters = pr.iters;
    p2.margin = pr.margin;
  }
  out.iters[1] = p2.iters;
  out.margin = std::min(out.margin, p2.margin);
  out.ehat = p2.ehat;
  out.L = p2.L;
  out.flags = (unsigned char)((p2.converged ? 1 : 0) | 2);
  return out;
}

template <class Real>
std::vector<Real> prior_llr(int n, const double* priors) {
  // LLR of the prior, log((1 - p) / p), evaluated in double and rounded once.
  std::vector<Real> lam(n);
  for (int v = 0; v < n; ++v) lam[v] = (Real)std::log((1.0 - priors[v]) / priors[v]);
  return lam;
}

template <class Real>
int decode_all(int m, int n, const int* hrp, const int* hci, int md, const int* drp, const int* dci,
               const double* priors, const double* weights, const OracleParams* prm, int64_t nshots,
               int64_t shot_offset, const unsigned char* syn, unsigned char* ehat, double* post,
               double* post1, unsigned char* cut, unsigned char* flags, int32_t* iters,
               double* margin, int nthreads) {
  if (!prm || m < 0 || n < 0 || md < 0 || nshots < 0) return 1;
  for (int v = 0; v < n; ++v)
    if (!(priors[v] > 0.0 && priors[v] < 1.0)) return 2;
  const Graph H = make_graph(m, n, hrp, hci);
  const Graph D = make_graph(md, n, drp, dci);
  const std::vector<Real> lam = prior_llr<Real>(n, priors);
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads > 0 ? nthreads : 1)
  for (int64_t b = 0; b < nshots; ++b) {
    ShotOut<Real> o = decode_shot<Real>(H, D, lam, weights, *prm, syn + b * (int64_t)m,
                                        (uint64_t)(shot_offset + b));
    for (int v = 0; v < n; ++v) {
      ehat[b * (int64_t)n + v] = o.ehat[v];
      if (post) post[b * (int64_t)n + v] = (double)o.L[v];
      if (post1) post1[b * (int64_t)n + v] = (double)o.L1[v];
      if (cut) cut[b * (int64_t)n + v] = o.cut[v];
    }
    flags[b] = o.flags;
    if (iters) {
      iters[2 * b] = o.iters[0];
      iters[2 * b + 1] = o.iters[1];
    }
    if (margin) margin[b] = o.margin;
  }
  return 0;
}

template <class Real>
int bp_once(int m, int n, const int* hrp, const int* hci, const double* prior_llr_in,
            const unsigned char* frozen, const double* weights, double alpha, int rule, int T,
            int stop_on_converge, double lsat, const unsigned char* syn, unsigned char* ehat,
            double* post, int32_t* iters) {
  const Graph H = make_graph(m, n, hrp, hci);
  std::vector<Real> lam(n);
  for (int v = 0; v < n; ++v) lam[v] = (Real)prior_llr_in[v];
  std::vector<unsigned char> fz(n, 0);
  if (frozen) fz.assign(frozen, frozen + n);
  std::vector<Real> w;
  if (weights) w.assign(weights, weights + hrp[m]);
  PassOut<Real> o = bp_decode<Real>(H, syn, lam, fz, weights ? w.data() : nullptr, (Real)alpha, rule,
                                    T, stop_on_converge != 0, (Real)lsat);
  for (int v = 0; v < n; ++v) {
    ehat[v] = o.ehat[v];
    post[v] = (double)o.L[v];
  }
  *iters = o.iters;
  return o.converged ? 1 : 0;
}

}  // namespace

extern "C" {

// Full BP+DC over `nshots` shots.  Syndromes and outputs are unpacked bytes
// (one per check / column), row-major per shot; optional outputs may be null.
// Returns 0 on success, nonzero on invalid arguments.
int oracle_decode_f64(int m, int n, const int* hrp, const int* hci, int md, const int* drp,
                      const int* dci, const double* priors, const double* weights,
                      const OracleParams* prm, int64_t nshots, int64_t shot_offset,
                      const unsigned char* syn, unsigned char* ehat, double* post, double* post1,
                      unsigned char* cut, unsigned char* flags, int32_t* iters, double* margin,
                      int nthreads) {
  return decode_all<double>(m, n, hrp, hci, md, drp, dci, priors, weights, prm, nshots, shot_offset,
                            syn, ehat, post, post1, cut, flags, iters, margin, nthreads);
}

int oracle_decode_f32(int m, int n, const int* hrp, const int* hci, int md, const int* drp,
                      const int* dci, const double* priors, const double* weights,
                      const OracleParams* prm, int64_t nshots, int64_t shot_offset,
                      const unsigned char* syn, unsigned char* ehat, double* post, double* post1,
                      unsigned char* cut, unsigned char* flags, int32_t* iters, double* margin,
                      int nthreads) {
  return decode_all<float>(m, n, hrp, hci, md, drp, dci, priors, weights, prm, nshots, shot_offset,
                           syn, ehat, post, post1, cut, flags, iters, margin, nthreads);
}

// A single BP_decode run with explicit prior LLRs and frozen columns (tree and
// closed-form tests).  Returns 1 if H ehat = s at exit, else 0.
int oracle_bp_f64(int m, int n, const int* hrp, const int* hci, const double* prior_llr_in,
                  const unsigned char* frozen, const double* weights, double alpha, int rule, int T,
                  int stop_on_converge, double lsat, const unsigned char* syn, unsigned char* ehat,
                  double* post, int32_t* iters) {
  return bp_once<double>(m, n, hrp, hci, prior_llr_in, frozen, weights, alpha, rule, T,
                         stop_on_converge, lsat, syn, ehat, post, iters);
}

int oracle_bp_f32(int m, int n, const int* hrp, const int* hci, const double* prior_llr_in,
                  const unsigned char* frozen, const double* weights, double alpha, int rule, int T,
                  int stop_on_converge, double lsat, const unsigned char* syn, unsigned char* ehat,
                  double* post, int32_t* iters) {
  return bp_once<float>(m, n, hrp, hci, prior_llr_in, frozen, weights, alpha, rule, T,
                        stop_on_converge, lsat, syn, ehat, post, iters);
}

// The tie-break draw, exported so that tests can pin it to published values.
uint64_t oracle_splitmix64(uint64_t x) { return splitmix64(x); }
uint64_t oracle_tie_hash(uint64_t seed, uint64_t shot, uint64_t row) { return tie_hash(seed, shot, row); }

}  // extern "C"
