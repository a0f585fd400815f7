// Generator of the code-specialised part of the lane kernel: for one Tanner
// graph H and degeneracy matrix D it writes the sizes and the straight-line
// sweep (see lane_kernel.hip) with every index a literal.
//
// Two layouts:
//  * single: one lane decodes one shot and holds the state of every check;
//  * paired: two adjacent lanes decode one shot.  This needs an automorphism
//    sigma of H that is an involution without fixed points, shifting the
//    checks cyclically by m/2 and the columns by half a block (the
//    translations of bivariate bicycle and toric codes are of this kind).
//    Lane A of a pair handles the columns of a set V_A with one column of
//    every orbit {v, sigma v} and the checks 0..m/2-1; lane B executes the
//    same instructions on sigma of them.  An edge whose check belongs to the
//    partner is exchanged with one DPP lane swap per value.  Each lane then
//    holds half the state, which keeps the kernel inside the VGPR file.
//
// The sweep visits the columns in an order chosen greedily to keep few
// checks "open" (some but not all of their edges visited) at any time,
// because every open check holds five accumulator registers.  The order only
// affects register pressure: a check's minima, argmin and sign parity do not
// depend on the order of its edges (ties of |q| give equal magnitudes), and
// each column still adds its incoming messages in ascending check order.
#include "lane_spec.h"

#include <algorithm>
#include <cstdint>
#include <map>
#include <numeric>
#include <sstream>

namespace bpdc {

namespace {

// Greedy order over `items` (each a list of slot ids, the checks it touches;
// deg[s] = number of events of slot s): prefer items that close slots, then
// items that continue open slots, avoid opening new slots.
std::vector<int> greedy_order(const std::vector<std::vector<int>>& items, const std::vector<int>& deg) {
  const int n = (int)items.size();
  std::vector<int> cnt(deg.size(), 0), order;
  std::vector<char> done(n, 0);
  order.reserve(n);
  for (int step = 0; step < n; ++step) {
    int best = -1, bs = 0;
    for (int v = 0; v < n; ++v) {
      if (done[v]) continue;
      int s = 0;
      for (int c : items[v]) {
        if (cnt[c] == deg[c] - 1) s += 4;
        else if (cnt[c] > 0) s += 2;
        else s -= 3;
      }
      if (best < 0 || s > bs) {
        best = v;
        bs = s;
      }
    }
    done[best] = 1;
    order.push_back(best);
    for (int c : items[best]) ++cnt[c];
  }
  return order;
}

int max_deg(const std::vector<std::vector<int>>& a) {
  int d = 0;
  for (auto& r : a) d = std::max(d, (int)r.size());
  return d;
}

}  // namespace

bool find_pairing(const HostGraph& g, Pairing* out) {
  const int n = g.n, m = g.m;
  if (n % 2 || m % 2) return false;
  std::map<std::vector<int>, int> row_of;
  for (int c = 0; c < m; ++c) {
    if (g.rows[c].empty()) return false;
    row_of[g.rows[c]] = c;
  }
  if ((int)row_of.size() != m) return false;  // repeated rows: ambiguous
  for (int B = n; B >= 2; --B) {
    if (n % B || B % 2) continue;
    std::vector<int> sv(n);
    for (int v = 0; v < n; ++v) sv[v] = (v / B) * B + ((v % B) + B / 2) % B;
    bool ok = true;
    for (int c = 0; c < m && ok; ++c) {
      std::vector<int> img;
      for (int v : g.rows[c]) img.push_back(sv[v]);
      std::sort(img.begin(), img.end());
      auto it = row_of.find(img);
      ok = it != row_of.end() && it->second == (c + m / 2) % m;
    }
    if (!ok) continue;
    out->block = B;
    out->sigma_v = sv;
    out->va.clear();
    for (int v = 0; v < n; ++v)
      if ((v % B) < B / 2) out->va.push_back(v);
    return true;
  }
  return false;
}

bool lane_eligible(const HostGraph& g, bool posterior, std::string* why) {
  auto fail = [&](const char* msg) {
    if (why) *why = msg;
    return false;
  };
  if (g.n > 250) return fail("more than 250 columns");
  if (g.m > 160) return fail("more than 160 checks");
  if (max_deg(g.rows) > 15) return fail("check degree above 15");
  if (max_deg(g.cols) > 16) return fail("column degree above 16");
  if (max_deg(g.drows) > 32) return fail("degeneracy-matrix row degree above 32");
  size_t dnnz = 0;
  for (auto& r : g.drows) dnnz += r.size();
  const size_t lds = (size_t)g.n * 65 * 4 * (posterior ? 2 : 1) + (g.drows.size() + 1) * 4 + dnnz * 2 +
                     ((g.n + 31) / 32) * 8 + (size_t)g.n * 6;
  if (lds > 64 * 1024) return fail("per-wave LDS above 64 KiB");
  return true;
}

std::string lane_spec(const HostGraph& g, bool posterior, bool uniform_prior) {
  const int n = g.n, m = g.m, md = (int)g.drows.size();
  Pairing pr;
  const bool paired = find_pairing(g, &pr);
  // ---- slots (checks held by one lane), rows (columns of one lane) ----
  const int nslots = paired ? m / 2 : m;
  const int nrows = paired ? n / 2 : n;
  std::vector<int> row_col(nrows);  // column handled by lane A (or the single lane) at row i
  if (paired) row_col = pr.va;
  else std::iota(row_col.begin(), row_col.end(), 0);
  // events of row i: (slot, remote, check of lane A's edge)
  struct Ev {
    int slot, remote, chk;
  };
  std::vector<std::vector<Ev>> ev(nrows);
  std::vector<std::vector<int>> items(nrows);
  for (int i = 0; i < nrows; ++i) {
    const int v = row_col[i];
    for (int c : g.cols[v]) {  // ascending checks
      const int slot = paired ? (c < m / 2 ? c : c - m / 2) : c;
      const int remote = paired && c >= m / 2;
      ev[i].push_back({slot, remote, c});
      items[i].push_back(slot);
    }
  }
  std::vector<int> sdeg(nslots, 0);
  for (auto& e : ev)
    for (auto& x : e) ++sdeg[x.slot];
  const std::vector<int> order = greedy_order(items, sdeg);
  // event position of each (row, edge) within its slot, in sweep order
  std::vector<std::vector<int>> pos(nrows);
  std::vector<int> seen(nslots, 0);
  for (int i : order) {
    pos[i].resize(ev[i].size());
    for (size_t j = 0; j < ev[i].size(); ++j) pos[i][j] = seen[ev[i][j].slot]++;
  }
  // packing of slot fields (2 * degree bits) into 32-bit words
  std::vector<int> cw(nslots), off(nslots);
  int word = 0, bit = 0;
  for (int s = 0; s < nslots; ++s) {
    const int bits = 2 * sdeg[s];
    if (bit + bits > 32) {
      ++word;
      bit = 0;
    }
    cw[s] = word;
    off[s] = bit;
    bit += bits;
  }
  const int nwc = word + 1;
  size_t dnnz = 0;
  for (auto& r : g.drows) dnnz += r.size();

  bool uniform_drows = !g.drows.empty();
  for (auto& r : g.drows) uniform_drows = uniform_drows && (int)r.size() == max_deg(g.drows);
  std::ostringstream o;
  o << "#define NB_M " << m << "\n#define NB_N " << n << "\n#define NB_MD " << md
    << "\n#define NB_SW32 " << (m + 31) / 32 << "\n#define NB_SW64 " << (m + 63) / 64
    << "\n#define NB_NW64 " << (n + 63) / 64 << "\n#define NB_NC32 " << (n + 31) / 32
    << "\n#define NB_SLOTS " << nslots << "\n#define NB_ROWS " << nrows << "\n#define NB_RC32 "
    << (nrows + 31) / 32 << "\n#define NB_NWC " << nwc << "\n#define NB_DNNZ " << std::max<size_t>(dnnz, 1)
    << "\n#define NB_DMAXROW " << std::max(1, max_deg(g.drows)) << "\n#define NB_DUNIFORM " << (uniform_drows ? 1 : 0)
    << "\n#define NB_POSTERIOR " << (posterior ? 1 : 0)
    << "\n#define NB_PAIRED " << (paired ? 1 : 0) << "\n#define NB_HALFOFF " << (paired ? pr.block / 2 : 0)
    << "\n#define NB_UNIFORM_PRIOR " << (uniform_prior ? 1 : 0)
    << "\n";
  // column -> (row, lane B?) map for the cooperative DC / output code, and the
  // column of lane B at each row
  o << "__device__ __constant__ const short nb_col_row[" << n << "] = {";
  {
    std::vector<int> cr(n, -1);
    for (int i = 0; i < nrows; ++i) {
      cr[row_col[i]] = i << 1;
      if (paired) cr[pr.sigma_v[row_col[i]]] = (i << 1) | 1;
    }
    for (int v = 0; v < n; ++v) o << cr[v] << (v + 1 < n ? "," : "");
  }
  o << "};\n";
  o << "__device__ __constant__ const short nb_row_col[2][" << nrows << "] = {{";
  for (int i = 0; i < nrows; ++i) o << row_col[i] << (i + 1 < nrows ? "," : "");
  o << "},{";
  for (int i = 0; i < nrows; ++i) o << (paired ? pr.sigma_v[row_col[i]] : row_col[i]) << (i + 1 < nrows ? "," : "");
  o << "}};\n";

  o << "#define NB_SWEEP() do { \\\n";
  for (int s = 0; s < nslots; ++s)
    if (sdeg[s]) o << "float m1_" << s << ", m2_" << s << "; u32 am_" << s << ", sb_" << s << ", ep_" << s << "; \\\n";
  for (int i : order) {
    const auto& e = ev[i];
    const int dv = (int)e.size();
    o << "{ float L = NB_LAM(" << i << ", " << row_col[i] << "); \\\n";
    for (int j = 0; j < dv; ++j) {
      const int s = e[j].slot, d = sdeg[s], b = d - 1 - pos[i][j];
      o << "const float r" << j << " = " << (e[j].remote ? "NB_SWAPF(" : "(") << "NB_DEC(" << s << ", " << cw[s]
        << ", " << (off[s] + d + b) << ", " << (off[s] + b) << ")); \\\n";
    }
    // summation order: lane A in ascending checks (instruction order); lane B
    // in ascending sigma(checks)
    std::vector<int> perm(dv);
    std::iota(perm.begin(), perm.end(), 0);
    if (paired) {
      std::vector<int> img(dv);
      for (int j = 0; j < dv; ++j) img[j] = (e[j].chk + m / 2) % m;
      std::sort(perm.begin(), perm.end(), [&](int a, int b) { return img[a] < img[b]; });
    }
    for (int p = 0; p < dv; ++p) {
      if (perm[p] == p) o << "L = L + r" << p << "; \\\n";
      else o << "L = L + NB_PICK(r" << p << ", r" << perm[p] << "); \\\n";
    }
    o << "NB_CUT(L, " << i << "); NB_STORE(" << row_col[i] << ", L); const u32 ev = __float_as_uint(L) - 1u; \\\n";
    bool any_remote = false;
    for (int j = 0; j < dv; ++j) any_remote |= e[j].remote != 0;
    if (any_remote) o << "const u32 evx = NB_SWAPU(ev); \\\n";
    for (int j = 0; j < dv; ++j) {
      const int s = e[j].slot, d = sdeg[s], p = pos[i][j], b = d - 1 - p;
      const char* acc = p == 0 ? "NB_ACC0(" : "NB_ACC(";
      if (e[j].remote)
        o << "{ const float q = NB_SWAPF(NB_Q(L, r" << j << ")); " << acc << s << ", q, evx, " << b << "); } \\\n";
      else
        o << "{ const float q = NB_Q(L, r" << j << "); " << acc << s << ", q, ev, " << b << "); } \\\n";
      if (p == d - 1) o << "NB_FIN(" << s << ", " << cw[s] << ", " << off[s] << ", " << d << "); \\\n";
    }
    o << "} \\\n";
  }
  for (int s = 0; s < nslots; ++s)
    if (!sdeg[s]) o << "U |= __builtin_amdgcn_ubfe(S[" << (s >> 5) << "], " << (s & 31) << ", 1) << 31; \\\n";
  o << "} while (0)\n";
  // Check state after the first iteration of a first pass with equal priors
  // lambda > 0 (every q = lambda): alpha*min1 = alpha*lambda, alpha*min2 the
  // same (or alpha*lsat for a check of degree 1), argmin the first edge, and
  // every r sign equal to the check's syndrome bit.
  // A check of degree >= 2 gets no argmin bit (its two minima are equal, so
  // every edge reads alpha*min1 and A2 need not be written); a check of
  // degree 1 marks its only edge, which reads alpha*lsat.
  o << "#define NB_INIT1() do { \\\n";
  {
    std::vector<uint32_t> amc(nwc, 0u);
    for (int s = 0; s < nslots; ++s)
      if (sdeg[s] == 1) amc[cw[s]] |= 1u << (off[s] + 1);
    for (int w = 0; w < nwc; ++w) o << "W[" << w << "] = " << amc[w] << "u; \\\n";
  }
  for (int s = 0; s < nslots; ++s) {
    if (!sdeg[s]) continue;
    const uint32_t mask = ((1u << sdeg[s]) - 1u) << off[s];
    o << "A1[" << s << "] = A1I; ";
    if (sdeg[s] == 1) o << "A2[" << s << "] = A2I1; ";
    o << "W[" << cw[s] << "] |= (u32)__builtin_amdgcn_sbfe((int)S[" << (s >> 5) << "], " << (s & 31) << ", 1) & "
      << mask << "u; \\\n";
  }
  o << "} while (0)\n";
  return o.str();
}

}  // namespace bpdc
