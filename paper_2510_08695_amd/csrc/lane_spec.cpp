// Generator of the code-specialised part of the lane kernel: for one Tanner
// graph H and degeneracy matrix D it writes the sizes and the straight-line
// sweep (see lane_kernel.hip) with every index a literal.
//
// The sweep visits the columns in an order chosen greedily to keep few
// checks "open" (some but not all of their edges visited) at any time,
// because every open check holds five accumulator registers.  The order only
// affects register pressure: a check's minima, argmin and sign parity do not
// depend on the order of its edges (ties of |q| give equal magnitudes), and
// each column still adds its incoming messages in ascending check order.
#include "lane_spec.h"

#include <algorithm>
#include <sstream>

namespace bpdc {

namespace {

std::vector<int> sweep_order(int n, int m, const std::vector<std::vector<int>>& rows,
                             const std::vector<std::vector<int>>& cols) {
  std::vector<int> cnt(m, 0), order;
  std::vector<char> done(n, 0);
  order.reserve(n);
  for (int step = 0; step < n; ++step) {
    int best = -1, bs = 0;
    for (int v = 0; v < n; ++v) {
      if (done[v]) continue;
      int s = 0;
      for (int c : cols[v]) {
        const int d = (int)rows[c].size();
        if (cnt[c] == d - 1) s += 4;       // closes c
        else if (cnt[c] > 0) s += 2;       // continues an open check
        else s -= 3;                       // opens a new check
      }
      if (best < 0 || s > bs) {
        best = v;
        bs = s;
      }
    }
    done[best] = 1;
    order.push_back(best);
    for (int c : cols[best]) ++cnt[c];
  }
  return order;
}

}  // namespace

bool lane_eligible(const HostGraph& g, bool posterior, std::string* why) {
  auto fail = [&](const char* msg) {
    if (why) *why = msg;
    return false;
  };
  if (g.n > 250) return fail("more than 250 columns");
  if (g.m > 160) return fail("more than 160 checks");
  int maxr = 0, maxc = 0, maxd = 0;
  for (auto& r : g.rows) maxr = std::max(maxr, (int)r.size());
  for (auto& c : g.cols) maxc = std::max(maxc, (int)c.size());
  for (auto& r : g.drows) maxd = std::max(maxd, (int)r.size());
  if (maxr > 15) return fail("check degree above 15");
  if (maxc > 16) return fail("column degree above 16");
  if (maxd > 32) return fail("degeneracy-matrix row degree above 32");
  size_t dnnz = 0;
  for (auto& r : g.drows) dnnz += r.size();
  const size_t lds = (size_t)g.n * 65 * 4 * (posterior ? 2 : 1) + (g.drows.size() + 1) * 4 + dnnz * 2 +
                     ((g.n + 31) / 32) * 4;
  if (lds > 64 * 1024) return fail("per-wave LDS above 64 KiB");
  return true;
}

std::string lane_spec(const HostGraph& g, bool posterior) {
  const int n = g.n, m = g.m, md = (int)g.drows.size();
  const std::vector<int> order = sweep_order(n, m, g.rows, g.cols);
  std::vector<int> pos(n);
  for (int i = 0; i < n; ++i) pos[order[i]] = i;

  // slot of each edge within its check (rank of the column in sweep order)
  std::vector<std::vector<int>> slot_of(m);  // slot_of[c][k] for k-th CSR column of c
  for (int c = 0; c < m; ++c) {
    const auto& r = g.rows[c];
    std::vector<int> idx(r.size());
    for (size_t k = 0; k < r.size(); ++k) idx[k] = (int)k;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return pos[r[a]] < pos[r[b]]; });
    slot_of[c].assign(r.size(), 0);
    for (size_t j = 0; j < idx.size(); ++j) slot_of[c][idx[j]] = (int)j;
  }
  // packing of check fields (2 * degree bits each) into 32-bit words
  std::vector<int> cw(m), off(m);
  int word = 0, bit = 0;
  for (int c = 0; c < m; ++c) {
    const int bits = 2 * (int)g.rows[c].size();
    if (bit + bits > 32) {
      ++word;
      bit = 0;
    }
    cw[c] = word;
    off[c] = bit;
    bit += bits;
  }
  const int nwc = word + 1;
  size_t dnnz = 0;
  int maxd = 1;
  for (auto& r : g.drows) {
    dnnz += r.size();
    maxd = std::max(maxd, (int)r.size());
  }

  std::ostringstream o;
  o << "#define NB_M " << m << "\n#define NB_N " << n << "\n#define NB_MD " << md
    << "\n#define NB_SW32 " << (m + 31) / 32 << "\n#define NB_SW64 " << (m + 63) / 64
    << "\n#define NB_NW64 " << (n + 63) / 64 << "\n#define NB_NC32 " << (n + 31) / 32
    << "\n#define NB_NWC " << nwc << "\n#define NB_DNNZ " << std::max<size_t>(dnnz, 1)
    << "\n#define NB_DMAXROW " << maxd << "\n#define NB_POSTERIOR " << (posterior ? 1 : 0) << "\n";
  o << "#define NB_SWEEP() do { \\\n";
  for (int c = 0; c < m; ++c)
    if (!g.rows[c].empty())
      o << "float m1_" << c << ", m2_" << c << "; u32 am_" << c << ", sb_" << c << ", ep_" << c
        << "; \\\n";
  // position of column v inside row c's CSR list
  auto kpos = [&](int c, int v) {
    const auto& r = g.rows[c];
    return (int)(std::lower_bound(r.begin(), r.end(), v) - r.begin());
  };
  for (int i = 0; i < n; ++i) {
    const int v = order[i];
    const auto& cs = g.cols[v];  // ascending checks
    o << "{ float L = NB_LAM(" << v << "); \\\n";
    for (size_t j = 0; j < cs.size(); ++j) {
      const int c = cs[j];
      const int d = (int)g.rows[c].size();
      const int s = slot_of[c][kpos(c, v)];
      const int b = d - 1 - s;
      o << "const float r" << j << " = NB_DEC(" << c << ", " << cw[c] << ", " << (off[c] + d + b)
        << ", " << (off[c] + b) << "); L = L + r" << j << "; \\\n";
    }
    o << "NB_CUT(L, " << v << "); NB_STORE(" << v << ", L); const u32 ev = __float_as_uint(L) - 1u; \\\n";
    for (size_t j = 0; j < cs.size(); ++j) {
      const int c = cs[j];
      const int d = (int)g.rows[c].size();
      const int s = slot_of[c][kpos(c, v)];
      const int b = d - 1 - s;
      o << "{ const float q = NB_Q(L, r" << j << "); " << (s == 0 ? "NB_ACC0(" : "NB_ACC(") << c
        << ", q, ev, " << b << "); } \\\n";
      if (s == d - 1) o << "NB_FIN(" << c << ", " << cw[c] << ", " << off[c] << ", " << d << "); \\\n";
    }
    o << "} \\\n";
  }
  for (int c = 0; c < m; ++c)
    if (g.rows[c].empty())
      o << "U |= __builtin_amdgcn_ubfe(S[" << (c >> 5) << "], " << (c & 31) << ", 1) << 31; \\\n";
  o << "} while (0)\n";
  return o.str();
}

}  // namespace bpdc
