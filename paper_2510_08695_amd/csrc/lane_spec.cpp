// Generator of the code-specialised part of the lane kernel: for one Tanner
// graph H and degeneracy matrix D it writes the sizes, lookup tables and the
// straight-line sweep (see lane_kernel.hip) with every index a literal.
//
// Lane groups.  A shot is decoded by a group of 1, 2 or 4 adjacent lanes.
// With more than one lane this needs a group of automorphisms of H acting
// freely on columns and checks (lane_spec.h): columns and checks fall into
// orbits, lane 0 holds one column of every column orbit ("rows") and one check
// of every check orbit ("slots"), and lane k executes the same instructions on
// the images under group element k.  An edge from lane 0's column to a check
// held by lane j (its relative element) is, on lane k, an edge to a check held
// by lane k xor j, so every lane fetches the check-to-variable message from,
// and returns the variable-to-check message to, lane k xor j: one DPP quad
// permutation per value.  Each lane holds 1/|group| of the state.
//
// The sweep visits the rows in an order chosen greedily to keep few checks
// "open" (some but not all of their edges visited), because every open check
// holds five accumulator registers.  The order only affects register
// pressure: a check's minima, argmin and sign parity do not depend on the
// order of its edges (ties of |q| give equal magnitudes).  Each lane adds the
// incoming messages of its column in ascending order of its own check
// indices; where that differs from the instruction order, the addition picks
// its operand by the lane's index in the group.
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

// Check permutation induced by the column permutation sv (rows matched as
// sets), or false if sv is not an automorphism of H.
bool induced_checks(const HostGraph& g, const std::map<std::vector<int>, int>& row_of, const std::vector<int>& sv,
                    std::vector<int>* sc) {
  sc->assign(g.m, -1);
  for (int c = 0; c < g.m; ++c) {
    std::vector<int> img;
    img.reserve(g.rows[c].size());
    for (int v : g.rows[c]) img.push_back(sv[v]);
    std::sort(img.begin(), img.end());
    auto it = row_of.find(img);
    if (it == row_of.end()) return false;
    (*sc)[c] = it->second;
  }
  return true;
}

bool fixed_point_free(const std::vector<int>& p) {
  for (size_t i = 0; i < p.size(); ++i)
    if (p[i] == (int)i) return false;
  return true;
}

std::vector<int> compose(const std::vector<int>& a, const std::vector<int>& b) {  // a after b
  std::vector<int> r(b.size());
  for (size_t i = 0; i < b.size(); ++i) r[i] = a[b[i]];
  return r;
}

}  // namespace

void find_group(const HostGraph& g, int max_lanes, LaneGroup* out) {
  const int n = g.n, m = g.m;
  out->lanes = 1;
  out->v.assign(1, std::vector<int>(n));
  out->c.assign(1, std::vector<int>(m));
  std::iota(out->v[0].begin(), out->v[0].end(), 0);
  std::iota(out->c[0].begin(), out->c[0].end(), 0);
  out->off = {0};
  out->block.clear();
  if (max_lanes < 2 || n % 2 || m % 2) return;
  std::map<std::vector<int>, int> row_of;
  for (int c = 0; c < m; ++c) {
    if (g.rows[c].empty()) return;
    row_of[g.rows[c]] = c;
  }
  if ((int)row_of.size() != m) return;  // repeated rows: a check is not determined by its support
  // candidate involutions: within blocks of B consecutive columns, shift by B/2
  std::vector<int> blocks;
  std::vector<std::vector<int>> inv_v, inv_c;
  for (int B = n; B >= 2; --B) {
    if (n % B || B % 2) continue;
    std::vector<int> sv(n), sc;
    for (int v = 0; v < n; ++v) sv[v] = (v / B) * B + ((v % B) + B / 2) % B;
    if (!induced_checks(g, row_of, sv, &sc) || !fixed_point_free(sc)) continue;
    blocks.push_back(B);
    inv_v.push_back(sv);
    inv_c.push_back(sc);
  }
  if (blocks.empty()) return;
  if (max_lanes >= 4) {
    // two generators whose half-block bits are independent (the smaller block
    // divides half the larger), so that lane k's columns are lane 0's shifted
    // by a constant
    for (size_t i = 0; i < blocks.size(); ++i)
      for (size_t j = i + 1; j < blocks.size(); ++j) {
        if ((blocks[i] / 2) % blocks[j]) continue;
        const auto pv = compose(inv_v[i], inv_v[j]), pc = compose(inv_c[i], inv_c[j]);
        if (pv != compose(inv_v[j], inv_v[i]) || pc != compose(inv_c[j], inv_c[i])) continue;
        if (!fixed_point_free(pv) || !fixed_point_free(pc)) continue;
        out->lanes = 4;
        out->v = {out->v[0], inv_v[i], inv_v[j], pv};
        out->c = {out->c[0], inv_c[i], inv_c[j], pc};
        out->off = {0, blocks[i] / 2, blocks[j] / 2, blocks[i] / 2 + blocks[j] / 2};
        out->block = {blocks[i], blocks[j]};
        return;
      }
  }
  out->lanes = 2;
  out->v = {out->v[0], inv_v[0]};
  out->c = {out->c[0], inv_c[0]};
  out->off = {0, blocks[0] / 2};
  out->block = {blocks[0]};
}

bool lane_eligible(const HostGraph& g, bool posterior, int max_lanes, int rule, bool soft, std::string* why) {
  auto fail = [&](const char* msg) {
    if (why) *why = msg;
    return false;
  };
  if (rule && soft) return fail("soft DC with product-sum runs on the plain kernel only");
  if (rule) {
    // product-sum: one lane per shot and one register per edge
    max_lanes = 1;
    size_t e = 0;
    for (auto& r : g.rows) e += r.size();
    if (e > 96) return fail("product-sum: more than 96 edges per lane");
  }
  if (g.n > 1024) return fail("more than 1024 columns");
  if (g.m > 1024) return fail("more than 1024 checks");
  if (max_deg(g.rows) > 15) return fail("check degree above 15");
  if (max_deg(g.cols) > 16) return fail("column degree above 16");
  if (max_deg(g.drows) > 32) return fail("degeneracy-matrix row degree above 32");
  LaneGroup grp;
  find_group(g, max_lanes, &grp);
  const int G = grp.lanes;
  if (g.n / G > 128) return fail("more than 128 columns per lane");
  if (g.m / G > 80) return fail("more than 80 checks per lane");
  const size_t lstr = 64 / G + 1;
  const size_t lds = (size_t)g.n * lstr * 4 * ((posterior || soft) ? 2 : 1) + g.drows.size() * max_deg(g.drows) * 2 +
                     g.drows.size() + (size_t)G * ((g.n / G + 31) / 32) * 4 + (size_t)g.n * 2 +
                     (size_t)G * (g.n / G) * 4 + 32 * (size_t)G * ((g.m / G + 31) / 32) * 4;
  if (lds > 64 * 1024) return fail("per-wave LDS above 64 KiB");
  return true;
}

LaneSpec lane_spec(const HostGraph& g, bool posterior, bool uniform_prior, int max_lanes, int rule, bool soft) {
  const int n = g.n, m = g.m, md = (int)g.drows.size();
  if (rule) max_lanes = 1;  // product-sum: one lane per shot
  LaneGroup grp;
  find_group(g, max_lanes, &grp);
  const int G = grp.lanes;
  // rows: lane 0's columns (lower half of every generator's block), ascending
  std::vector<int> row_col;
  for (int v = 0; v < n; ++v) {
    bool low = true;
    for (int B : grp.block) low = low && (v % B) < B / 2;
    if (low) row_col.push_back(v);
  }
  const int nrows = (int)row_col.size();
  // slots: check orbits.  Lane 0 holds the check of each orbit with the most
  // edges to lane 0's own columns, so that as many edges as possible stay
  // within a lane (no exchange).
  std::vector<char> is_row(n, 0);
  for (int v : row_col) is_row[v] = 1;
  std::vector<int> slot_of(m, -1), rel_of(m, 0), slot_base;
  for (int c0 = 0; c0 < m; ++c0) {
    if (slot_of[c0] >= 0) continue;
    int c = c0, best = -1;
    for (int k = 0; k < G; ++k) {
      const int ck = grp.c[k][c0];
      int own = 0;
      for (int v : g.rows[ck]) own += is_row[v];
      if (own > best) best = own, c = ck;
    }
    const int s = (int)slot_base.size();
    slot_base.push_back(c);
    for (int k = 0; k < G; ++k) {
      slot_of[grp.c[k][c]] = s;
      rel_of[grp.c[k][c]] = k;
    }
  }
  const int nslots = (int)slot_base.size();
  // events of row i: lane 0's column's edges in ascending check order
  struct Ev {
    int slot, rel, chk;
  };
  std::vector<std::vector<Ev>> ev(nrows);
  std::vector<std::vector<int>> items(nrows);
  for (int i = 0; i < nrows; ++i)
    for (int c : g.cols[row_col[i]]) {
      ev[i].push_back({slot_of[c], rel_of[c], c});
      items[i].push_back(slot_of[c]);
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
  const int spw = std::max(1, (nslots + 31) / 32);
  size_t dnnz = 0;
  for (auto& r : g.drows) dnnz += r.size();
  bool uniform_drows = !g.drows.empty();
  for (auto& r : g.drows) uniform_drows = uniform_drows && (int)r.size() == max_deg(g.drows);

  std::ostringstream o;
  o << "#define NB_M " << m << "\n#define NB_N " << n << "\n#define NB_MD " << md << "\n#define NB_SW64 "
    << (m + 63) / 64 << "\n#define NB_SPW " << spw << "\n#define NB_NW64 " << (n + 63) / 64 << "\n#define NB_SLOTS "
    << nslots << "\n#define NB_ROWS " << nrows << "\n#define NB_RC32 " << (nrows + 31) / 32 << "\n#define NB_NWC "
    << nwc << "\n#define NB_DNNZ " << std::max<size_t>(dnnz, 1) << "\n#define NB_DMAXROW "
    << std::max(1, max_deg(g.drows)) << "\n#define NB_DUNIFORM " << (uniform_drows ? 1 : 0)
    << "\n#define NB_POSTERIOR " << (posterior ? 1 : 0) << "\n#define NB_G " << G << "\n#define NB_PS "
    << (rule ? 1 : 0) << "\n#define NB_SOFT " << (soft ? 1 : 0);
  for (int k = 1; k < 4; ++k) o << "\n#define NB_LOFF" << k << " " << (k < G ? grp.off[k] : 0);
  o << "\n#define NB_UNIFORM_PRIOR " << (uniform_prior ? 1 : 0) << "\n";
  // column -> (row << 2 | lane in group), for the cooperative DC code
  o << "__device__ __constant__ const short nb_col_row[" << n << "] = {";
  {
    std::vector<int> cr(n, -1);
    for (int k = 0; k < G; ++k)
      for (int i = 0; i < nrows; ++i) cr[grp.v[k][row_col[i]]] = (i << 2) | k;
    for (int v = 0; v < n; ++v) o << cr[v] << (v + 1 < n ? "," : "");
  }
  o << "};\n";
  o << "__device__ __constant__ const short nb_row_col[" << G << "][" << nrows << "] = {";
  for (int k = 0; k < G; ++k) {
    o << "{";
    for (int i = 0; i < nrows; ++i) o << grp.v[k][row_col[i]] << (i + 1 < nrows ? "," : "");
    o << "}" << (k + 1 < G ? "," : "");
  }
  o << "};\n";
  // Syndrome words of every lane of a group in slot order, from the shot's
  // packed syndrome s32[] (32-bit words): out[k * NB_SPW + w] bit j = syndrome
  // bit of the check that lane k holds in slot 32 w + j.
  o << "#define NB_PREP(s32, out) do { \\\n";
  for (int k = 0; k < G; ++k)
    for (int w = 0; w < spw; ++w) {
      o << "out[" << k * spw + w << "] = 0u";
      for (int j = 0; j < 32 && 32 * w + j < nslots; ++j) {
        const int c = grp.c[k][slot_base[32 * w + j]];
        o << " | (((s32[" << (c >> 5) << "] >> " << (c & 31) << ") & 1u) << " << j << ")";
      }
      o << "; \\\n";
    }
  o << "} while (0)\n";

  if (rule) {
    // Product-sum (one lane per shot): one register R[k] per edge, k running
    // over the checks (slots) and, within a check, its columns in ascending
    // order.  R[k] holds the edge's r until its column is swept, then
    // phi(|q|); at the check's last edge the new r of every edge is formed
    // from them (leave-one-out sums left to right in column order, phi,
    // saturation, sign) and written back.
    std::vector<int> rbase(nslots + 1, 0);
    for (int sl = 0; sl < nslots; ++sl) rbase[sl + 1] = rbase[sl] + (int)g.rows[slot_base[sl]].size();
    o << "#define NB_NR " << std::max(1, rbase[nslots]) << "\n";
    o << "#define NB_SWEEP() do { \\\n";
    for (int sl = 0; sl < nslots; ++sl)
      if (sdeg[sl]) o << "u32 sb_" << sl << ", ep_" << sl << "; \\\n";
    for (int i : order) {
      const auto& e = ev[i];
      const int dv = (int)e.size();
      o << "{ float L = NB_LAM(" << i << ", " << row_col[i] << "); \\\n";
      std::vector<int> kk(dv), bb(dv);
      for (int j = 0; j < dv; ++j) {
        const auto& cols = g.rows[slot_base[e[j].slot]];
        bb[j] = (int)(std::lower_bound(cols.begin(), cols.end(), row_col[i]) - cols.begin());
        kk[j] = rbase[e[j].slot] + bb[j];
        o << "const float r" << j << " = R[" << kk[j] << "]; \\\n";
      }
      for (int j = 0; j < dv; ++j) o << "L = L + r" << j << "; \\\n";  // ascending check order
      o << "NB_CUT(L, " << i << "); NB_STORE(" << row_col[i] << ", L); const u32 ev = __float_as_uint(L) - 1u; \\\n";
      for (int j = 0; j < dv; ++j) {
        const int sl = e[j].slot, d = (int)g.rows[slot_base[sl]].size();
        // q = sat(L - r), +inf from a cut column (L = +inf): unlike min-sum, phi sees
        // |q| itself, so a posterior beyond lsat is held there and a cut column
        // contributes phi(+inf) = 0.
        o << "{ const float q = bpdc_dev::ps_q(L, r" << j << ", LS); " << (pos[i][j] == 0 ? "NB_EP0(" : "NB_EP(") << sl << ", ev); "
          << (pos[i][j] == 0 ? "NB_PSACC0(" : "NB_PSACC(") << sl << ", " << kk[j] << ", " << bb[j] << ", q); } \\\n";
        if (pos[i][j] == sdeg[sl] - 1) {
          // finalise check slot sl: d edges in registers rbase[sl] ..
          const int k0 = rbase[sl];
          o << "{ const u32 par_ = ((u32)__builtin_popcount(sb_" << sl << ") + (S[" << (sl >> 5) << "] >> " << (sl & 31)
            << ")) & 1u; ";
          for (int b = 0; b < d; ++b) o << "const float t" << b << "_ = R[" << k0 + b << "]; ";
          for (int b = 0; b < d; ++b) {
            std::string sum;
            for (int x = 0; x < d; ++x) {
              if (x == b) continue;
              sum = sum.empty() ? "t" + std::to_string(x) + "_" : "(" + sum + ") + t" + std::to_string(x) + "_";
            }
            if (sum.empty()) sum = "0.0f";
            o << "R[" << k0 + b << "] = NB_PSR(" << sum << ", par_ ^ ((sb_" << sl << " >> " << b << ") & 1u)); ";
          }
          o << "U |= ep_" << sl << "; } \\\n";
        }
      }
      o << "} \\\n";
    }
    for (int sl = 0; sl < nslots; ++sl)
      if (!sdeg[sl]) o << "U |= __builtin_amdgcn_ubfe(S[" << (sl >> 5) << "], " << (sl & 31) << ", 1) << 31; \\\n";
    o << "} while (0)\n";
    o << "#define NB_INIT1(W_, A1_, A2_, S_) do { } while (0)\n";
    LaneSpec out;
    out.src = o.str();
    out.lanes = G;
    out.spw = spw;
    return out;
  }
  o << "#define NB_SWEEP() do { \\\n";
  for (int s = 0; s < nslots; ++s)
    if (sdeg[s]) o << "float m1_" << s << ", m2_" << s << "; u32 am_" << s << ", sb_" << s << ", ep_" << s << "; \\\n";
  for (int i : order) {
    const auto& e = ev[i];
    const int dv = (int)e.size();
    o << "{ float L = NB_LAM(" << i << ", " << row_col[i] << "); \\\n";
    // rr: r of the edge at the lane holding its check.  A value of another
    // lane of the group is fetched (one DPP permutation) right where it is
    // consumed, so that the permutation can be folded into the consuming
    // instruction.
    for (int j = 0; j < dv; ++j) {
      const int s = e[j].slot, d = sdeg[s], b = d - 1 - pos[i][j];
      o << "const float rr" << j << " = NB_DEC(" << s << ", " << cw[s] << ", " << (off[s] + d + b) << ", "
        << (off[s] + b) << "); const float r" << j << " = NB_XF" << e[j].rel << "(rr" << j << "); \\\n";
    }
    auto xk = [&](int rel, const std::string& v, const char* kind) {
      if (!rel) return v;
      return std::string("NB_X") + kind + std::to_string(rel) + "(" + v + ")";
    };
    // summation: lane k adds in ascending order of its own checks
    std::vector<std::vector<int>> perm(G, std::vector<int>(dv));
    for (int k = 0; k < G; ++k) {
      std::vector<int> img(dv);
      for (int j = 0; j < dv; ++j) img[j] = grp.c[k][e[j].chk];
      std::iota(perm[k].begin(), perm[k].end(), 0);
      std::sort(perm[k].begin(), perm[k].end(), [&](int a, int b) { return img[a] < img[b]; });
    }
    for (int p = 0; p < dv; ++p) {
      std::vector<std::pair<int, int>> src;  // (edge, mask of lanes taking it)
      for (int k = 0; k < G; ++k) {
        auto it = std::find_if(src.begin(), src.end(),
                               [&](const std::pair<int, int>& x) { return x.first == perm[k][p]; });
        if (it == src.end()) src.push_back({perm[k][p], 1 << k});
        else it->second |= 1 << k;
      }
      auto rj = [&](int j) { return "r" + std::to_string(j); };
      std::string x = rj(src.back().first);
      for (int q = (int)src.size() - 2; q >= 0; --q)
        x = "NB_SEL(" + std::to_string(src[q].second) + ", " + rj(src[q].first) + ", " + x + ")";
      o << "L = L + " << x << "; \\\n";
    }
    o << "NB_CUT(L, " << i << "); NB_STORE(" << row_col[i] << ", L); const u32 ev = __float_as_uint(L) - 1u; \\\n";
    int kinds = 0;
    for (int j = 0; j < dv; ++j) kinds |= 1 << e[j].rel;
    // q = L - r at the lane holding the check, with L of the column's lane;
    // then the stop-test parities, then the check states
    (void)kinds;
    for (int j = 0; j < dv; ++j)
      o << (pos[i][j] == 0 ? "NB_EP0(" : "NB_EP(") << e[j].slot << ", " << xk(e[j].rel, "ev", "U") << "); \\\n";
    for (int j = 0; j < dv; ++j) {
      const int s = e[j].slot, d = sdeg[s], p = pos[i][j], b = d - 1 - p;
      const char* acc = p == 0 ? "NB_ACC0(" : "NB_ACC(";
      o << "{ const float q = NB_Q(" << xk(e[j].rel, "L", "F") << ", rr" << j << "); " << acc << s << ", q, " << b
        << "); } \\\n";
      if (p == d - 1) o << "NB_FIN(" << s << ", " << cw[s] << ", " << off[s] << ", " << d << "); \\\n";
    }
    o << "} \\\n";
  }
  for (int s = 0; s < nslots; ++s)
    if (!sdeg[s]) o << "U |= __builtin_amdgcn_ubfe(S[" << (s >> 5) << "], " << (s & 31) << ", 1) << 31; \\\n";
  o << "} while (0)\n";
  // Check state after the first iteration of a first pass with equal priors
  // lambda > 0 (every q = lambda): alpha*min1 = alpha*lambda, the same second
  // minimum (or alpha*lsat for a check of degree 1), and every r sign equal to
  // the check's syndrome bit.  A check of degree >= 2 gets no argmin bit (its
  // two minima are equal, so every edge reads alpha*min1 and A2 need not be
  // written); a check of degree 1 marks its only edge, which reads alpha*lsat.
  o << "#define NB_INIT1(W_, A1_, A2_, S_) do { \\\n";
  {
    std::vector<uint32_t> amc(nwc, 0u);
    for (int s = 0; s < nslots; ++s)
      if (sdeg[s] == 1) amc[cw[s]] |= 1u << (off[s] + 1);
    for (int w = 0; w < nwc; ++w) o << "W_[" << w << "] = " << amc[w] << "u; \\\n";
  }
  for (int s = 0; s < nslots; ++s) {
    if (!sdeg[s]) continue;
    const uint32_t mask = ((1u << sdeg[s]) - 1u) << off[s];
    o << "A1_[" << s << "] = A1I; ";
    if (sdeg[s] == 1) o << "A2_[" << s << "] = A2I1; ";
    o << "W_[" << cw[s] << "] |= (u32)__builtin_amdgcn_sbfe((int)S_[" << (s >> 5) << "], " << (s & 31) << ", 1) & "
      << mask << "u; \\\n";
  }
  o << "} while (0)\n";
  LaneSpec out;
  out.src = o.str();
  out.lanes = G;
  out.spw = spw;
  return out;
}

}  // namespace bpdc
