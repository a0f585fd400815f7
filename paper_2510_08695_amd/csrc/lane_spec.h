// Host-side description of a code used to generate the code-specialised lane
// kernel (lane_spec.cpp).
#pragma once

#include <string>
#include <vector>

namespace bpdc {

struct HostGraph {
  int n = 0, m = 0;
  std::vector<std::vector<int>> rows;   // H: columns of each row, ascending
  std::vector<std::vector<int>> cols;   // H: rows of each column, ascending
  std::vector<std::vector<int>> drows;  // D: columns of each row, ascending
};

// A group of automorphisms of H acting freely on columns and on checks, of
// order 1, 2 or 4: the trivial group, one involution, or two commuting
// involutions.  Each generator shifts the columns by half a block within
// blocks of `block` consecutive columns (the translations of bivariate
// bicycle and toric codes are of this kind).  Element k (k = 0 .. lanes-1) is
// the product of the generators selected by the bits of k, so elements
// compose by XOR of their indices.  Lane 0 of a shot's group holds the
// columns that lie in the lower half of their block for every generator;
// lane k holds their images under element k, which are lane 0's columns
// shifted by off[k].
struct LaneGroup {
  int lanes = 1;
  std::vector<std::vector<int>> v;  // v[k][column]
  std::vector<std::vector<int>> c;  // c[k][check]
  std::vector<int> off;             // off[k]: column offset of lane k
  std::vector<int> block;           // block size of each generator
};

// The layout the generator chose, with the kernel source.
struct LaneSpec {
  std::string src;
  int lanes = 1;  // lanes per shot
  int spw = 1;    // 32-bit syndrome words per lane (slot order)
};

void find_group(const HostGraph& g, int max_lanes, LaneGroup* out);
// rule: 0 scaled min-sum, 1 product-sum (one lane per shot, one register per edge);
// soft: intermittent soft DC in the first pass (min-sum only; a per-shot prior array in LDS)
bool lane_eligible(const HostGraph& g, bool posterior, int max_lanes, int rule, bool soft, std::string* why);
LaneSpec lane_spec(const HostGraph& g, bool posterior, bool uniform_prior, int max_lanes, int rule, bool soft);

}  // namespace bpdc
