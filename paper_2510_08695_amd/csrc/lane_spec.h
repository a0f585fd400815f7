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

// An involutive automorphism of H used to split a shot over two lanes: columns
// shifted by half a block of size `block`, checks by m/2.
struct Pairing {
  int block = 0;
  std::vector<int> sigma_v;  // column permutation
  std::vector<int> va;       // columns of lane A (one per orbit), ascending
};

bool find_pairing(const HostGraph& g, Pairing* out);
bool lane_eligible(const HostGraph& g, bool posterior, std::string* why);
std::string lane_spec(const HostGraph& g, bool posterior, bool uniform_prior);

}  // namespace bpdc
