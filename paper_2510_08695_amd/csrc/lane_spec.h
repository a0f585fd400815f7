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

bool lane_eligible(const HostGraph& g, bool posterior, std::string* why);
std::string lane_spec(const HostGraph& g, bool posterior);

}  // namespace bpdc
