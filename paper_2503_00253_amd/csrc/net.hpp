// Internal view of the warm-start network handle.
#pragma once
#include <cstdint>

namespace infoesrf {

struct Net {
  int H = 64;              // hidden channels
  int K = 9;               // kernel width (odd)
  int64_t count = 0;       // number of FP32 parameters
  float* params = nullptr; // device
};

int64_t net_param_count(int H, int K);

}  // namespace infoesrf
