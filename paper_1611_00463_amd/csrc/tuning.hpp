// Tuning cache: handler schedule, fan-in, merge tile and radix tile per shape and
// device architecture, chosen by measurement (lbsort_autotune).
#pragma once
#include <stdint.h>

namespace lbs {

struct Tuned {
  uint32_t fanin;       // 0 = no entry
  uint32_t merge_tile;  // 0 = no entry
  uint32_t radix_tile;  // 0 = no entry
  uint32_t handler;     // 0 = no entry
  uint32_t presorted;   // 0 = no entry
};

// Entry for (architecture of the current device, key width, values or not,
// instance size, batched or not, P); zeros if none.
Tuned tuning_lookup(uint32_t key_bytes, bool values, uint64_t n, uint32_t B, uint32_t P);

}  // namespace lbs
