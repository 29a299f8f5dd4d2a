// Tuning cache: merge fan-in and merge tile per shape, chosen by measurement.
#pragma once
#include <stdint.h>

namespace lbs {

struct Tuned {
  uint32_t fanin;       // 0 = no entry
  uint32_t merge_tile;  // 0 = no entry
};

// Entry for (key type, value type, instance size, instances, P); zeros if none.
Tuned tuning_lookup(int key_type, int val_type, uint64_t n, uint32_t B, uint32_t P);

}  // namespace lbs
