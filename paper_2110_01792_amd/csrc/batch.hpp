// Batched level step (placeholder).
#pragma once
#include "qk_device.hpp"
namespace qk {
struct BatchCache {
  int dummy = 0;
};
inline void batch_cache_clear(BatchCache&) {}
}  // namespace qk
