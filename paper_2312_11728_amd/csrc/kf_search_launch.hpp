// Workspace and launch functions of the candidate search (host side).
#pragma once

#include <hip/hip_runtime.h>

#include "kf_search.hpp"

namespace kf {

// The binned copy of the hit pool.
struct PoolBins {
  PoolHit* hits;     // [n] in bin order
  int32_t* bin_off;  // [n_bins + 1]
};

// Scratch of one search call (carved out of a context-owned allocation).
struct SearchWork {
  int32_t* count;      // [n_bins]
  int32_t* bin_of;     // [n_pool]
  int32_t* rank;       // [n_pool]
  int32_t* block_sum;  // [n_bins / 2048 + 1]
  int32_t* total;      // [1]
  PoolBins pool;
};

hipError_t launch_bin_pool(const BinTable& t, const float* pos, const float* cov, const int32_t* id,
                           const int32_t* module, int64_t n, int64_t n_bins, const SearchWork& w, hipStream_t s);
// layers: the plan's host array (a.plan_len entries), copied to d_layers on
// the stream before the search kernel reads it there
hipError_t launch_search(SearchArgs a, const SearchLayer* layers, SearchLayer* d_layers, hipStream_t s);

}  // namespace kf
