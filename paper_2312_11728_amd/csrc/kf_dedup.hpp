// Duplicate removal among found tracks: launcher and workspace size.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace kf {

struct DedupArgs {
  int64_t n;               // tracks
  const int32_t* hits;     // hit id of track t at layer l: hits[t * hit_stride + l] (-1 miss, -2 none)
  int64_t hit_stride;
  int32_t n_layers;        // 1..64
  const float* score;      // score[t * score_stride]; -inf: no candidate
  int64_t score_stride;
  float frac;              // duplicates share >= frac * min(hit counts) hits (and >= 1)
  uint8_t* keep;           // [n]
  int32_t* dup_of;         // [n] or null
};

// Bytes of device workspace a call over n tracks of n_layers needs.
size_t dedup_workspace_bytes(int64_t n, int32_t n_layers);

hipError_t launch_dedup(const DedupArgs& a, void* work, size_t work_bytes, hipStream_t s);

}  // namespace kf
