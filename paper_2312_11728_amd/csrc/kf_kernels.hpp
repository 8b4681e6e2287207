// Kernel argument structures and launch helpers shared by the host API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kf_math.hpp"

namespace kf {

constexpr int kMaxLayers = 64;

// Detector description passed by value in the kernel arguments.
struct GeomArgs {
  int32_t n_layers;
  int8_t kind[kMaxLayers];
  double pos[kMaxLayers];
  double x0[kMaxLayers];
  double bz;
  double mass;
};

template <typename T>
struct SeedArgs {
  int64_t n, ld, n_hits;
  const int32_t* hit_offsets;
  const uint8_t* hit_valid;
  const T* hit_pos;
  double bz;
  int32_t mode;
  T* seed_state;
  T* seed_cov;
  int8_t* seed_charge;
  uint32_t* trk_status;
};

template <typename T>
struct PropArgs {
  int64_t n, ld;
  const T* state_in;
  const T* cov_in;
  const int8_t* charge;
  const int16_t* target;
  const int16_t* from;
  int32_t material;
  T* state_out;
  T* cov_out;
  T* path;
  uint32_t* trk_status;
};

template <typename T>
struct UpdArgs {
  int64_t n, ld;
  T* state;
  T* cov;
  int8_t* charge;
  const T* hit_pos;
  const T* hit_cov;
  T* chi2;
  uint32_t* trk_status;
};

constexpr int kTile = 64;   // tracks per tile of the packed hit layout (one wave)

// Hits in the packed, tile-transposed layout: tracks sorted by decreasing
// entry count fill tiles of kTile slots; entry k of the track in slot s is at
// index tile_base[s / kTile] + k * kTile + s % kTile of every component array,
// so the entry-k loads of one wave read kTile consecutive elements.
template <typename T>
struct PackedHits {
  const int32_t* order;      // [n] slot -> track
  const int64_t* tile_base;  // [n_tiles + 1]
  const int32_t* lv;         // layer | valid << 16
  const T* hit;              // [9][stride]: x, y, z, then the packed 3x3 covariance
  int64_t stride;
};

template <typename T>
struct FitArgs {
  int64_t n, ld, n_hits;
  int32_t max_len;           // entries beyond this are ignored (track flagged)
  const T* seed_state;
  const T* seed_cov;
  const int8_t* seed_charge;
  const int32_t* hit_offsets;
  const int16_t* hit_layer;
  const uint8_t* hit_valid;
  const T* hit_pos;
  const T* hit_cov;
  const T* align;  // [2][n_layers] or null
  T* state_out;
  T* cov_out;
  int8_t* charge_out;
  T* chi2;
  int32_t* ndf;
  T* ckpt;  // [28][ld * n_seg] or null
  int32_t seg;
  int32_t n_seg;
  uint32_t* trk_status;
  int32_t* tile_counter;  // persistent mode
  int64_t n_tiles;
  int32_t packed;         // layout: 0 CSR, 1 CSR in length-sorted order, 2 sorted and packed (pk),
                          // 3 CSR staged through LDS, 4 length-sorted CSR staged through LDS
  PackedHits<T> pk;
  // seeding inside the fit: 0 reads seed_state / seed_cov / seed_charge;
  // 1 + m seeds every track from its hits as the seeding kernel does in mode
  // m, and writes the seeds to the *_out arrays that are not null
  int32_t make_seeds;
  T* seed_state_out;        // [6][ld] or null
  T* seed_cov_out;          // [21][ld] or null
  int8_t* seed_charge_out;  // [n] or null
};

// Workspace of the packed layout (carved out of one device allocation).
struct PackWork {
  int32_t* hist;       // [kMaxLen + 2] per-length counts, then cursors
  int32_t* cursor;     // [kMaxLen + 2]
  int32_t* order;      // [max_tracks] slot -> track
  int32_t* slot_of;    // [max_tracks] track -> slot
  int64_t* tile_base;  // [max_tiles + 1]
  int32_t* lv;         // [cap]
  void* hit;           // [9][cap] of float or double
  int64_t cap;         // entries per component array
  int64_t max_tracks;
  int32_t max_len;
};
constexpr int kMaxLen = 64;

template <typename T>
hipError_t launch_pack(const FitArgs<T>& a, const PackWork& w, int layout, PackedHits<T>* out, hipStream_t s);

// Launch functions (defined in kf_kernels.hip).
template <typename T>
hipError_t launch_seeds(const SeedArgs<T>& a, hipStream_t s);
template <typename T>
hipError_t launch_propagate(const PropArgs<T>& a, const GeomArgs& g, hipStream_t s);
template <typename T>
hipError_t launch_update(const UpdArgs<T>& a, hipStream_t s);

struct FitLaunch {
  int block;        // threads per block (multiple of 64)
  int persistent;   // 0: one thread per track; 1: persistent blocks pulling tiles
  int blocks_per_cu;
  int waves;        // register budget: at least this many waves per SIMD (1 or 2)
  int layout;       // 0 CSR, 1 length-sorted CSR, 2 length-sorted packed, 3 LDS-staged CSR,
                    // 4 LDS-staged length-sorted CSR (1, 2, 4 need a workspace)
};
template <typename T>
hipError_t launch_fit(const FitArgs<T>& a, const GeomArgs& g, const FitLaunch& l, int n_cu, hipStream_t s);

// Reverse pass of the fit (gradient of sum_t w_t chi2_t).
template <typename T>
struct AdjArgs {
  FitArgs<T> f;                // the forward fit's inputs and checkpoints (outputs unused)
  const T* w;                  // [n] chi2 weights or null (= 1)
  const uint32_t* fwd_status;  // [n] status of the forward fit
  T* grad_seed;                // [6][ld]
  T* grad_hit;                 // [3][n_hits]
  T* grad_align;               // [2][n_layers] or null
  T* partial;                  // [adjoint_partial_blocks(n_hits)][2][kMaxLayers] when grad_align is set
  // the states before entries 1 .. max_len - 1 of every track, recomputed
  // segment by segment from the checkpoints by a pass before the reverse
  // sweep ([max_len - 1][kSegVals][n], entry j's state at
  // ((j - 1) * kSegVals + value) * n + track), or null: each state is then
  // recomputed from its segment's checkpoint when the reverse sweep needs it
  T* seg_buf;
};
constexpr int kSegVals = 29;   // state (6), covariance (21), charge, layer of the previous entry
// blocks of the alignment reduction (kAlignPerBlock entries each)
constexpr int kAlignPerBlock = 64 * 32;
inline int64_t adjoint_partial_blocks(int64_t n_hits) { return (n_hits + kAlignPerBlock - 1) / kAlignPerBlock; }
template <typename T>
hipError_t launch_adjoint(const AdjArgs<T>& a, const GeomArgs& g, hipStream_t s);

// Backward fit: f.seed_state / seed_cov / seed_charge hold the forward fit's
// result (the state on each track's last entry), f.state_out ... the result
// on its first valid entry.  f.ckpt and f.align are unused (null).
template <typename T>
struct BwdArgs {
  FitArgs<T> f;
  const uint32_t* fwd_status;  // [n] status of the forward fit, or null
  T cov_scale;                 // the forward covariance is multiplied by this first
  // smoothing (all null / 0 for the plain backward fit): the forward fit's
  // filtered state after every entry, as its checkpoints with seg = 1
  // ([28][ld * n_seg_f], slot m = after entry k0 + m), and the smoothed
  // state of entry r of track t at [6 or 21][r * ld + t] (ld * max_len)
  const T* fwd_ckpt;
  int32_t n_seg_f;
  T* smooth_state;
  T* smooth_cov;
};
template <typename T>
hipError_t launch_backward(const BwdArgs<T>& a, const GeomArgs& g, hipStream_t s);

}  // namespace kf
