// Arguments and launchers of the final fit with outlier rejection: rounds of
// refit (the fused seeding and forward fit, then the backward fit with the
// two-filter smoother) and reject-the-worst, on each hit's unbiased chi2
// (against the estimate from its track's other hits).
#pragma once
#include "kf_kernels.hpp"

namespace kf {

// track status: at least one hit was rejected as an outlier
constexpr uint32_t TRK_OUTLIER = 128u;

// per-track round state (FinalRoundArgs::open)
constexpr uint8_t kFinalOpen = 1, kFinalRejected = 2;

template <typename T>
struct FinalRoundArgs {
  int64_t n, ld;                 // tracks; leading dimension of the outputs
  const int32_t* hit_offsets;    // [n + 1]
  const int16_t* hit_layer;      // [n_hits]
  const uint8_t* hit_valid;      // [n_hits] the caller's valid flags
  const T* hit_pos;              // [3][n_hits]
  const T* hit_cov;              // [6][n_hits]
  int64_t n_hits;
  int32_t max_len;
  int32_t round, max_reject, min_keep;
  double chi2_cut;
  uint8_t* used;                 // [n_hits] valid, not rejected, track still open
  uint8_t* open;                 // [n] kFinalOpen | kFinalRejected, or null: every track of the batch is open
  // After the first round a round runs on a sub-batch of the open tracks
  // (hit_offsets ... used then describe the sub-batch): map[i] is the
  // caller's track of sub-batch track i, orig_offsets the caller's hit
  // offsets, and the round's decisions go to the caller-indexed used_orig
  // and open_orig (and outlier, hit_chi2).  Without a sub-batch map is null
  // and used_orig / open_orig are used / open.
  const int32_t* map;            // [n] or null
  const int32_t* orig_offsets;   // the caller's [n_tracks + 1]
  uint8_t* used_orig;
  uint8_t* open_orig;
  uint8_t* outlier;              // [n_hits] 1 rejected
  T* hit_chi2;                   // [n_hits] the caller's copy of the unbiased chi2, or null
  T* chi2_work;                  // [n_hits] this round's unbiased chi2 of the used hits
  // this round's forward fit (leading dimension n): seeds, filtered state
  // after every entry (checkpoints, seg = 1: slot m after entry k0 + m)
  const T* seed_state;           // [6][n]
  const int8_t* seed_charge;     // [n]
  const T* ckpt;                 // [28][(max_len - 1) * n]
  // this round's backward pass: its prediction at every entry, turned
  // outward (entry r of track t at [i][r * n + t]; NaN where not reached)
  const T* pred_state;           // [6][max_len * n]
  const T* pred_cov;             // [21][max_len * n]
  const T* b_state;              // [6][n]
  const T* b_cov;                // [21][n]
  const int8_t* b_charge;
  const T* b_chi2;
  const int32_t* b_ndf;
  const uint32_t* b_status;
  // final outputs (leading dimension ld)
  T* state_out;
  T* cov_out;
  int8_t* charge_out;
  T* chi2_out;
  int32_t* ndf_out;
  uint32_t* status_out;
};

// Entries of the n tracks: outlier = 0, used = hit_valid, hit_chi2 = NaN;
// every track open.
template <typename T>
hipError_t launch_final_init(const FinalRoundArgs<T>& a, hipStream_t s);
// The unbiased chi2 of every used hit of the open tracks, one thread per
// entry and track (after the round's fit and backward pass).
template <typename T>
hipError_t launch_final_chi2(const FinalRoundArgs<T>& a, const GeomArgs& g, hipStream_t s);
// One round's decisions (after launch_final_chi2).
template <typename T>
hipError_t launch_final_round(const FinalRoundArgs<T>& a, hipStream_t s);

// The open tracks of the caller's batch gathered into a sub-batch for the
// next round: the caller's n tracks (hit_offsets, hit_layer, used, hit_pos,
// hit_cov, open) in, the sub-batch's map, offsets, layers, used flags,
// positions and covariances out, in the caller's track order, and counts[0]
// = its tracks, counts[1] = its entries (device).  flag, len, pos, epos: [n]
// int32 scratch; scan_temp / scan_bytes: hipCUB scan storage (null: only
// report the storage needed in scan_bytes).
template <typename T>
struct GatherArgs {
  int64_t n;
  const int32_t* hit_offsets;
  const int16_t* hit_layer;
  const uint8_t* used;
  const T* hit_pos;
  const T* hit_cov;
  int64_t n_hits;
  const uint8_t* open;
  int32_t* flag;
  int32_t* len;
  int32_t* pos;
  int32_t* epos;
  int32_t* map;
  int32_t* sub_offsets;   // [n + 1]
  int16_t* sub_layer;     // [n_hits]
  uint8_t* sub_used;      // [n_hits]
  T* sub_pos;             // [3][n_hits] (leading dimension n_hits)
  T* sub_cov;             // [6][n_hits]
  int32_t* counts;        // [2]
  void* scan_temp;
  size_t scan_bytes;
};
template <typename T>
hipError_t launch_final_gather(GatherArgs<T>& a, hipStream_t s);
// The backward pass of the smoother alone: its prediction at every entry
// stored in b.smooth_state / b.smooth_cov, without the combination.  block:
// threads per block (64, 128, 192 or 256; anything else: 256).
template <typename T>
hipError_t launch_backward_predictions(const BwdArgs<T>& b, const GeomArgs& g, hipStream_t s, int block = 256);

}  // namespace kf
