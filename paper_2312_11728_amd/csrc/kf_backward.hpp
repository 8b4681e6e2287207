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
  uint8_t* open;                 // [n] kFinalOpen | kFinalRejected
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
// The backward pass of the smoother alone: its prediction at every entry
// stored in b.smooth_state / b.smooth_cov, without the combination.
template <typename T>
hipError_t launch_backward_predictions(const BwdArgs<T>& b, const GeomArgs& g, hipStream_t s);

}  // namespace kf
