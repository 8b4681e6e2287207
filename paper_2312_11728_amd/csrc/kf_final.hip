// Kernels of the final fit with outlier rejection: the per-round decision
// (the worst used hit by unbiased chi2 rejected, or the track closed with the
// round's backward-fit result) and the set-up of the per-entry masks, one
// track per thread.  The unbiased chi2 itself is computed entry-parallel
// beside the backward pass whose combination it reuses.
#include <cmath>

#include "kf_backward.hpp"

namespace kf {

namespace {

constexpr int kFinalBlock = 256;

template <typename T>
__global__ void __launch_bounds__(kFinalBlock) final_init_kernel(FinalRoundArgs<T> a) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const int64_t e0 = a.hit_offsets[t], e1 = a.hit_offsets[t + 1];
  for (int64_t e = e0; e < e1; ++e) {
    a.outlier[e] = 0;
    a.used[e] = a.hit_valid[e] ? 1 : 0;
    a.chi2_work[e] = T(NAN);
    if (a.hit_chi2) a.hit_chi2[e] = T(NAN);
  }
  a.open[t] = kFinalOpen;
}

template <typename T>
__global__ void __launch_bounds__(kFinalBlock) final_round_kernel(FinalRoundArgs<T> a) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const uint8_t op = a.open[t];
  if (!(op & kFinalOpen)) return;
  const uint32_t bst = a.b_status[t];
  const bool refitted = !(bst & TRK_BAD_INPUT);
  const int64_t e0 = a.hit_offsets[t], e1 = a.hit_offsets[t + 1];
  int n_e = int(e1 - e0);
  if (n_e > a.max_len) n_e = a.max_len;
  double worst = -INFINITY;
  int worst_r = -1, n_used = 0;
  for (int r = 0; r < n_e; ++r) {
    const int64_t e = e0 + r;
    if (!a.used[e]) continue;
    ++n_used;
    const T c2 = a.chi2_work[e];   // NaN unless refitted (launch_final_chi2)
    if (a.hit_chi2) a.hit_chi2[e] = c2;
    if (double(c2) > worst) {   // NaN never counts; the first entry among equals
      worst = double(c2);
      worst_r = r;
    }
  }
  const bool reject = a.round < a.max_reject && refitted && worst_r >= 0 && worst > a.chi2_cut &&
                      n_used - 1 >= a.min_keep;
  if (reject) {
    const int64_t e = e0 + worst_r;
    a.outlier[e] = 1;
    a.used[e] = 0;
    a.open[t] = kFinalOpen | kFinalRejected;
    return;
  }
  // closed: this round's backward-fit result
#pragma unroll
  for (int i = 0; i < 6; ++i) a.state_out[i * a.ld + t] = a.b_state[i * a.n + t];
#pragma unroll
  for (int i = 0; i < 21; ++i) a.cov_out[i * a.ld + t] = a.b_cov[i * a.n + t];
  a.charge_out[t] = a.b_charge[t];
  a.chi2_out[t] = a.b_chi2[t];
  a.ndf_out[t] = a.b_ndf[t];
  a.status_out[t] = bst | ((op & kFinalRejected) ? TRK_OUTLIER : 0u);
  a.open[t] = 0;
  for (int64_t e = e0; e < e1; ++e) a.used[e] = 0;   // later rounds skip the track
}

}  // namespace

template <typename T>
hipError_t launch_final_init(const FinalRoundArgs<T>& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(final_init_kernel<T>, dim3(unsigned((a.n + kFinalBlock - 1) / kFinalBlock)), dim3(kFinalBlock),
                     0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_final_round(const FinalRoundArgs<T>& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(final_round_kernel<T>, dim3(unsigned((a.n + kFinalBlock - 1) / kFinalBlock)), dim3(kFinalBlock),
                     0, s, a);
  return hipGetLastError();
}

template hipError_t launch_final_init<float>(const FinalRoundArgs<float>&, hipStream_t);
template hipError_t launch_final_init<double>(const FinalRoundArgs<double>&, hipStream_t);
template hipError_t launch_final_round<float>(const FinalRoundArgs<float>&, hipStream_t);
template hipError_t launch_final_round<double>(const FinalRoundArgs<double>&, hipStream_t);

}  // namespace kf
