// Kernels of the final fit with outlier rejection: the per-round decision
// (the worst used hit by unbiased chi2 rejected, or the track closed with the
// round's backward-fit result) and the set-up of the per-entry masks, one
// track per thread.  The unbiased chi2 itself is computed entry-parallel
// beside the backward pass whose combination it reuses.
#include <cmath>

#include <hipcub/hipcub.hpp>

#include "kf_backward.hpp"

namespace kf {

namespace {

constexpr int kFinalBlock = 256;

// Set-up, one thread per track (its open flag) and per entry: the tracks'
// entries are the one range [hit_offsets[0], hit_offsets[n]), written
// thread by thread.
template <typename T>
__global__ void __launch_bounds__(kFinalBlock) final_init_kernel(FinalRoundArgs<T> a) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < a.n) a.open[i] = kFinalOpen;
  const int64_t e = int64_t(a.hit_offsets[0]) + i;
  if (e >= a.hit_offsets[a.n] || e >= a.n_hits) return;
  a.outlier[e] = 0;
  a.used[e] = a.hit_valid[e] ? 1 : 0;
  a.chi2_work[e] = T(NAN);
  if (a.hit_chi2) a.hit_chi2[e] = T(NAN);
}

// The gather runs a grid of (tracks / kFinalBlock) x kFinalRows blocks:
// thread (t, y) copies entries y, y + kFinalRows, ... of track t, so that a
// track's entries are copied in parallel.
constexpr int kFinalRows = 8;

template <typename T>
__global__ void __launch_bounds__(kFinalBlock) final_round_kernel(FinalRoundArgs<T> a) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const int64_t to = a.map ? int64_t(a.map[t]) : t;   // the caller's track
  const uint8_t op = a.open_orig[to];
  if (!(op & kFinalOpen)) return;
  const uint32_t bst = a.b_status[t];
  const bool refitted = !(bst & TRK_BAD_INPUT);
  const int64_t e0 = a.hit_offsets[t], e1 = a.hit_offsets[t + 1];
  const int64_t e0o = a.map ? int64_t(a.orig_offsets[to]) : e0;   // the caller's entries
  int n_e = int(e1 - e0);
  if (n_e > a.max_len) n_e = a.max_len;
  double worst = -INFINITY;
  int worst_r = -1, n_used = 0;
#pragma unroll 4
  for (int r = 0; r < n_e; ++r) {
    if (!a.used[e0 + r]) continue;
    ++n_used;
    const T c2 = a.chi2_work[e0 + r];   // NaN unless refitted (launch_final_chi2)
    if (a.hit_chi2) a.hit_chi2[e0o + r] = c2;
    if (double(c2) > worst) {   // NaN never counts; the first entry among equals
      worst = double(c2);
      worst_r = r;
    }
  }
  const bool reject = a.round < a.max_reject && refitted && worst_r >= 0 && worst > a.chi2_cut &&
                      n_used - 1 >= a.min_keep;
  if (reject) {
    a.outlier[e0o + worst_r] = 1;
    a.used_orig[e0o + worst_r] = 0;
    a.open_orig[to] = kFinalOpen | kFinalRejected;
    return;
  }
  // closed: this round's backward-fit result
#pragma unroll
  for (int i = 0; i < 6; ++i) a.state_out[i * a.ld + to] = a.b_state[i * a.n + t];
#pragma unroll
  for (int i = 0; i < 21; ++i) a.cov_out[i * a.ld + to] = a.b_cov[i * a.n + t];
  a.charge_out[to] = a.b_charge[t];
  a.chi2_out[to] = a.b_chi2[t];
  a.ndf_out[to] = a.b_ndf[t];
  a.status_out[to] = bst | ((op & kFinalRejected) ? TRK_OUTLIER : 0u);
  a.open_orig[to] = 0;
  for (int64_t e = e0o; e < e0o + (e1 - e0); ++e) a.used_orig[e] = 0;   // later rounds skip the track
}

// Per caller track: whether it is open, and its entry count if so.
__global__ void __launch_bounds__(kFinalBlock) final_flag_kernel(int64_t n, const int32_t* hit_offsets,
                                                                 const uint8_t* open, int32_t* flag, int32_t* len) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const bool o = (open[t] & kFinalOpen) != 0;
  flag[t] = o ? 1 : 0;
  len[t] = o ? hit_offsets[t + 1] - hit_offsets[t] : 0;
}

// Open track t goes to sub-batch place pos[t], its entries to epos[t]...;
// the last track also writes the totals and the closing offset.
template <typename T>
__global__ void __launch_bounds__(kFinalBlock) final_gather_kernel(GatherArgs<T> a) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const bool head = blockIdx.y == 0;
  if (head && t == a.n - 1) {
    const int32_t ns = a.pos[t] + a.flag[t], nh = a.epos[t] + a.len[t];
    a.counts[0] = ns;
    a.counts[1] = nh;
    a.sub_offsets[ns] = nh;
  }
  if (!a.flag[t]) return;
  const int32_t i = a.pos[t], d0 = a.epos[t], m = a.len[t];
  const int64_t s0 = a.hit_offsets[t];
  if (head) {
    a.map[i] = int32_t(t);
    a.sub_offsets[i] = d0;
  }
  for (int32_t r = int32_t(blockIdx.y); r < m; r += int32_t(gridDim.y)) {
    const int64_t e = s0 + r, d = int64_t(d0) + r;
    a.sub_layer[d] = a.hit_layer[e];
    a.sub_used[d] = a.used[e];
#pragma unroll
    for (int k = 0; k < 3; ++k) a.sub_pos[k * a.n_hits + d] = a.hit_pos[k * a.n_hits + e];
#pragma unroll
    for (int k = 0; k < 6; ++k) a.sub_cov[k * a.n_hits + d] = a.hit_cov[k * a.n_hits + e];
  }
}

}  // namespace

template <typename T>
hipError_t launch_final_init(const FinalRoundArgs<T>& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int64_t m = a.n > a.n_hits ? a.n : a.n_hits;
  hipLaunchKernelGGL(final_init_kernel<T>, dim3(unsigned((m + kFinalBlock - 1) / kFinalBlock)), dim3(kFinalBlock), 0,
                     s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_final_round(const FinalRoundArgs<T>& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(final_round_kernel<T>, dim3(unsigned((a.n + kFinalBlock - 1) / kFinalBlock)), dim3(kFinalBlock),
                     0, s, a);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_final_gather(GatherArgs<T>& a, hipStream_t s) {
  // scans of the open flags and of the open tracks' entry counts
  size_t need = 0;
  hipError_t e = hipcub::DeviceScan::ExclusiveSum(nullptr, need, a.flag, a.pos, int(a.n), s);
  if (e != hipSuccess) return e;
  if (!a.scan_temp) {
    a.scan_bytes = need;
    return hipSuccess;
  }
  if (a.n == 0) return hipSuccess;
  const unsigned grid = unsigned((a.n + kFinalBlock - 1) / kFinalBlock);
  hipLaunchKernelGGL(final_flag_kernel, dim3(grid), dim3(kFinalBlock), 0, s, a.n, a.hit_offsets, a.open, a.flag,
                     a.len);
  size_t bytes = a.scan_bytes;
  e = hipcub::DeviceScan::ExclusiveSum(a.scan_temp, bytes, a.flag, a.pos, int(a.n), s);
  if (e != hipSuccess) return e;
  bytes = a.scan_bytes;
  e = hipcub::DeviceScan::ExclusiveSum(a.scan_temp, bytes, a.len, a.epos, int(a.n), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(final_gather_kernel<T>, dim3(grid, kFinalRows), dim3(kFinalBlock), 0, s, a);
  return hipGetLastError();
}

template hipError_t launch_final_init<float>(const FinalRoundArgs<float>&, hipStream_t);
template hipError_t launch_final_init<double>(const FinalRoundArgs<double>&, hipStream_t);
template hipError_t launch_final_round<float>(const FinalRoundArgs<float>&, hipStream_t);
template hipError_t launch_final_round<double>(const FinalRoundArgs<double>&, hipStream_t);
template hipError_t launch_final_gather<float>(GatherArgs<float>&, hipStream_t);
template hipError_t launch_final_gather<double>(GatherArgs<double>&, hipStream_t);

}  // namespace kf
