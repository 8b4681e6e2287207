// Arguments and launcher of the final fit with outlier rejection (the backward
// fit in which a hit whose chi2 against the backward prediction exceeds a cut
// is not used).
#pragma once
#include "kf_kernels.hpp"

namespace kf {

// track status: at least one hit was rejected as an outlier
constexpr uint32_t TRK_OUTLIER = 128u;

template <typename T>
struct FinalArgs {
  BwdArgs<T> b;
  T chi2_cut;         // a valid hit with chi2 > chi2_cut is rejected (+inf: none)
  uint8_t* outlier;   // [n_hits] per CSR entry: 1 rejected, 0 otherwise; may be null
};

template <typename T>
hipError_t launch_final_fit(const FinalArgs<T>& a, const GeomArgs& g, hipStream_t s);

}  // namespace kf
