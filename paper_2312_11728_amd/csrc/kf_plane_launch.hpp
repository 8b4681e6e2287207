// Kernel arguments and launchers of the tilted-module entry points (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kf {

// The module table and the field: table [10][n_modules] in the call's type.
template <typename T>
struct PlaneGeomArgs {
  const T* table;
  int64_t n_modules;
  double bz;
  double mass;
};

template <typename T>
struct PlanePropArgs {
  int64_t n, ld;
  const T* state_in;
  const T* cov_in;
  const int8_t* charge;
  const int32_t* module;   // [n]
  int32_t material;
  T* state_out;
  T* cov_out;
  T* path;
  uint32_t* trk_status;
};

template <typename T>
struct PlaneUpdArgs {
  int64_t n, ld;
  T* state;
  T* cov;
  int8_t* charge;
  const int32_t* module;   // [n]
  const T* hit_uv;         // [2][ld]
  const T* hit_cov_uv;     // [3][ld] (uu, vu, vv)
  T* chi2;
  uint32_t* trk_status;
};

template <typename T>
struct PlaneFitArgs {
  int64_t n, ld, n_hits;
  const T* seed_state;
  const T* seed_cov;
  const int8_t* seed_charge;
  const int32_t* hit_offsets;
  const int32_t* hit_module;
  const uint8_t* hit_valid;
  const T* hit_uv;         // [2][n_hits]
  const T* hit_cov_uv;     // [3][n_hits]
  T* state_out;
  T* cov_out;
  int8_t* charge_out;
  T* chi2;
  int32_t* ndf;
  uint32_t* trk_status;
};

template <typename T>
hipError_t launch_propagate_plane(const PlanePropArgs<T>& a, const PlaneGeomArgs<T>& g, hipStream_t s);
template <typename T>
hipError_t launch_update_plane(const PlaneUpdArgs<T>& a, const PlaneGeomArgs<T>& g, hipStream_t s);
template <typename T>
hipError_t launch_fit_plane(const PlaneFitArgs<T>& a, const PlaneGeomArgs<T>& g, hipStream_t s);
template <typename T>
hipError_t launch_plane_to_global(int64_t nh, const int32_t* module, const T* uv, const PlaneGeomArgs<T>& g, T* pos,
                                  hipStream_t s);

}  // namespace kf
