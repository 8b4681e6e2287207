// Per-block staging of the detector description (and the alignment) in LDS,
// shared by the fit and adjoint kernels.
#pragma once

#include "kf_kernels.hpp"

namespace kf {

// ---- geometry staged in LDS --------------------------------------------------
template <typename T>
struct GeomLds {
  T pos[kMaxLayers];
  T x0[kMaxLayers];
  int kind[kMaxLayers];
};

template <typename T>
__device__ __forceinline__ void stage_geometry(GeomLds<T>& sg, const GeomArgs& g) {
  for (int i = threadIdx.x; i < g.n_layers; i += blockDim.x) {
    sg.pos[i] = T(g.pos[i]);
    sg.x0[i] = T(g.x0[i]);
    sg.kind[i] = g.kind[i];
  }
  __syncthreads();
}

template <typename T>
__device__ __forceinline__ void stage_align(T* sal, const FitArgs<T>& a, const GeomArgs& g) {
  if (a.align) {
    for (int i = threadIdx.x; i < g.n_layers; i += blockDim.x) {
      sal[i] = a.align[i];
      sal[kMaxLayers + i] = a.align[g.n_layers + i];
    }
  }
}

}  // namespace kf
