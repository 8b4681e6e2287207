// Per-block staging of the detector description (and the alignment) in LDS,
// shared by the fit and adjoint kernels, and the per-wave staging buffer of
// the hit entries used by the staged fit kernels (forward and backward).
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

// ---- hits of a wave staged in LDS, a few entries per track at a time ----------

// entries per track and chunk: the LDS of a 256-thread block (4 waves) plus
// the state backup must allow the WAVES blocks per CU the register budget
// allows
template <typename T, int WAVES>
constexpr int stage_entries() {
  return sizeof(T) == 4 ? (WAVES == 1 ? 8 : 4) : (WAVES == 1 ? 4 : 1);
}

template <typename T, int J>
struct StageBuf {
  T v[9][J][64];        // hit x, y, z, then the 6 covariance terms
  int32_t lv[J][64];    // layer (low 16 bits) | valid << 16
  int64_t e0[64];       // first entry of each lane's track
  int32_t len[64];      // entries of each lane's track (0: no track)
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

}  // namespace kf
