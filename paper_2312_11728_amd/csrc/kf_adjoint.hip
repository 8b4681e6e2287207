// HIP kernels of the reverse pass: one track per lane for the adjoint sweep,
// then a deterministic two-stage reduction of the hit-position gradients into
// the per-layer alignment gradient (fixed summation order: the result does
// not depend on scheduling).
#include "kf_adjoint.hpp"
#include "kf_stage.hpp"

namespace kf {

template <typename T>
__global__ void __launch_bounds__(256) adjoint_kernel(AdjArgs<T> a, GeomArgs g) {
  __shared__ GeomLds<T> sg;
  __shared__ T sal[2 * kMaxLayers];
  stage_align(sal, a.f, g);
  stage_geometry(sg, g);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.f.n) return;
  const int64_t e0 = a.f.hit_offsets[t];
  const int len = int(a.f.hit_offsets[t + 1] - e0);
  CsrTrack<T> acc{a.f, e0};
  adjoint_track(a, TrackGeom<T>{sg.kind, sg.pos, sg.x0, g.n_layers, T(g.bz), T(g.mass)}, a.f.align ? sal : nullptr,
                t, acc, len, e0);
}

// Sum over the 64 lanes of a wave by a fixed butterfly.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Stage 1: block b sums the contributions of hits [b, b+1) * kAlignChunk per
// layer.  A barrel hit h with gradient hb contributes (h_x hb_y - h_y hb_x)/R
// to the r-phi offset of its layer (the rotation m = R(a/R) h keeps the
// cross product) and hb_z to the z offset; disk hits and holes contribute 0.
// Each wave takes 64 consecutive hits at a time and, for every layer present
// among them, adds the wave sum of that layer's contributions into its own
// LDS row; the four rows are then added in a fixed order.
template <typename T>
__global__ void __launch_bounds__(256) align_partial_kernel(AdjArgs<T> a, GeomArgs g) {
  __shared__ T part[4][2][kMaxLayers];
  for (int i = threadIdx.x; i < 4 * 2 * kMaxLayers; i += blockDim.x) (&part[0][0][0])[i] = T(0);
  __syncthreads();
  const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t nh = a.f.n_hits;
  const int64_t base = int64_t(blockIdx.x) * kAlignChunk + int64_t(wv) * (kAlignChunk / 4);
  for (int b = 0; b < kAlignChunk / 4; b += 64) {
    const int64_t e = base + b + lane;
    int lay = -1;
    T cr = T(0), cz = T(0);
    if (e < nh && a.f.hit_valid[e]) {
      const int l = a.f.hit_layer[e];
      if (l >= 0 && l < g.n_layers && g.kind[l] == 0) {
        lay = l;
        const T hx = a.f.hit_pos[e], hy = a.f.hit_pos[nh + e];
        const T gx = a.grad_hit[e], gy = a.grad_hit[nh + e], gz = a.grad_hit[2 * nh + e];
        cr = (hx * gy - hy * gx) / T(g.pos[l]);
        cz = gz;
      }
    }
    uint64_t rem = __ballot(lay >= 0);
    while (rem) {
      const int leader = __ffsll((unsigned long long)rem) - 1;
      const int L = __shfl(lay, leader, 64);
      const bool mine = (lay == L);
      const T sr = wave_sum(mine ? cr : T(0));
      const T sz = wave_sum(mine ? cz : T(0));
      if (lane == 0) {
        part[wv][0][L] += sr;
        part[wv][1][L] += sz;
      }
      rem &= ~__ballot(mine);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < 2 * kMaxLayers; i += blockDim.x) {
    const int c = i / kMaxLayers, l = i % kMaxLayers;
    a.partial[int64_t(blockIdx.x) * 2 * kMaxLayers + i] = ((part[0][c][l] + part[1][c][l]) + part[2][c][l]) + part[3][c][l];
  }
}

// Stage 2: one thread per (component, layer) adds the block partials in
// block order.
template <typename T>
__global__ void __launch_bounds__(128) align_final_kernel(AdjArgs<T> a, int32_t n_layers, int64_t n_blocks) {
  const int i = threadIdx.x;
  const int c = i / kMaxLayers, l = i % kMaxLayers;
  if (c >= 2 || l >= n_layers) return;
  T acc = T(0);
  for (int64_t b = 0; b < n_blocks; ++b) acc += a.partial[b * 2 * kMaxLayers + i];
  a.grad_align[c * n_layers + l] = acc;
}

template <typename T>
hipError_t launch_adjoint(const AdjArgs<T>& a, const GeomArgs& g, hipStream_t s) {
  if (a.f.n > 0) {
    const int64_t grid = (a.f.n + 255) / 256;
    hipLaunchKernelGGL(adjoint_kernel<T>, dim3(unsigned(grid)), dim3(256), 0, s, a, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.grad_align) {
    const int64_t nb = adjoint_partial_blocks(a.f.n_hits);
    if (nb > 0) hipLaunchKernelGGL(align_partial_kernel<T>, dim3(unsigned(nb)), dim3(256), 0, s, a, g);
    hipLaunchKernelGGL(align_final_kernel<T>, dim3(1), dim3(128), 0, s, a, g.n_layers, nb);
  }
  return hipGetLastError();
}

template hipError_t launch_adjoint<float>(const AdjArgs<float>&, const GeomArgs&, hipStream_t);
template hipError_t launch_adjoint<double>(const AdjArgs<double>&, const GeomArgs&, hipStream_t);

}  // namespace kf
