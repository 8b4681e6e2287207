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

// The states the reverse sweep reads, one thread per track (seg > 1 with a
// state buffer): every checkpoint segment recomputed once, at the forward
// fit's occupancy rather than under the reverse pass's registers.
template <typename T>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 2 : 1) refill_kernel(AdjArgs<T> a, GeomArgs g) {
  __shared__ GeomLds<T> sg;
  __shared__ T sal[2 * kMaxLayers];
  stage_align(sal, a.f, g);
  stage_geometry(sg, g);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.f.n) return;
  const int64_t e0 = a.f.hit_offsets[t];
  const int len = int(a.f.hit_offsets[t + 1] - e0);
  CsrTrack<T> acc{a.f, e0};
  refill_track(a, TrackGeom<T>{sg.kind, sg.pos, sg.x0, g.n_layers, T(g.bz), T(g.mass)}, a.f.align ? sal : nullptr,
               t, acc, len);
}

// Stage 1: one wave per kAlignPerBlock consecutive entries of the batch
// (entries hit_offsets[0] .. hit_offsets[n]), lane l taking entries l,
// l + 64, ... of the block's range, so that every load of the wave is
// coalesced.  A barrel hit h with gradient hb contributes
// (h_x hb_y - h_y hb_x)/R to the r-phi offset of its layer (the rotation
// m = R(a/R) h keeps the cross product) and hb_z to the z offset; disk hits
// and holes contribute 0.  Each lane adds into its own LDS column; then lane
// l adds the 64 columns of layer l in lane order.  Fixed order throughout:
// the result does not depend on scheduling.
template <typename T>
__global__ void __launch_bounds__(64) align_partial_kernel(AdjArgs<T> a, GeomArgs g) {
  __shared__ T part[2][kMaxLayers][64];
  const int lane = threadIdx.x;
  for (int l = 0; l < kMaxLayers; ++l) {
    part[0][l][lane] = T(0);
    part[1][l][lane] = T(0);
  }
  const int64_t nh = a.f.n_hits;
  const int64_t first = a.f.hit_offsets[0], last = a.f.hit_offsets[a.f.n];
  const int64_t b0 = first + int64_t(blockIdx.x) * kAlignPerBlock;
  // loads from a clamped index and predicates instead of early exits, so
  // that the loads of several iterations are in flight together
#pragma unroll 8
  for (int k = 0; k < kAlignPerBlock / 64; ++k) {
    const int64_t e = b0 + int64_t(k) * 64 + lane;
    const bool in = e < last;
    const int64_t ee = in ? e : first;
    const bool v = a.f.hit_valid[ee] != 0;
    const int l = a.f.hit_layer[ee];
    const T hx = a.f.hit_pos[ee], hy = a.f.hit_pos[nh + ee];
    const T gx = a.grad_hit[ee], gy = a.grad_hit[nh + ee], gz = a.grad_hit[2 * nh + ee];
    if (in && v && l >= 0 && l < g.n_layers && g.kind[l] == 0) {
      part[0][l][lane] += (hx * gy - hy * gx) / T(g.pos[l]);
      part[1][l][lane] += gz;
    }
  }
  __syncthreads();
  T* out = a.partial + int64_t(blockIdx.x) * 2 * kMaxLayers;
  for (int c = 0; c < 2; ++c) {
    T acc = T(0);
    for (int k = 0; k < 64; ++k) acc += part[c][lane][k];
    out[c * kMaxLayers + lane] = acc;
  }
}

// Stage 2: one block per (component, layer): thread k adds the partials of
// blocks k, k + 256, ... in order, then a fixed tree over the threads.
template <typename T>
__global__ void __launch_bounds__(256) align_final_kernel(AdjArgs<T> a, int32_t n_layers, int64_t n_blocks) {
  __shared__ T red[256];
  const int c = blockIdx.x / n_layers, l = blockIdx.x % n_layers;
  T acc = T(0);
  for (int64_t b = threadIdx.x; b < n_blocks; b += 256) acc += a.partial[b * 2 * kMaxLayers + c * kMaxLayers + l];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.grad_align[c * n_layers + l] = red[0];
}

template <typename T>
hipError_t launch_adjoint(const AdjArgs<T>& a, const GeomArgs& g, hipStream_t s) {
  if (a.f.n > 0) {
    const int64_t grid = (a.f.n + 255) / 256;
    if (a.seg_buf) hipLaunchKernelGGL(refill_kernel<T>, dim3(unsigned(grid)), dim3(256), 0, s, a, g);
    hipLaunchKernelGGL(adjoint_kernel<T>, dim3(unsigned(grid)), dim3(256), 0, s, a, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (a.grad_align) {
    // no tracks: nothing contributes (and the offsets may be absent)
    const int64_t nb = a.f.n > 0 ? adjoint_partial_blocks(a.f.n_hits) : 0;
    if (nb > 0) hipLaunchKernelGGL(align_partial_kernel<T>, dim3(unsigned(nb)), dim3(64), 0, s, a, g);
    hipLaunchKernelGGL(align_final_kernel<T>, dim3(unsigned(2 * g.n_layers)), dim3(256), 0, s, a, g.n_layers, nb);
  }
  return hipGetLastError();
}

template hipError_t launch_adjoint<float>(const AdjArgs<float>&, const GeomArgs&, hipStream_t);
template hipError_t launch_adjoint<double>(const AdjArgs<double>&, const GeomArgs&, hipStream_t);

}  // namespace kf
