// HIP kernels for gfx950: seeding, single-step propagate / update, and the
// fused per-track layer loop of the Kalman fit.  One track per lane; all
// per-track arrays are structure-of-arrays so that a wave's 64 lanes read and
// write contiguous memory.
#include "kf_kernels.hpp"
#include "kf_track.hpp"

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

// ---- seeding -----------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) seeds_kernel(SeedArgs<T> a) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  seed_track(a, t);
}

template <typename T>
hipError_t launch_seeds(const SeedArgs<T>& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int block = 256;
  const int64_t grid = (a.n + block - 1) / block;
  hipLaunchKernelGGL(seeds_kernel<T>, dim3(unsigned(grid)), dim3(block), 0, s, a);
  return hipGetLastError();
}

// ---- single-step propagate ----------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) propagate_kernel(PropArgs<T> a, GeomArgs g) {
  __shared__ GeomLds<T> sg;
  stage_geometry(sg, g);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  T p[6], c[21];
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = a.state_in[i * a.ld + t];
#pragma unroll
  for (int i = 0; i < 21; ++i) c[i] = a.cov_in[i * a.ld + t];
  const int q = a.charge[t];
  const int lay = a.target[t];
  uint32_t st = 0;
  T path = T(0);
  if (lay < 0 || lay >= g.n_layers) {
    st |= TRK_BAD_INPUT;
  } else {
    const bool same = a.from ? (a.from[t] == lay) : false;
    propagate(p, c, q, sg.kind[lay], sg.pos[lay], sg.x0[lay], same, a.material != 0, T(g.bz), T(g.mass), st,
              &path);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) a.state_out[i * a.ld + t] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) a.cov_out[i * a.ld + t] = c[i];
  if (a.path) a.path[t] = path;
  a.trk_status[t] |= st;
}

template <typename T>
hipError_t launch_propagate(const PropArgs<T>& a, const GeomArgs& g, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int block = 256;
  const int64_t grid = (a.n + block - 1) / block;
  hipLaunchKernelGGL(propagate_kernel<T>, dim3(unsigned(grid)), dim3(block), 0, s, a, g);
  return hipGetLastError();
}

// ---- single-step update ---------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) update_kernel(UpdArgs<T> a) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  T p[6], c[21], m[3], V[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = a.state[i * a.ld + t];
#pragma unroll
  for (int i = 0; i < 21; ++i) c[i] = a.cov[i * a.ld + t];
#pragma unroll
  for (int i = 0; i < 3; ++i) m[i] = a.hit_pos[i * a.ld + t];
#pragma unroll
  for (int i = 0; i < 6; ++i) V[i] = a.hit_cov[i * a.ld + t];
  int q = a.charge[t];
  uint32_t st = 0;
  T chi2 = T(0);
  update(p, c, q, m, V, chi2, st);
#pragma unroll
  for (int i = 0; i < 6; ++i) a.state[i * a.ld + t] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) a.cov[i * a.ld + t] = c[i];
  a.charge[t] = int8_t(q);
  a.chi2[t] = chi2;
  a.trk_status[t] |= st;
}

template <typename T>
hipError_t launch_update(const UpdArgs<T>& a, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int block = 256;
  const int64_t grid = (a.n + block - 1) / block;
  hipLaunchKernelGGL(update_kernel<T>, dim3(unsigned(grid)), dim3(block), 0, s, a);
  return hipGetLastError();
}

// ---- fused per-track layer loop ----------------------------------------------------

template <typename T>
__device__ __forceinline__ void stage_align(T* sal, const FitArgs<T>& a, const GeomArgs& g) {
  if (a.align) {
    for (int i = threadIdx.x; i < g.n_layers; i += blockDim.x) {
      sal[i] = a.align[i];
      sal[kMaxLayers + i] = a.align[g.n_layers + i];
    }
  }
}

constexpr int kFitBlock = 256;   // upper bound of the fit kernels' block size

// One thread per track.  WAVES: the minimum number of waves per SIMD the
// register allocation must allow (1 or 2); the autotuner picks the faster.
template <typename T, int WAVES>
__global__ void __launch_bounds__(kFitBlock, WAVES) fit_kernel(FitArgs<T> a, GeomArgs g) {
  __shared__ GeomLds<T> sg;
  __shared__ T sal[2 * kMaxLayers];
  __shared__ T bk[28 * kFitBlock];
  stage_align(sal, a, g);
  stage_geometry(sg, g);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  fit_track(a, TrackGeom<T>{sg.kind, sg.pos, sg.x0, g.n_layers, T(g.bz), T(g.mass)}, a.align ? sal : nullptr, t,
            bk + threadIdx.x, int(blockDim.x));
}

// Persistent form: a fixed grid of blocks pulls tiles of blockDim.x tracks from
// a device counter until none are left; every block reaches the exit.
template <typename T, int WAVES>
__global__ void __launch_bounds__(kFitBlock, WAVES) fit_persistent_kernel(FitArgs<T> a, GeomArgs g) {
  __shared__ GeomLds<T> sg;
  __shared__ T sal[2 * kMaxLayers];
  __shared__ T bk[28 * kFitBlock];
  __shared__ int64_t tile;
  stage_align(sal, a, g);
  stage_geometry(sg, g);
  for (;;) {
    if (threadIdx.x == 0) tile = atomicAdd(a.tile_counter, 1);
    __syncthreads();
    const int64_t my = tile;
    __syncthreads();
    if (my >= a.n_tiles) break;
    const int64_t t = my * blockDim.x + threadIdx.x;
    if (t < a.n)
      fit_track(a, TrackGeom<T>{sg.kind, sg.pos, sg.x0, g.n_layers, T(g.bz), T(g.mass)}, a.align ? sal : nullptr, t,
                bk + threadIdx.x, int(blockDim.x));
  }
}

__global__ void reset_counter_kernel(int32_t* c) { *c = 0; }

template <typename T, int WAVES>
hipError_t launch_fit_w(const FitArgs<T>& a, const GeomArgs& g, const FitLaunch& l, int n_cu, hipStream_t s) {
  const int block = l.block;
  if (!l.persistent) {
    const int64_t grid = (a.n + block - 1) / block;
    hipLaunchKernelGGL((fit_kernel<T, WAVES>), dim3(unsigned(grid)), dim3(block), 0, s, a, g);
    return hipGetLastError();
  }
  FitArgs<T> b = a;
  b.n_tiles = (a.n + block - 1) / block;
  int64_t grid = int64_t(n_cu) * l.blocks_per_cu;
  if (grid > b.n_tiles) grid = b.n_tiles;
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, a.tile_counter);
  hipLaunchKernelGGL((fit_persistent_kernel<T, WAVES>), dim3(unsigned(grid)), dim3(block), 0, s, b, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fit(const FitArgs<T>& a, const GeomArgs& g, const FitLaunch& l, int n_cu, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  if (l.waves == 2) return launch_fit_w<T, 2>(a, g, l, n_cu, s);
  return launch_fit_w<T, 1>(a, g, l, n_cu, s);
}

// explicit instantiations
template hipError_t launch_seeds<float>(const SeedArgs<float>&, hipStream_t);
template hipError_t launch_seeds<double>(const SeedArgs<double>&, hipStream_t);
template hipError_t launch_propagate<float>(const PropArgs<float>&, const GeomArgs&, hipStream_t);
template hipError_t launch_propagate<double>(const PropArgs<double>&, const GeomArgs&, hipStream_t);
template hipError_t launch_update<float>(const UpdArgs<float>&, hipStream_t);
template hipError_t launch_update<double>(const UpdArgs<double>&, hipStream_t);
template hipError_t launch_fit<float>(const FitArgs<float>&, const GeomArgs&, const FitLaunch&, int, hipStream_t);
template hipError_t launch_fit<double>(const FitArgs<double>&, const GeomArgs&, const FitLaunch&, int, hipStream_t);

}  // namespace kf
