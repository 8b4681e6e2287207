// Kernels of the tilted-module entry points: one track per lane, the module
// table read from global memory (thousands of modules, each read by the few
// tracks crossing it, so the L2 serves it).
#include <hip/hip_runtime.h>

#include "kf_plane.hpp"
#include "kf_plane_fit.hpp"
#include "kf_plane_launch.hpp"

namespace kf {

namespace {

template <typename T>
__global__ void __launch_bounds__(256) propagate_plane_kernel(PlanePropArgs<T> a, PlaneGeomArgs<T> g) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  T p[6], c[21];
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = a.state_in[i * a.ld + t];
#pragma unroll
  for (int i = 0; i < 21; ++i) c[i] = a.cov_in[i * a.ld + t];
  const int q = a.charge[t];
  const int64_t mod = a.module[t];
  uint32_t st = 0;
  T path = T(0);
  if (mod < 0 || mod >= g.n_modules) {
    st |= TRK_BAD_INPUT;
  } else {
    Plane<T> pl;
    load_plane(g.table, g.n_modules, mod, pl);
    propagate_plane(p, c, q, pl, a.material != 0, T(g.bz), T(g.mass), st, &path);
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) a.state_out[i * a.ld + t] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) a.cov_out[i * a.ld + t] = c[i];
  if (a.path) a.path[t] = path;
  a.trk_status[t] |= st;
}

template <typename T>
__global__ void __launch_bounds__(256) update_plane_kernel(PlaneUpdArgs<T> a, PlaneGeomArgs<T> g) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const int64_t mod = a.module[t];
  if (mod < 0 || mod >= g.n_modules) {
    a.chi2[t] = T(0);
    a.trk_status[t] |= TRK_BAD_INPUT;
    return;
  }
  T p[6], c[21], m[2], V[3];
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = a.state[i * a.ld + t];
#pragma unroll
  for (int i = 0; i < 21; ++i) c[i] = a.cov[i * a.ld + t];
  m[0] = a.hit_uv[t];
  m[1] = a.hit_uv[a.ld + t];
#pragma unroll
  for (int i = 0; i < 3; ++i) V[i] = a.hit_cov_uv[i * a.ld + t];
  Plane<T> pl;
  load_plane(g.table, g.n_modules, mod, pl);
  int q = a.charge[t];
  uint32_t st = 0;
  T chi2 = T(0);
  update_plane(p, c, q, pl, m, V, chi2, st);
#pragma unroll
  for (int i = 0; i < 6; ++i) a.state[i * a.ld + t] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) a.cov[i * a.ld + t] = c[i];
  a.charge[t] = int8_t(q);
  a.chi2[t] = chi2;
  a.trk_status[t] |= st;
}

// Forward fit over tilted modules, one track per lane (fit_plane_track).
template <typename T>
__global__ void __launch_bounds__(256) fit_plane_kernel(PlaneFitArgs<T> a, PlaneGeomArgs<T> g) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  fit_plane_track(a, g, t);
}

template <typename T>
__global__ void __launch_bounds__(256) plane_to_global_kernel(int64_t nh, const int32_t* __restrict__ module,
                                                              const T* __restrict__ uv, PlaneGeomArgs<T> g,
                                                              T* __restrict__ pos) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= nh) return;
  const int64_t mod = module[e];
  T x = k_nan<T>(), y = k_nan<T>(), z = k_nan<T>();
  if (mod >= 0 && mod < g.n_modules) {
    Plane<T> pl;
    load_plane(g.table, g.n_modules, mod, pl);
    const T mu = uv[e], mv = uv[nh + e];
    x = pl.cx + mu * pl.ux + mv * pl.vx;
    y = pl.cy + mu * pl.uy + mv * pl.vy;
    z = pl.cz + mu * pl.uz + mv * pl.vz;
  }
  pos[e] = x;
  pos[nh + e] = y;
  pos[2 * nh + e] = z;
}

inline int64_t grid_of(int64_t n) { return (n + 255) / 256; }

}  // namespace

template <typename T>
hipError_t launch_propagate_plane(const PlanePropArgs<T>& a, const PlaneGeomArgs<T>& g, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(propagate_plane_kernel<T>, dim3(unsigned(grid_of(a.n))), dim3(256), 0, s, a, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_update_plane(const PlaneUpdArgs<T>& a, const PlaneGeomArgs<T>& g, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(update_plane_kernel<T>, dim3(unsigned(grid_of(a.n))), dim3(256), 0, s, a, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fit_plane(const PlaneFitArgs<T>& a, const PlaneGeomArgs<T>& g, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(fit_plane_kernel<T>, dim3(unsigned(grid_of(a.n))), dim3(256), 0, s, a, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_plane_to_global(int64_t nh, const int32_t* module, const T* uv, const PlaneGeomArgs<T>& g, T* pos,
                                  hipStream_t s) {
  if (nh == 0) return hipSuccess;
  hipLaunchKernelGGL(plane_to_global_kernel<T>, dim3(unsigned(grid_of(nh))), dim3(256), 0, s, nh, module, uv, g, pos);
  return hipGetLastError();
}

template hipError_t launch_plane_to_global<float>(int64_t, const int32_t*, const float*, const PlaneGeomArgs<float>&,
                                                  float*, hipStream_t);
template hipError_t launch_plane_to_global<double>(int64_t, const int32_t*, const double*,
                                                   const PlaneGeomArgs<double>&, double*, hipStream_t);
template hipError_t launch_propagate_plane<float>(const PlanePropArgs<float>&, const PlaneGeomArgs<float>&,
                                                  hipStream_t);
template hipError_t launch_propagate_plane<double>(const PlanePropArgs<double>&, const PlaneGeomArgs<double>&,
                                                   hipStream_t);
template hipError_t launch_update_plane<float>(const PlaneUpdArgs<float>&, const PlaneGeomArgs<float>&, hipStream_t);
template hipError_t launch_update_plane<double>(const PlaneUpdArgs<double>&, const PlaneGeomArgs<double>&,
                                                hipStream_t);
template hipError_t launch_fit_plane<float>(const PlaneFitArgs<float>&, const PlaneGeomArgs<float>&, hipStream_t);
template hipError_t launch_fit_plane<double>(const PlaneFitArgs<double>&, const PlaneGeomArgs<double>&, hipStream_t);

}  // namespace kf
