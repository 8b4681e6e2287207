// HIP kernels for gfx950: seeding, single-step propagate / update, and the
// fused per-track layer loop of the Kalman fit.  One track per lane; all
// per-track arrays are structure-of-arrays so that a wave's 64 lanes read and
// write contiguous memory.
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

// ---- seeding -----------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) seeds_kernel(SeedArgs<T> a) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const int64_t e0 = a.hit_offsets[t], e1 = a.hit_offsets[t + 1];
  const int64_t nh = a.n_hits;
  int64_t pick[3] = {-1, -1, -1};
  int cnt = 0;
  T lx = T(0), ly = T(0);
  for (int64_t e = e0; e < e1 && cnt < 3; ++e) {
    if (!a.hit_valid[e]) continue;
    const T hx = a.hit_pos[e], hy = a.hit_pos[nh + e];
    bool take = (cnt == 0);
    if (!take) {
      if (a.mode == 0) {
        take = true;
      } else {
        const T dx = hx - lx, dy = hy - ly;
        take = k_sqrt(dx * dx + dy * dy) >= T(3.0);
      }
    }
    if (take) {
      pick[cnt++] = e;
      lx = hx;
      ly = hy;
    }
  }
  T p[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
  int q = 1;
  uint32_t st = 0;
  if (cnt == 3) {
    T h[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) h[k][c] = a.hit_pos[c * nh + pick[k]];
    seed_from_hits(h[0], h[1], h[2], T(a.bz), p, q);
  } else {
    st |= TRK_BAD_INPUT;
  }
  const T diag[6] = {T(1), T(1), T(1), T(1), T(0.01), T(0.01)};
#pragma unroll
  for (int i = 0; i < 6; ++i) a.seed_state[i * a.ld + t] = p[i];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) a.seed_cov[sym(i, j) * a.ld + t] = (i == j) ? diag[i] : T(0);
  a.seed_charge[t] = int8_t(q);
  a.trk_status[t] = st;
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
__device__ __forceinline__ void write_checkpoint(const FitArgs<T>& a, int64_t t, int slot, const T p[6],
                                                 const T c[21], int q) {
  const int64_t stride = a.ld * int64_t(a.n_seg);
  T* base = a.ckpt + int64_t(slot) * a.ld + t;
#pragma unroll
  for (int i = 0; i < 6; ++i) base[i * stride] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) base[(6 + i) * stride] = c[i];
  base[27 * stride] = T(q);
}

template <typename T>
__device__ __forceinline__ void fit_one(const FitArgs<T>& a, const GeomArgs& g, const GeomLds<T>& sg,
                                        const T* __restrict__ sal, int64_t t) {
  const int64_t ld = a.ld, nh = a.n_hits;
  T p[6], c[21];
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = a.seed_state[i * ld + t];
#pragma unroll
  for (int i = 0; i < 21; ++i) c[i] = a.seed_cov[i * ld + t];
  int q = a.seed_charge[t];
  const int64_t e0 = a.hit_offsets[t], e1 = a.hit_offsets[t + 1];
  int64_t k0 = e0;
  while (k0 < e1 && !a.hit_valid[k0]) ++k0;
  uint32_t st = 0;
  T chi2 = T(0);
  int nval = 0;
  const T bz = T(g.bz), mass = T(g.mass);
  if (k0 >= e1) {
    st |= TRK_BAD_INPUT;
  } else {
    int prev = a.hit_layer[k0];
    for (int64_t e = k0; e < e1; ++e) {
      const int lay = a.hit_layer[e];
      if (lay < 0 || lay >= g.n_layers) {
        st |= TRK_BAD_INPUT;
        break;
      }
      const int j = int(e - k0);
      if (a.ckpt && j >= 1 && ((j - 1) % a.seg) == 0) write_checkpoint(a, t, (j - 1) / a.seg, p, c, q);
      T pp[6], cc[21];
#pragma unroll
      for (int i = 0; i < 6; ++i) pp[i] = p[i];
#pragma unroll
      for (int i = 0; i < 21; ++i) cc[i] = c[i];
      const int qq = q;
      uint32_t sst = 0;
      const int kind = sg.kind[lay];
      if (j > 0) {
        if (!propagate(p, c, q, kind, sg.pos[lay], sg.x0[lay], lay == prev, true, bz, mass, sst)) {
          st |= sst;
          break;
        }
      } else {
        add_material_here(p, c, kind, sg.x0[lay], mass, sst);
      }
      T c2 = T(0);
      const bool valid = a.hit_valid[e] != 0;
      if (valid) {
        T m[3], V[6];
        m[0] = a.hit_pos[e];
        m[1] = a.hit_pos[nh + e];
        m[2] = a.hit_pos[2 * nh + e];
#pragma unroll
        for (int i = 0; i < 6; ++i) V[i] = a.hit_cov[i * nh + e];
        if (sal && kind == 0) {
          const T ang = sal[lay] / sg.pos[lay];
          T sa, ca;
          k_sincos(ang, &sa, &ca);
          const T hx = m[0], hy = m[1];
          m[0] = ca * hx - sa * hy;
          m[1] = sa * hx + ca * hy;
          m[2] += sal[kMaxLayers + lay];
        }
        update(p, c, q, m, V, c2, sst);
      }
      if (!all_finite(p, c, c2)) {
        st |= sst | TRK_NONFINITE;
#pragma unroll
        for (int i = 0; i < 6; ++i) p[i] = pp[i];
#pragma unroll
        for (int i = 0; i < 21; ++i) c[i] = cc[i];
        q = qq;
        break;
      }
      st |= sst;
      chi2 += c2;
      nval += valid ? 1 : 0;
      prev = lay;
    }
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) a.state_out[i * ld + t] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) a.cov_out[i * ld + t] = c[i];
  a.charge_out[t] = int8_t(q);
  a.chi2[t] = chi2;
  a.ndf[t] = 2 * nval - 5;
  a.trk_status[t] = st;
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

template <typename T>
__global__ void __launch_bounds__(256) fit_kernel(FitArgs<T> a, GeomArgs g) {
  __shared__ GeomLds<T> sg;
  __shared__ T sal[2 * kMaxLayers];
  stage_align(sal, a, g);
  stage_geometry(sg, g);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  fit_one(a, g, sg, a.align ? sal : nullptr, t);
}

// Persistent form: a fixed grid of blocks pulls tiles of blockDim.x tracks from
// a device counter until none are left; every block reaches the exit.
template <typename T>
__global__ void __launch_bounds__(256) fit_persistent_kernel(FitArgs<T> a, GeomArgs g) {
  __shared__ GeomLds<T> sg;
  __shared__ T sal[2 * kMaxLayers];
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
    if (t < a.n) fit_one(a, g, sg, a.align ? sal : nullptr, t);
  }
}

__global__ void reset_counter_kernel(int32_t* c) { *c = 0; }

template <typename T>
hipError_t launch_fit(const FitArgs<T>& a, const GeomArgs& g, const FitLaunch& l, int n_cu, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int block = l.block;
  if (!l.persistent) {
    const int64_t grid = (a.n + block - 1) / block;
    hipLaunchKernelGGL(fit_kernel<T>, dim3(unsigned(grid)), dim3(block), 0, s, a, g);
    return hipGetLastError();
  }
  FitArgs<T> b = a;
  b.n_tiles = (a.n + block - 1) / block;
  int64_t grid = int64_t(n_cu) * l.blocks_per_cu;
  if (grid > b.n_tiles) grid = b.n_tiles;
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, a.tile_counter);
  hipLaunchKernelGGL(fit_persistent_kernel<T>, dim3(unsigned(grid)), dim3(block), 0, s, b, g);
  return hipGetLastError();
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
