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

// The states the reverse sweep reads (seg > 1 with a state buffer), one
// thread per track, at the forward fit's occupancy rather than under the
// reverse pass's registers: for every entry j >= 1 (relative to the track's
// first valid entry), the state before it -- the checkpoint at the start of
// each segment, then the segment's forward steps -- stored in slot j - 1.
// These are the steps fill_segment takes, in the same order on the same
// values.  The wave's hits come through LDS a few entries per track at a
// time, as in the forward fit: all rows of a chunk are loaded before any is
// written, consecutive lanes reading consecutive entries of one track (a
// slot past a track's end loads its last entry and is never read).
constexpr int kRefillBlock = 256;

template <typename T, int J>
__device__ void refill_wave_staged(const AdjArgs<T>& a, const TrackGeom<T>& g, const T* __restrict__ sal, int64_t w0,
                                   StageBuf<T, J>& sb) {
  const FitArgs<T>& f = a.f;
  const int lane = int(threadIdx.x) & 63;
  const int64_t t = w0 + lane;
  const bool in_range = t < f.n;
  int64_t e0 = 0;
  int len = 0;
  if (in_range) {
    e0 = f.hit_offsets[t];
    len = int(f.hit_offsets[t + 1] - e0);
    if (len > f.max_len) len = f.max_len;
  }
  sb.e0[lane] = e0;
  sb.len[lane] = len;
  const int kmax = wave_max(len);
  const int64_t nh = f.n_hits, n = f.n, cst = f.ld * int64_t(f.n_seg);
  T p[6], c[21];
  int q = 0, prev = 0, prev_lay = 0, k0 = -1;
  wave_sync();
  for (int j0 = 0; j0 < kmax; j0 += J) {
    int32_t lvr[J];
    T vr[J][9];
#pragma unroll
    for (int r = 0; r < J; ++r) {
      const int idx = r * 64 + lane;
      const int l = idx / J, jj = idx % J;
      const int ln = sb.len[l];
      const int64_t e = ln > 0 ? sb.e0[l] + min(j0 + jj, ln - 1) : 0;
      lvr[r] = int32_t(uint16_t(f.hit_layer[e])) | (f.hit_valid[e] ? (1 << 16) : 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) vr[r][k] = f.hit_pos[k * nh + e];
#pragma unroll
      for (int k = 0; k < 6; ++k) vr[r][3 + k] = f.hit_cov[k * nh + e];
    }
#pragma unroll
    for (int r = 0; r < J; ++r) {
      const int idx = r * 64 + lane;
      const int l = idx / J, jj = idx % J;
      sb.lv[jj][l] = lvr[r];
#pragma unroll
      for (int k = 0; k < 9; ++k) sb.v[k][jj][l] = vr[r][k];
    }
    wave_sync();
    const int jn = min(J, kmax - j0);
    for (int jj = 0; jj < jn; ++jj) {
      const int k = j0 + jj;
      if (!in_range || k >= len) continue;
      const int32_t lv = sb.lv[jj][lane];
      const bool valid = (lv >> 16) != 0;
      const int lay = int16_t(lv & 0xffff);
      if (k0 < 0) {
        if (valid) k0 = k;   // entry j = 0: its state is the seed
        prev_lay = lay;
        continue;
      }
      const int j = k - k0;
      if ((j - 1) % f.seg == 0) {
        // a segment starts: its checkpoint, after entry j - 1 of layer prev_lay
        const T* base = f.ckpt + int64_t((j - 1) / f.seg) * f.ld + t;
#pragma unroll
        for (int i = 0; i < 6; ++i) p[i] = base[i * cst];
#pragma unroll
        for (int i = 0; i < 21; ++i) c[i] = base[(6 + i) * cst];
        q = int(base[27 * cst]);
        prev = prev_lay;
      }
      T* slot = a.seg_buf + int64_t(j - 1) * kSegVals * n + t;
#pragma unroll
      for (int i = 0; i < 6; ++i) slot[i * n] = p[i];
#pragma unroll
      for (int i = 0; i < 21; ++i) slot[(6 + i) * n] = c[i];
      slot[27 * n] = T(q);
      slot[28 * n] = T(prev);
      if (j % f.seg != 0 && j + 1 < len - k0) {
        T m[3], V[6];
#pragma unroll
        for (int x = 0; x < 3; ++x) m[x] = sb.v[x][jj][lane];
#pragma unroll
        for (int x = 0; x < 6; ++x) V[x] = sb.v[3 + x][jj][lane];
        T c2;
        uint32_t sst = 0;
        step_forward(p, c, q, j, lay, prev, valid, m, V, g, sal, c2, sst);
        prev = lay;
      }
      prev_lay = lay;
    }
    wave_sync();   // every lane has read the chunk before the next one is staged
  }
}

template <typename T>
__global__ void __launch_bounds__(kRefillBlock, sizeof(T) == 4 ? 2 : 1) refill_kernel(AdjArgs<T> a, GeomArgs g) {
  constexpr int J = stage_entries<T, sizeof(T) == 4 ? 2 : 1>();
  __shared__ GeomLds<T> sg;
  __shared__ T sal[2 * kMaxLayers];
  __shared__ StageBuf<T, J> sb[kRefillBlock / 64];
  stage_align(sal, a.f, g);
  stage_geometry(sg, g);
  const int64_t w0 = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u);
  refill_wave_staged<T, J>(a, TrackGeom<T>{sg.kind, sg.pos, sg.x0, g.n_layers, T(g.bz), T(g.mass)},
                           a.f.align ? sal : nullptr, w0, sb[threadIdx.x >> 6]);
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
    if (a.seg_buf)
      hipLaunchKernelGGL(refill_kernel<T>, dim3(unsigned((a.f.n + kRefillBlock - 1) / kRefillBlock)), dim3(kRefillBlock), 0,
                         s, a, g);
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
