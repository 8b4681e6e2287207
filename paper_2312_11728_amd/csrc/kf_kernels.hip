// HIP kernels for gfx950: seeding, single-step propagate / update, and the
// fused per-track layer loop of the Kalman fit.  One track per lane; all
// per-track arrays are structure-of-arrays so that a wave's 64 lanes read and
// write contiguous memory.
#include "kf_kernels.hpp"
#include "kf_stage.hpp"
#include "kf_track.hpp"

namespace kf {

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

constexpr int kFitBlock = 256;   // upper bound of the fit kernels' block size

// One thread per track.  WAVES: the minimum number of waves per SIMD the
// register allocation must allow (1 or 2); the autotuner picks the faster.
template <typename T, int WAVES, int LAYOUT>
__global__ void __launch_bounds__(kFitBlock, WAVES) fit_kernel(FitArgs<T> a, GeomArgs g) {
  __shared__ GeomLds<T> sg;
  __shared__ T sal[2 * kMaxLayers];
  __shared__ T bk[28 * kFitBlock];
  stage_align(sal, a, g);
  stage_geometry(sg, g);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  fit_slot<T, LAYOUT>(a, TrackGeom<T>{sg.kind, sg.pos, sg.x0, g.n_layers, T(g.bz), T(g.mass)},
                      a.align ? sal : nullptr, t, bk + threadIdx.x, int(blockDim.x));
}

// Persistent form: a fixed grid of blocks pulls tiles of blockDim.x tracks from
// a device counter until none are left; every block reaches the exit.
template <typename T, int WAVES, int LAYOUT>
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
      fit_slot<T, LAYOUT>(a, TrackGeom<T>{sg.kind, sg.pos, sg.x0, g.n_layers, T(g.bz), T(g.mass)},
                          a.align ? sal : nullptr, t, bk + threadIdx.x, int(blockDim.x));
  }
}

// ---- CSR hits staged through LDS by each wave (layouts 3 and 4) ------------------
//
// A lane reading its own track's entries from the CSR arrays touches one cache
// line per lane and per load, and the lines are evicted before the next entry
// reuses them.  Here the 64 lanes of a wave first copy the next J entries of
// all 64 tracks into LDS together -- consecutive lanes read consecutive entries
// of one track, so a load instruction covers 64 / J runs of J contiguous
// values -- and then each lane steps through its own J entries from LDS.  The
// entry loop is uniform over the wave (the longest track of the wave sets its
// length); lanes whose track has ended or stopped sit out the steps but still
// take part in the staging.  No pass over the hits before the fit.

// Forward fit of the tracks in slots [w0, w0 + 64) (one wave; slot i holds
// track order[i] when sorted, else track i; slots >= n hold no track).  Every
// lane of the wave must call it.
template <typename T, int J, bool SORTED>
__device__ void fit_wave_staged(const FitArgs<T>& a, const TrackGeom<T>& g, const T* __restrict__ sal, int64_t w0,
                                StageBuf<T, J>& sb, T* bk, int bk_stride) {
  static_assert((J & (J - 1)) == 0 && J <= 64, "J must be a power of two <= 64");
  const int lane = int(threadIdx.x) & 63;
  const int64_t i = w0 + lane;
  const bool in_range = i < a.n;
  int64_t t = 0, e0 = 0;
  int len = 0;
  if (in_range) {
    t = SORTED ? int64_t(a.pk.order[i]) : i;
    e0 = a.hit_offsets[t];
    len = int(a.hit_offsets[t + 1] - e0);
  }
  uint32_t st = 0;
  if (len > a.max_len) {
    st |= TRK_BAD_INPUT;
    len = a.max_len;
  }
  sb.e0[lane] = e0;
  sb.len[lane] = len;
  const int kmax = wave_max(len);
  T p[6], c[21];
  int q = 0;
  if (in_range) load_seed(a, t, g.bz, p, c, q, st);
  T chi2 = T(0);
  int nval = 0, prev = 0, k0 = -1;
  bool live = in_range;
  const int64_t nh = a.n_hits;
  wave_sync();
  for (int j0 = 0; j0 < kmax; j0 += J) {
    // All J rows are loaded before any is written to LDS, so the chunk costs
    // one memory round trip.  A slot past the end of its track loads the
    // track's last entry instead (an address that is always valid: kmax > 0
    // means some track has an entry, so n_hits > 0); that slot is never read.
    int32_t lvr[J];
    T vr[J][9];
#pragma unroll
    for (int r = 0; r < J; ++r) {
      const int idx = r * 64 + lane;
      const int l = idx / J, jj = idx % J;
      const int ln = sb.len[l];
      const int64_t e = ln > 0 ? sb.e0[l] + min(j0 + jj, ln - 1) : 0;
      lvr[r] = int32_t(uint16_t(a.hit_layer[e])) | (a.hit_valid[e] ? (1 << 16) : 0);
#pragma unroll
      for (int k = 0; k < 3; ++k) vr[r][k] = a.hit_pos[k * nh + e];
#pragma unroll
      for (int k = 0; k < 6; ++k) vr[r][3 + k] = a.hit_cov[k * nh + e];
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
      if (!live || k >= len) continue;
      const int32_t lv = sb.lv[jj][lane];
      const bool valid = (lv >> 16) != 0;
      const int lay = int16_t(lv & 0xffff);
      if (k0 < 0) {
        if (!valid) continue;   // leading holes: the fit starts at the first valid entry
        k0 = k;
        prev = lay;
      }
      T m[3], V[6];
#pragma unroll
      for (int x = 0; x < 3; ++x) m[x] = sb.v[x][jj][lane];
#pragma unroll
      for (int x = 0; x < 6; ++x) V[x] = sb.v[3 + x][jj][lane];
      live = fit_entry(a, g, sal, t, k - k0, lay, prev, valid, m, V, p, c, q, st, chi2, nval, bk, bk_stride);
    }
    wave_sync();   // every lane has read the chunk before the next one is staged
  }
  if (in_range) {
    if (k0 < 0) st |= TRK_BAD_INPUT;
    store_fit(a, t, p, c, q, chi2, nval, st);
  }
}

template <typename T, int WAVES, bool SORTED>
__global__ void __launch_bounds__(kFitBlock, WAVES) fit_staged_kernel(FitArgs<T> a, GeomArgs g) {
  constexpr int J = stage_entries<T, WAVES>();
  __shared__ GeomLds<T> sg;
  __shared__ T sal[2 * kMaxLayers];
  __shared__ T bk[28 * kFitBlock];
  __shared__ StageBuf<T, J> sb[kFitBlock / 64];
  stage_align(sal, a, g);
  stage_geometry(sg, g);
  const int64_t w0 = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u);
  fit_wave_staged<T, J, SORTED>(a, TrackGeom<T>{sg.kind, sg.pos, sg.x0, g.n_layers, T(g.bz), T(g.mass)},
                                a.align ? sal : nullptr, w0, sb[threadIdx.x >> 6], bk + threadIdx.x,
                                int(blockDim.x));
}

template <typename T, int WAVES, bool SORTED>
__global__ void __launch_bounds__(kFitBlock, WAVES) fit_staged_persistent_kernel(FitArgs<T> a, GeomArgs g) {
  constexpr int J = stage_entries<T, WAVES>();
  __shared__ GeomLds<T> sg;
  __shared__ T sal[2 * kMaxLayers];
  __shared__ T bk[28 * kFitBlock];
  __shared__ StageBuf<T, J> sb[kFitBlock / 64];
  __shared__ int64_t tile;
  stage_align(sal, a, g);
  stage_geometry(sg, g);
  for (;;) {
    if (threadIdx.x == 0) tile = atomicAdd(a.tile_counter, 1);
    __syncthreads();
    const int64_t my = tile;
    __syncthreads();
    if (my >= a.n_tiles) break;
    const int64_t w0 = my * blockDim.x + (threadIdx.x & ~63u);
    fit_wave_staged<T, J, SORTED>(a, TrackGeom<T>{sg.kind, sg.pos, sg.x0, g.n_layers, T(g.bz), T(g.mass)},
                                  a.align ? sal : nullptr, w0, sb[threadIdx.x >> 6], bk + threadIdx.x,
                                  int(blockDim.x));
  }
}

__global__ void reset_counter_kernel(int32_t* c) { *c = 0; }

// ---- packed, length-sorted hit layout ------------------------------------------

__global__ void zero_ints_kernel(int32_t* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Tracks of the length sort per block: a contiguous range, walked in steps of
// the block size, so that a 500k-track batch needs a few hundred blocks and
// the per-block global atomics stay few.
constexpr int kSortPerBlock = 2048;

__device__ __forceinline__ int clamped_length(const int32_t* off, int64_t t, int32_t max_len) {
  const int len = off[t + 1] - off[t];
  return len < 0 ? 0 : (len > max_len ? max_len : len);
}

// entry count of every track (clamped to max_len) into a histogram: per-block
// counts in LDS, then one global atomic per block and length
constexpr int kSortBlock = 1024;

__global__ void __launch_bounds__(kSortBlock) length_hist_kernel(const int32_t* off, int64_t n, int32_t max_len,
                                                          int32_t* hist) {
  __shared__ int32_t h[kMaxLen + 1];
  for (int i = threadIdx.x; i <= kMaxLen; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int64_t b0 = int64_t(blockIdx.x) * kSortPerBlock;
  const int64_t b1 = b0 + kSortPerBlock < n ? b0 + kSortPerBlock : n;
  for (int64_t base = b0; base < b1; base += blockDim.x) {
    const int64_t t = base + threadIdx.x;
    if (t < b1) atomicAdd(&h[clamped_length(off, t, max_len)], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= kMaxLen; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Cursors of the length-sorted order (longest first) and, for the packed
// layout, the first element of every tile: the tracks of tile tau are slots
// tau*64 ... tau*64+63 of that order, the first of them is the longest, and its
// length -- read off the histogram -- is the tile's number of rows.
__global__ void __launch_bounds__(1024) cursor_tiles_kernel(const int32_t* hist, int32_t max_len, int64_t n,
                                                             int32_t* cursor, int64_t* tile_base) {
  __shared__ int32_t cur[kMaxLen + 1];
  __shared__ int32_t cnt[kMaxLen + 1];
  __shared__ int64_t part[1024];
  __shared__ int64_t carry;
  const int tid = threadIdx.x;
  if (tid == 0) {
    int acc = 0;
    for (int L = max_len; L >= 0; --L) {
      cur[L] = acc;
      cursor[L] = acc;
      cnt[L] = hist[L];
      acc += hist[L];
    }
    carry = 0;
  }
  __syncthreads();
  if (!tile_base) return;
  const int64_t n_tiles = (n + kTile - 1) / kTile;
  for (int64_t c0 = 0; c0 < n_tiles; c0 += 1024) {
    const int64_t tau = c0 + tid;
    int64_t v = 0;
    if (tau < n_tiles) {
      const int64_t slot = tau * kTile;
      for (int L = max_len; L >= 0; --L)
        if (slot < int64_t(cur[L]) + cnt[L]) {
          v = int64_t(L) * kTile;
          break;
        }
    }
    part[tid] = v;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
      const int64_t add = tid >= d ? part[tid - d] : 0;
      __syncthreads();
      part[tid] += add;
      __syncthreads();
    }
    if (tau < n_tiles) tile_base[tau] = carry + part[tid] - v;
    __syncthreads();
    if (tid == 1023) carry += part[1023];
    __syncthreads();
  }
  if (tid == 0) tile_base[n_tiles] = carry;
}

// Slots of the length-sorted order: the block counts its tracks per length,
// reserves its places with one global atomic per length on the cursors, then
// hands them out through LDS atomics.  The order of tracks of equal length
// depends on scheduling; no result does (every track is fitted by its own
// lane with the same arithmetic, wherever it sits).
__global__ void __launch_bounds__(kSortBlock) length_scatter_kernel(const int32_t* off, int64_t n, int32_t max_len,
                                                                    int32_t* cursor, int32_t* order,
                                                                    int32_t* slot_of) {
  __shared__ int32_t h[kMaxLen + 1];
  __shared__ int32_t base[kMaxLen + 1];
  for (int i = threadIdx.x; i <= kMaxLen; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const int64_t b0 = int64_t(blockIdx.x) * kSortPerBlock;
  const int64_t b1 = b0 + kSortPerBlock < n ? b0 + kSortPerBlock : n;
  for (int64_t s0 = b0; s0 < b1; s0 += blockDim.x) {
    const int64_t t = s0 + threadIdx.x;
    if (t < b1) atomicAdd(&h[clamped_length(off, t, max_len)], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i <= kMaxLen; i += blockDim.x) {
    base[i] = h[i] ? atomicAdd(&cursor[i], h[i]) : 0;
    h[i] = 0;
  }
  __syncthreads();
  for (int64_t s0 = b0; s0 < b1; s0 += blockDim.x) {
    const int64_t t = s0 + threadIdx.x;
    if (t < b1) {
      const int len = clamped_length(off, t, max_len);
      const int slot = base[len] + atomicAdd(&h[len], 1);
      order[slot] = int32_t(t);
      slot_of[t] = slot;
    }
  }
}


// Fill the packed layout, one block per tile, through an LDS transpose: the
// tile's entries are read track by track (each track's entries are contiguous
// in the CSR arrays) into buffers [k][slot], then written row by row (entry k
// of the tile's 64 slots is contiguous in the packed layout).  The buffers
// hold `group` components at a time (sized by max_len), so that a typical
// tile needs two passes.  Entries beyond a track's length are never read by
// the fit and are left unwritten.
constexpr int kPackBlock = 256;
constexpr int kPackPer = (kTile * kMaxLen + kPackBlock - 1) / kPackBlock;   // entries per thread, at most
constexpr int kPackLds = 48 * 1024;                                         // dynamic LDS budget

template <typename T>
__global__ void __launch_bounds__(kPackBlock) pack_kernel(const int32_t* off, const int16_t* layer,
                                                          const uint8_t* valid, const T* pos, const T* cov,
                                                          int64_t n_hits, int64_t n, int32_t max_len, int32_t group,
                                                          const int32_t* order, const int64_t* tile_base, int32_t* lv,
                                                          T* hit, int64_t stride) {
  extern __shared__ __align__(16) unsigned char pack_smem[];
  __shared__ int32_t len_s[kTile];
  __shared__ int32_t pre_s[kTile + 1];   // exclusive prefix of the lengths
  __shared__ int64_t e0_s[kTile];
  const int cap = max_len * kTile;       // elements of one buffer
  int32_t* lbuf = reinterpret_cast<int32_t*>(pack_smem);
  T* buf = reinterpret_cast<T*>(pack_smem + ((cap * 4 + 15) / 16) * 16);
  const int64_t tile = blockIdx.x;
  const int tid = threadIdx.x;
  if (tid < kTile) {
    const int64_t slot = tile * kTile + tid;
    int len = 0;
    int64_t e0 = 0;
    if (slot < n) {
      const int64_t t = order[slot];
      e0 = off[t];
      len = int(off[t + 1] - e0);
      len = len < 0 ? 0 : (len > max_len ? max_len : len);
    }
    len_s[tid] = len;
    e0_s[tid] = e0;
  }
  __syncthreads();
  if (tid < kTile) {
    // exclusive prefix of the 64 lengths (wave-wide, in LDS)
    int acc = 0;
    for (int j = 0; j < tid; ++j) acc += len_s[j];
    pre_s[tid] = acc;
    if (tid == kTile - 1) pre_s[kTile] = acc + len_s[tid];
  }
  __syncthreads();
  const int total = pre_s[kTile];
  const int rows = len_s[0];   // the longest track leads its tile
  int64_t src[kPackPer];
  int dst[kPackPer];   // k * kTile + slot, or -1
#pragma unroll
  for (int m = 0; m < kPackPer; ++m) {
    const int f = tid + m * kPackBlock;
    src[m] = 0;
    dst[m] = -1;
    if (f < total) {
      int lo = 0, hi = kTile;   // pre_s[lo] <= f < pre_s[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre_s[mid] <= f) lo = mid;
        else hi = mid;
      }
      const int k = f - pre_s[lo];
      src[m] = e0_s[lo] + k;
      dst[m] = k * kTile + lo;
    }
  }
  const int64_t base = tile_base[tile];
  for (int c0 = 0; c0 < 9; c0 += group) {
    const int gn = c0 + group <= 9 ? group : 9 - c0;
#pragma unroll
    for (int m = 0; m < kPackPer; ++m) {
      if (dst[m] < 0) continue;
      if (c0 == 0) lbuf[dst[m]] = int32_t(uint16_t(layer[src[m]])) | (int32_t(valid[src[m]] != 0) << 16);
      for (int g = 0; g < gn; ++g) {
        const int c = c0 + g;
        const T* srcc = c < 3 ? pos + int64_t(c) * n_hits : cov + int64_t(c - 3) * n_hits;
        buf[g * cap + dst[m]] = srcc[src[m]];
      }
    }
    __syncthreads();
    for (int i = tid; i < rows * kTile; i += kPackBlock) {
      if (i / kTile >= len_s[i % kTile]) continue;
      if (c0 == 0) lv[base + i] = lbuf[i];
      for (int g = 0; g < gn; ++g) hit[int64_t(c0 + g) * stride + base + i] = buf[g * cap + i];
    }
    __syncthreads();
  }
}

template <typename T>
hipError_t launch_pack(const FitArgs<T>& a, const PackWork& w, int layout, PackedHits<T>* out, hipStream_t s) {
  const int B = 256;
  const int nh = kMaxLen + 2;
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(128), 0, s, w.hist, nh);
  const unsigned sort_grid = unsigned((a.n + kSortPerBlock - 1) / kSortPerBlock);
  hipLaunchKernelGGL(length_hist_kernel, dim3(sort_grid), dim3(kSortBlock), 0, s, a.hit_offsets, a.n, a.max_len,
                     w.hist);
  hipLaunchKernelGGL(cursor_tiles_kernel, dim3(1), dim3(1024), 0, s, w.hist, a.max_len, a.n, w.cursor,
                     layout == 2 ? w.tile_base : nullptr);
  hipLaunchKernelGGL(length_scatter_kernel, dim3(sort_grid), dim3(kSortBlock), 0, s, a.hit_offsets, a.n,
                     a.max_len, w.cursor, w.order, w.slot_of);
  out->order = w.order;
  out->tile_base = nullptr;
  out->lv = nullptr;
  out->hit = nullptr;
  out->stride = 0;
  if (layout == 2) {
    const unsigned n_tiles = unsigned((a.n + kTile - 1) / kTile);
    // components per pass: as many [max_len][64] buffers as the LDS budget holds
    const int cap = a.max_len * kTile;
    const int lbytes = ((cap * 4 + 15) / 16) * 16;
    int group = (kPackLds - lbytes) / (cap * int(sizeof(T)));
    group = group < 1 ? 1 : (group > 9 ? 9 : group);
    const size_t smem = size_t(lbytes) + size_t(group) * cap * sizeof(T);
    if (a.n_hits > 0)
      hipLaunchKernelGGL(pack_kernel<T>, dim3(n_tiles), dim3(kPackBlock), smem, s, a.hit_offsets, a.hit_layer,
                         a.hit_valid, a.hit_pos, a.hit_cov, a.n_hits, a.n, a.max_len, group, w.order, w.tile_base,
                         w.lv, (T*)w.hit, w.cap);
    out->tile_base = w.tile_base;
    out->lv = w.lv;
    out->hit = (const T*)w.hit;
    out->stride = w.cap;
  }
  return hipGetLastError();
}

template <typename T, int WAVES, int LAYOUT>
hipError_t launch_fit_w(const FitArgs<T>& a, const GeomArgs& g, const FitLaunch& l, int n_cu, hipStream_t s) {
  const int block = l.block;
  if (!l.persistent) {
    const int64_t grid = (a.n + block - 1) / block;
    if constexpr (LAYOUT >= 3)
      hipLaunchKernelGGL((fit_staged_kernel<T, WAVES, LAYOUT == 4>), dim3(unsigned(grid)), dim3(block), 0, s, a, g);
    else
      hipLaunchKernelGGL((fit_kernel<T, WAVES, LAYOUT>), dim3(unsigned(grid)), dim3(block), 0, s, a, g);
    return hipGetLastError();
  }
  FitArgs<T> b = a;
  b.n_tiles = (a.n + block - 1) / block;
  int64_t grid = int64_t(n_cu) * l.blocks_per_cu;
  if (grid > b.n_tiles) grid = b.n_tiles;
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, s, a.tile_counter);
  if constexpr (LAYOUT >= 3)
    hipLaunchKernelGGL((fit_staged_persistent_kernel<T, WAVES, LAYOUT == 4>), dim3(unsigned(grid)), dim3(block), 0,
                       s, b, g);
  else
    hipLaunchKernelGGL((fit_persistent_kernel<T, WAVES, LAYOUT>), dim3(unsigned(grid)), dim3(block), 0, s, b, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fit(const FitArgs<T>& a, const GeomArgs& g, const FitLaunch& l, int n_cu, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  if (a.packed == 4) return l.waves == 2 ? launch_fit_w<T, 2, 4>(a, g, l, n_cu, s) : launch_fit_w<T, 1, 4>(a, g, l, n_cu, s);
  if (a.packed == 3) return l.waves == 2 ? launch_fit_w<T, 2, 3>(a, g, l, n_cu, s) : launch_fit_w<T, 1, 3>(a, g, l, n_cu, s);
  if (a.packed == 2) return l.waves == 2 ? launch_fit_w<T, 2, 2>(a, g, l, n_cu, s) : launch_fit_w<T, 1, 2>(a, g, l, n_cu, s);
  if (a.packed == 1) return l.waves == 2 ? launch_fit_w<T, 2, 1>(a, g, l, n_cu, s) : launch_fit_w<T, 1, 1>(a, g, l, n_cu, s);
  return l.waves == 2 ? launch_fit_w<T, 2, 0>(a, g, l, n_cu, s) : launch_fit_w<T, 1, 0>(a, g, l, n_cu, s);
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
template hipError_t launch_pack<float>(const FitArgs<float>&, const PackWork&, int, PackedHits<float>*, hipStream_t);
template hipError_t launch_pack<double>(const FitArgs<double>&, const PackWork&, int, PackedHits<double>*, hipStream_t);

}  // namespace kf
