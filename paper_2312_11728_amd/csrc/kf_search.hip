// HIP kernels of the combinatorial candidate search: binning of the hit pool
// by (layer, phi, z), then the search itself in one launch (one thread per
// candidate slot, one wave per block; per layer of the plan the selection,
// the extend with its window scan, and at the end the final pass that writes
// the kept candidates).
#include "kf_kernels.hpp"
#include "kf_search.hpp"
#include "kf_search_launch.hpp"

namespace kf {

// ---- binning -------------------------------------------------------------------

__global__ void __launch_bounds__(256) fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}

__device__ __forceinline__ int layer_of_hit(const BinTable& t, int32_t h) {
  int lo = 0, hi = t.n_layers;   // off[lo] <= h < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (t.off[mid] <= h) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int32_t bin_of_hit(const BinTable& t, int L, float x, float y, float z) {
  const float phi = atan2f(y, x);
  return t.base[L] + phi_bin(phi, t.nphi[L]) * t.nz[L] + z_bin(z, t.lo[L], t.hi[L], t.nz[L]);
}

// count hits per bin; each hit keeps its rank inside its bin
__global__ void __launch_bounds__(256) bin_count_kernel(BinTable t, const float* pos, int64_t n, int32_t* count,
                                                        int32_t* bin_of, int32_t* rank) {
  const int64_t h = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (h >= n) return;
  const int L = layer_of_hit(t, int32_t(h));
  const int32_t b = bin_of_hit(t, L, pos[h], pos[n + h], pos[2 * n + h]);
  bin_of[h] = b;
  rank[h] = atomicAdd(&count[b], 1);
}

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;   // per thread

// exclusive scan of counts[0..n) into off, block by block; block totals out
__global__ void __launch_bounds__(kScanBlock) scan_blocks_kernel(const int32_t* in, int64_t n, int32_t* out,
                                                                 int32_t* block_sum) {
  __shared__ int32_t s[kScanBlock];
  const int64_t base = int64_t(blockIdx.x) * kScanBlock * kScanItems + int64_t(threadIdx.x) * kScanItems;
  int32_t v[kScanItems];
  int32_t tot = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0;
    tot += v[k];
  }
  s[threadIdx.x] = tot;
  __syncthreads();
  for (int o = 1; o < kScanBlock; o <<= 1) {
    const int32_t add = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += add;
    __syncthreads();
  }
  int32_t run = s[threadIdx.x] - tot;   // exclusive prefix of this thread
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == kScanBlock - 1) block_sum[blockIdx.x] = s[threadIdx.x];
}

// exclusive scan of the block totals (one block, chunks with a carry);
// total[0] = grand total
__global__ void __launch_bounds__(1024) scan_sums_kernel(int32_t* sums, int64_t nb, int32_t* total) {
  __shared__ int32_t s[1024];
  __shared__ int32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t c0 = 0; c0 < nb; c0 += 1024) {
    const int64_t i = c0 + threadIdx.x;
    const int32_t v = i < nb ? sums[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int32_t add = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
      __syncthreads();
      s[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nb) sums[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) total[0] = carry;
}

__global__ void __launch_bounds__(256) scan_add_kernel(int32_t* out, int64_t n, const int32_t* sums,
                                                       const int32_t* total) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] += sums[i / (kScanBlock * kScanItems)];
  if (i == n) out[n] = total[0];
}

// copy every hit to its binned position (x, y, z, phi, covariance, id,
// module: three 16-byte stores)
__global__ void __launch_bounds__(256) bin_scatter_kernel(BinTable t, const float* pos, const float* cov,
                                                          const int32_t* id, const int32_t* module, int64_t n,
                                                          const int32_t* bin_off, const int32_t* bin_of,
                                                          const int32_t* rank, PoolBins o) {
  const int64_t h = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (h >= n) return;
  const int64_t d = int64_t(bin_off[bin_of[h]]) + rank[h];
  const float x = pos[h], y = pos[n + h];
  float4* dst = reinterpret_cast<float4*>(o.hits + d);
  dst[0] = make_float4(x, y, pos[2 * n + h], atan2f(y, x));
  dst[1] = make_float4(cov[h], cov[n + h], cov[2 * n + h], cov[3 * n + h]);
  dst[2] = make_float4(cov[4 * n + h], cov[5 * n + h], __int_as_float(id[h]), __int_as_float(module ? module[h] : -1));
}

// ---- search ------------------------------------------------------------------

// The whole search in one launch.  Block b owns the seeds [b * spb,
// (b + 1) * spb), spb = blockDim.x / beam, and their slots: thread i <
// spb * beam is slot b * spb * beam + i.  At every layer the slot first
// runs the previous layer's selection for itself (its candidate and that
// candidate's state, read from its seed's slots in LDS), then, after a
// block barrier, its extend, which leaves its child list and the state it
// goes on with in LDS for the next selection; a second barrier closes the
// layer.  After the last layer come the last selection and the final pass.
// A seed's slots exchange data only with each other, so blocks never wait
// for one another: each runs its seeds through the layers at its own pace.
// B: a compile-time bound on beam (2, 4, 6 or 8), the size of the child
// lists held in registers and LDS.
template <int B>
__global__ void __launch_bounds__(kSearchBlock, kSearchWaves) search_kernel(SearchArgs a,
                                                                          const SearchLayer* __restrict__ layers) {
  __shared__ SlotExchange<B> X;
  const int spb = kSearchBlock / a.beam;
  const int i = int(threadIdx.x);
  const int64_t seed0 = int64_t(blockIdx.x) * spb;
  const int64_t s = seed0 * a.beam + i;
  const int64_t t = seed0 + i;
  const bool slot = i < spb * a.beam && s < a.n * a.beam;
  // the seeds' status words collect the bits of their slots' steps
  if (i < spb && t < a.n) a.status[t] = 0u;
  __syncthreads();
  Cand k;
  k.live = false;
  for (int step = 0; step < a.plan_len; ++step) {
    if (slot) {
      if (step == 0)
        seed_candidate(a, s, k);
      else
        select_slot<B>(a, X, step - 1, s, i, k);
    }
    __syncthreads();
    const SearchLayer& L = layers[step];
    uint32_t st = 0;
    float score = 0.f;
    ScanWindow w;
    w.scan = false;
    const bool open = slot && extend_open<B>(a, X, L, layers[step > 0 ? step - 1 : 0], step, s, i, k, score, w, st);
    Kids<B> K;
    kids_init(K);
    scan_window<B>(a, L, w, k.p, k.c, score, K, st);
    if (open) extend_close<B>(a, X, i, k, score, K);
    if (st) atomicOr(&a.status[s / a.beam], st);
    __syncthreads();
  }
  if (slot) select_slot<B>(a, X, a.plan_len - 1, s, i, k);
  __syncthreads();
  if (slot) {
    const uint32_t st = finish_candidate(a, layers[a.plan_len - 1], s, k);
    if (st) atomicOr(&a.status[s / a.beam], st);
  }
}

static unsigned blocks(int64_t n, int b) { return unsigned((n + b - 1) / b); }

hipError_t launch_bin_pool(const BinTable& t, const float* pos, const float* cov, const int32_t* id,
                           const int32_t* module, int64_t n, int64_t n_bins, const SearchWork& w, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1024), dim3(256), 0, s, w.count, n_bins, 0);
  if (n > 0)
    hipLaunchKernelGGL(bin_count_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, t, pos, n, w.count, w.bin_of,
                       w.rank);
  const int64_t nb = (n_bins + kScanBlock * kScanItems - 1) / (kScanBlock * kScanItems);
  hipLaunchKernelGGL(scan_blocks_kernel, dim3(unsigned(nb)), dim3(kScanBlock), 0, s, w.count, n_bins,
                     w.pool.bin_off, w.block_sum);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, s, w.block_sum, nb, w.total);
  hipLaunchKernelGGL(scan_add_kernel, dim3(blocks(n_bins + 1, 256)), dim3(256), 0, s, w.pool.bin_off, n_bins,
                     w.block_sum, w.total);
  if (n > 0)
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(blocks(n, 256)), dim3(256), 0, s, t, pos, cov, id, module, n,
                       w.pool.bin_off, w.bin_of, w.rank, w.pool);
  return hipGetLastError();
}

hipError_t launch_search(SearchArgs a, const SearchLayer* layers, SearchLayer* d_layers, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(d_layers, layers, size_t(a.plan_len) * sizeof(SearchLayer), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return e;
  const int spb = kSearchBlock / a.beam;
  const dim3 grid(blocks(a.n, spb)), block(kSearchBlock);
  const SearchLayer* L = d_layers;
  if (a.beam <= 2)
    hipLaunchKernelGGL(search_kernel<2>, grid, block, 0, s, a, L);
  else if (a.beam <= 4)
    hipLaunchKernelGGL(search_kernel<4>, grid, block, 0, s, a, L);
  else if (a.beam <= 6)
    hipLaunchKernelGGL(search_kernel<6>, grid, block, 0, s, a, L);
  else
    hipLaunchKernelGGL(search_kernel<kMaxBeam>, grid, block, 0, s, a, L);
  return hipGetLastError();
}

}  // namespace kf
