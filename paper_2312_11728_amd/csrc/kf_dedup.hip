// Duplicate removal among found tracks (one track per seed, one hit id per
// layer of the plan).  Tracks t and u are duplicates when they carry the same
// hit id at >= 1 layer and at >= frac * min(n_t, n_u) layers (n: hit count);
// u outranks t on (score, then lower index); t is removed when an outranking
// track is its duplicate, and dup_of[t] names the highest-ranked one.
//
// The candidate partners of a track are the tracks that share one of its hit
// ids: the (hit id, track) pairs of all tracks are sorted by hit id (radix
// sort).  One thread per (track, layer) finds its hit id's run of pairs by
// binary search and compares its track's hit list with each outranking
// partner's, layer by layer; the highest-ranked duplicate of a track is the
// minimum of a 64-bit rank key over its layers (atomic min).
#include <hipcub/hipcub.hpp>

#include "kf_dedup.hpp"

namespace kf {

namespace {

constexpr uint32_t kNoKey = 0xffffffffu;   // after every hit id (ids are < 2^31)

__device__ inline bool has_candidate(float s) { return s > -__builtin_huge_valf(); }

// Pair (hit id, track) of entry i = t * n_layers + l; the entries of a track
// without a candidate and the misses sort last.  Also resets the track's
// best-duplicate key.
__global__ void dedup_pairs_kernel(DedupArgs a, uint32_t* keys, int32_t* vals, unsigned long long* best) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t m = a.n * a.n_layers;
  if (i >= m) return;
  const int64_t t = i / a.n_layers;
  const int l = int(i - t * a.n_layers);
  const int32_t h = a.hits[t * a.hit_stride + l];
  const bool has = h >= 0 && has_candidate(a.score[t * a.score_stride]);
  keys[i] = has ? uint32_t(h) : kNoKey;
  vals[i] = has ? int32_t(t) : -1;
  if (l == 0) best[t] = ~0ull;
}

// The rank of track u as an unsigned key: smaller is higher ranked (score
// descending, then index ascending); -0 and +0 rank alike.
__device__ inline unsigned long long rank_key(float s, int64_t u) {
  if (s == 0.0f) s = 0.0f;
  const uint32_t b = __float_as_uint(s);
  const uint32_t ord = (b & 0x80000000u) ? ~b : (b | 0x80000000u);   // increasing with s
  return (static_cast<unsigned long long>(~ord) << 32) | static_cast<uint32_t>(u);
}

// Entry (t, l): the tracks carrying t's hit id at l that outrank t and are
// its duplicates; the highest-ranked of them goes to best[t] (atomic min).
__global__ void dedup_scan_kernel(DedupArgs a, const uint32_t* keys, const int32_t* vals, int64_t m,
                                  unsigned long long* best) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int L = a.n_layers;
  const int64_t t = i / L;
  const int l = int(i - t * L);
  const int32_t* ht = a.hits + t * a.hit_stride;
  const int32_t h = ht[l];
  const float st = a.score[t * a.score_stride];
  if (h < 0 || !has_candidate(st)) return;
  // first pair with key h
  int64_t lo = 0, hi = m;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < uint32_t(h)) lo = mid + 1; else hi = mid;
  }
  int nt = -1;
  unsigned long long mine = ~0ull;
  for (int64_t j = lo; j < m && keys[j] == uint32_t(h); ++j) {
    const int64_t u = vals[j];
    if (u == t) continue;
    const float su = a.score[u * a.score_stride];
    if (!(su > st || (su == st && u < t))) continue;   // u does not outrank t
    const unsigned long long ku = rank_key(su, u);
    if (ku >= mine) continue;   // ranks below a duplicate found already
    if (nt < 0) {
      nt = 0;
      for (int k = 0; k < L; ++k) nt += ht[k] >= 0 ? 1 : 0;
    }
    const int32_t* hu = a.hits + u * a.hit_stride;
    int nu = 0, shared = 0;
    for (int k = 0; k < L; ++k) {
      const int32_t x = hu[k];
      nu += x >= 0 ? 1 : 0;
      shared += (x >= 0 && x == ht[k]) ? 1 : 0;
    }
    const int nmin = nt < nu ? nt : nu;
    // exact: a float times an integer <= 64 is exact in double
    if (shared >= 1 && double(shared) >= double(a.frac) * double(nmin)) mine = ku;
  }
  if (mine != ~0ull) atomicMin(&best[t], mine);
}

__global__ void dedup_finish_kernel(DedupArgs a, const unsigned long long* best) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= a.n) return;
  const bool has = has_candidate(a.score[t * a.score_stride]);
  const unsigned long long b = best[t];
  a.keep[t] = (has && b == ~0ull) ? 1 : 0;
  if (a.dup_of) a.dup_of[t] = (has && b != ~0ull) ? int32_t(uint32_t(b)) : -1;
}

size_t sort_temp_bytes(int64_t m) {
  size_t bytes = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, static_cast<const uint32_t*>(nullptr),
                                         static_cast<uint32_t*>(nullptr), static_cast<const int32_t*>(nullptr),
                                         static_cast<int32_t*>(nullptr), int(m), 0, 32) != hipSuccess)
    return 0;
  return bytes;
}

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

size_t dedup_workspace_bytes(int64_t n, int32_t n_layers) {
  const int64_t m = n * n_layers;
  return 4 * up256(size_t(m) * 4) + up256(size_t(n) * 8) + up256(sort_temp_bytes(m));
}

hipError_t launch_dedup(const DedupArgs& a, void* work, size_t work_bytes, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  const int64_t m = a.n * a.n_layers;
  if (work_bytes < dedup_workspace_bytes(a.n, a.n_layers)) return hipErrorInvalidValue;
  char* p = static_cast<char*>(work);
  uint32_t* k_in = reinterpret_cast<uint32_t*>(p);
  p += up256(size_t(m) * 4);
  uint32_t* k_out = reinterpret_cast<uint32_t*>(p);
  p += up256(size_t(m) * 4);
  int32_t* v_in = reinterpret_cast<int32_t*>(p);
  p += up256(size_t(m) * 4);
  int32_t* v_out = reinterpret_cast<int32_t*>(p);
  p += up256(size_t(m) * 4);
  unsigned long long* best = reinterpret_cast<unsigned long long*>(p);
  p += up256(size_t(a.n) * 8);
  size_t temp = sort_temp_bytes(m);
  const unsigned gm = unsigned((m + 255) / 256), gn = unsigned((a.n + 255) / 256);
  hipLaunchKernelGGL(dedup_pairs_kernel, dim3(gm), dim3(256), 0, s, a, k_in, v_in, best);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipcub::DeviceRadixSort::SortPairs(p, temp, k_in, k_out, v_in, v_out, int(m), 0, 32, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dedup_scan_kernel, dim3(gm), dim3(256), 0, s, a, k_out, v_out, m, best);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dedup_finish_kernel, dim3(gn), dim3(256), 0, s, a, best);
  return hipGetLastError();
}

}  // namespace kf
