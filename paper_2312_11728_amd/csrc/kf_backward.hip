// HIP kernel of the backward fit: every track is traversed again from its last
// entry down to its first valid entry and refitted, starting from the forward
// fit's result with its covariance scaled up and the direction of motion
// reversed, so that the forward step (propagation, material, update) runs
// unchanged on the reversed entry list.  One track per lane; the entries of a
// wave's 64 tracks are staged through LDS a few at a time, as in the forward
// fit.
#include "kf_backward.hpp"
#include "kf_kernels.hpp"
#include "kf_stage.hpp"
#include "kf_track.hpp"

// waves per SIMD that the register allocation of the smoother's combination
// and of the final fit's chi2 kernel must allow
#ifndef KF_SMOOTH_WAVES
#define KF_SMOOTH_WAVES 2
#endif
#ifndef KF_FINAL_CHI2_WAVES
#define KF_FINAL_CHI2_WAVES 2
#endif

namespace kf {

namespace {

constexpr int kBwdBlock = 256;

// Two estimates of one state on a surface, from disjoint sets of hits,
// combined (two-filter smoother): with the gain K = C_f (C_f + C_b)^+,
// x = x_f + K (x_b - x_f) and C = (I - K) C_f (I - K)^T + K C_b K^T (equal to
// C_f - C_f (C_f + C_b)^+ C_f, without its cancellation where C_f is much
// larger than the result).  ^+ inverts on the 5 directions the state can
// move in (the surface normal is a null vector of both): the frame
// (u, w, ipt, phi, theta) with u, w the unit position directions along the
// surface (barrel: the tangent (-y, x)/R and z; disk: x and y), so
// K = C_f B (B^T (C_f + C_b) B)^-1 B^T.  The 5x5 system is solved by
// Cholesky in FP64, with divisions only on its 5 pivots.  Returns false
// (outputs untouched) when it is not positive definite.
template <typename T>
__device__ inline bool combine_on_surface(const T pf[6], const T cf[21], const T pb[6], const T cb[21], int kind,
                                          T pos, T ps[6], T cs[21]) {
  double u[3], w[3];
  if (kind == 1) {
    u[0] = 1.0; u[1] = 0.0; u[2] = 0.0;
    w[0] = 0.0; w[1] = 1.0; w[2] = 0.0;
  } else {
    const double ri = 1.0 / double(pos);
    u[0] = -double(pf[1]) * ri; u[1] = double(pf[0]) * ri; u[2] = 0.0;
    w[0] = 0.0; w[1] = 0.0; w[2] = 1.0;
  }
  // S = C_f + C_b; G = C_f B (6 x 5); M = B^T S B (5 x 5, packed)
  double S[21];
#pragma unroll
  for (int i = 0; i < 21; ++i) S[i] = double(cf[i]) + double(cb[i]);
  double G[6][5];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double gu = 0.0, gw = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gu += double(cf[sym(i, k)]) * u[k];
      gw += double(cf[sym(i, k)]) * w[k];
    }
    G[i][0] = gu;
    G[i][1] = gw;
#pragma unroll
    for (int k = 0; k < 3; ++k) G[i][2 + k] = double(cf[sym(i, 3 + k)]);
  }
  double Su[6], Sw[6];   // S u, S w over the position block
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    Su[i] = 0.0;
    Sw[i] = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Su[i] += S[sym(i, k)] * u[k];
      Sw[i] += S[sym(i, k)] * w[k];
    }
  }
  double M[5][5];
  M[0][0] = u[0] * Su[0] + u[1] * Su[1] + u[2] * Su[2];
  M[1][0] = w[0] * Su[0] + w[1] * Su[1] + w[2] * Su[2];
  M[1][1] = w[0] * Sw[0] + w[1] * Sw[1] + w[2] * Sw[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    M[2 + k][0] = Su[3 + k];
    M[2 + k][1] = Sw[3 + k];
#pragma unroll
    for (int l = 0; l <= k; ++l) M[2 + k][2 + l] = S[sym(3 + k, 3 + l)];
  }
  // Cholesky M = L L^T (lower triangle in place), inverse pivots kept
  double il[5];
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    double dj = M[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) dj -= M[j][k] * M[j][k];
    if (!(dj > 0.0)) return false;
    il[j] = 1.0 / sqrt(dj);
#pragma unroll
    for (int i = j + 1; i < 5; ++i) {
      double v = M[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= M[i][k] * M[j][k];
      M[i][j] = v * il[j];
    }
  }
  // W = G M^-1 (each row of G solved in place), then the gain K = W B^T
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      double v = G[i][a];
#pragma unroll
      for (int k = 0; k < a; ++k) v -= M[a][k] * G[i][k];
      G[i][a] = v * il[a];
    }
#pragma unroll
    for (int a = 4; a >= 0; --a) {
      double v = G[i][a];
#pragma unroll
      for (int k = a + 1; k < 5; ++k) v -= M[k][a] * G[i][k];
      G[i][a] = v * il[a];
    }
  }
  double K[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int k = 0; k < 3; ++k) K[i][k] = G[i][0] * u[k] + G[i][1] * w[k];
#pragma unroll
    for (int l = 0; l < 3; ++l) K[i][3 + l] = G[i][2 + l];
  }
  // x = x_f + K (x_b - x_f)
  double d[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) d[i] = double(pb[i]) - double(pf[i]);
  d[4] = wrap_phi(d[4]);
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double v = double(pf[i]);
#pragma unroll
    for (int k = 0; k < 6; ++k) v += K[i][k] * d[k];
    ps[i] = T(v);
  }
  ps[4] = wrap_phi(ps[4]);
  // C = (I - K) C_f (I - K)^T + K C_b K^T, row by row: with t1 = row i of
  // (I - K) C_f and t2 = row i of K C_b, C_ij = t1_j - t1 . K_j + t2 . K_j
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double t1[6], t2[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double a1 = double(cf[sym(i, j)]), a2 = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        a1 -= K[i][k] * double(cf[sym(k, j)]);
        a2 += K[i][k] * double(cb[sym(k, j)]);
      }
      t1[j] = a1;
      t2[j] = a2;
    }
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double v = t1[j];
#pragma unroll
      for (int k = 0; k < 6; ++k) v += (t2[k] - t1[k]) * K[j][k];
      cs[sym(i, j)] = T(v);
    }
  }
  return true;
}

// The backward prediction at an entry, turned outward (phi - pi, pi - theta;
// the theta terms of the covariance change sign), stored in the smoothed-state
// arrays as propagate() hands it over, before the layer's material.
template <typename T>
struct StorePrediction {
  T* so;
  T* co;
  int64_t os;
  KF_HD void operator()(const T* p, const T* c) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) so[i * os] = p[i];
    so[4 * os] = wrap_phi(p[4] + T(kPi));
    so[5 * os] = T(kPi) - p[5];
#pragma unroll
    for (int i = 0; i < 21; ++i) co[i * os] = (i >= 15 && i < 20) ? -c[i] : c[i];
  }
};

// One step of the smoothing backward pass (backward index k >= 1, entry r of
// the track): the step of the plain backward pass, with the backward
// prediction stored on the way (the combination with the forward filtered
// state is a separate, entry-parallel pass: smooth_combine_kernel).  The rest
// as in fit_entry (layer check, backup, roll-back of a non-finite step).
template <typename T>
__device__ inline bool smooth_step(const BwdArgs<T>& b, const TrackGeom<T>& g, int64_t t, int k, int r, int lay,
                                   int& prev, bool valid, const T m[3], const T V[6], T p[6], T c[21], int& q,
                                   uint32_t& st, T& chi2, int& nval, T* bk, int bk_stride) {
  const FitArgs<T>& a = b.f;
  if (lay < 0 || lay >= g.n_layers) {
    st |= TRK_BAD_INPUT;
    return false;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) bk[i * bk_stride] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) bk[(6 + i) * bk_stride] = c[i];
  const int qq = q;
  uint32_t sst = 0;
  const int kind = g.kind[lay];
  const int64_t at = int64_t(r) * a.ld + t;
  const StorePrediction<T> store{b.smooth_state + at, b.smooth_cov + at, a.ld * int64_t(a.max_len)};
  if (k == 0) {
    add_material_here(p, c, kind, g.x0[lay], g.mass, sst);   // the first entry: its prediction is the input
  } else if (!propagate(p, c, q, kind, g.pos[lay], g.x0[lay], lay == prev, true, g.bz, g.mass, sst,
                        static_cast<T*>(nullptr), static_cast<PropTape<T>*>(nullptr), store)) {
    st |= sst;
    return false;
  }
  T c2 = T(0);
  if (valid) {
    T mm[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) mm[i] = m[i];
    update(p, c, q, mm, V, c2, sst);
  }
  if (!all_finite(p, c, c2)) {
    st |= sst | TRK_NONFINITE;
#pragma unroll
    for (int i = 0; i < 6; ++i) p[i] = bk[i * bk_stride];
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = bk[(6 + i) * bk_stride];
    q = qq;
    return false;
  }
  st |= sst;
  chi2 += c2;
  nval += valid ? 1 : 0;
  prev = lay;
  return true;
}

// Smoothing, entry-parallel: thread (r, t) combines the backward prediction
// stored at entry r of track t with the forward filtered state of that entry
// (forward checkpoint slot r - k0) and overwrites it with the smoothed state.
// Entries from the first valid one to the last but one of refitted tracks
// whose prediction is finite; the last entry already holds its filtered state.
template <typename T>
__global__ void __launch_bounds__(256, KF_SMOOTH_WAVES) smooth_combine_kernel(BwdArgs<T> b, GeomArgs g) {
  const FitArgs<T>& a = b.f;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = int(blockIdx.y);
  if (t >= a.n) return;
  if (a.trk_status[t] & TRK_BAD_INPUT) return;   // not refitted
  const int64_t e0 = a.hit_offsets[t];
  int n_e = int(a.hit_offsets[t + 1] - e0);
  if (n_e > a.max_len) n_e = a.max_len;
  if (r >= n_e - 1) return;
  int k0 = 0;
  while (k0 <= r && a.hit_valid[e0 + k0] == 0) ++k0;
  if (r < k0) return;
  const int64_t os = a.ld * int64_t(a.max_len), at = int64_t(r) * a.ld + t;
  T* so = b.smooth_state + at;
  T* co = b.smooth_cov + at;
  T pb[6], cb[21];
#pragma unroll
  for (int i = 0; i < 6; ++i) pb[i] = so[i * os];
  if (!(pb[0] == pb[0])) return;   // NaN: the backward pass stopped before this entry
#pragma unroll
  for (int i = 0; i < 21; ++i) cb[i] = co[i * os];
  const int64_t cst = a.ld * int64_t(b.n_seg_f);
  const T* f = b.fwd_ckpt + int64_t(r - k0) * a.ld + t;
  T pf[6], cf[21];
#pragma unroll
  for (int i = 0; i < 6; ++i) pf[i] = f[i * cst];
#pragma unroll
  for (int i = 0; i < 21; ++i) cf[i] = f[(6 + i) * cst];
  const int lay = a.hit_layer[e0 + r];
  if (lay < 0 || lay >= g.n_layers) return;
  T ps[6], cs[21];
  if (combine_on_surface(pf, cf, pb, cb, int(g.kind[lay]), T(g.pos[lay]), ps, cs)) {
#pragma unroll
    for (int i = 0; i < 6; ++i) so[i * os] = ps[i];
#pragma unroll
    for (int i = 0; i < 21; ++i) co[i * os] = cs[i];
  } else {
    so[0] = k_nan<T>();
    atomicOr(&a.trk_status[t], uint32_t(TRK_COV_NOT_PSD));
  }
}

// Backward fit of tracks [w0, w0 + 64) (one wave; every lane must call it).
// Entry k of a track's backward pass is CSR entry last - k; the pass has
// n_entries - k0 entries (k0: the first valid entry in crossing order).
// MODE: kPlain (the backward fit), kSmooth (the backward pass of the
// smoother).
constexpr int kPlain = 0, kSmooth = 1;

template <typename T, int J, int MODE>
__device__ void backward_wave_staged(const BwdArgs<T>& b, const TrackGeom<T>& g, int64_t w0, StageBuf<T, J>& sb,
                                     T* bk, int bk_stride) {
  constexpr bool SMOOTH = MODE == kSmooth;
  const FitArgs<T>& a = b.f;
  const int lane = int(threadIdx.x) & 63;
  const int64_t t = w0 + lane;
  const bool in_range = t < a.n;
  int64_t last = 0;
  int len = 0, n_e = 0, k0 = 0;
  T p[6], c[21];
  int q = 0;
  uint32_t st = 0;
  bool run = false;
  if (in_range) {
    const int64_t e0 = a.hit_offsets[t];
    n_e = int(a.hit_offsets[t + 1] - e0);
    if (n_e > a.max_len) n_e = a.max_len;
#pragma unroll
    for (int i = 0; i < 6; ++i) p[i] = a.seed_state[i * a.ld + t];
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = a.seed_cov[i * a.ld + t];
    q = a.seed_charge[t];
    while (k0 < n_e && a.hit_valid[e0 + k0] == 0) ++k0;
    const uint32_t stop = TRK_NO_CROSSING | TRK_NONFINITE | TRK_BAD_INPUT;
    run = k0 < n_e && !(b.fwd_status && (b.fwd_status[t] & stop));
    if (run) {
      last = e0 + n_e - 1;
      len = n_e - k0;
      if constexpr (SMOOTH) {
        // the last entry's smoothed state is its forward filtered state: the input
        const int64_t os = a.ld * int64_t(a.max_len), at = int64_t(n_e - 1) * a.ld + t;
#pragma unroll
        for (int i = 0; i < 6; ++i) b.smooth_state[i * os + at] = p[i];
#pragma unroll
        for (int i = 0; i < 21; ++i) b.smooth_cov[i * os + at] = c[i];
      }
#pragma unroll
      for (int i = 0; i < 21; ++i) c[i] *= b.cov_scale;
      // the surface of the last entry's layer, imposed again: scaled up, the
      // rounding residue of the stored covariance along its normal would no
      // longer be negligible (a bad layer id is caught by the first step)
      const int ll = a.hit_layer[last];
      if (ll >= 0 && ll < g.n_layers) impose_surface(c, p, g.kind[ll], g.pos[ll]);
      reverse_direction(p, c, q);
    } else {
      st = TRK_BAD_INPUT;   // not refitted: the input is returned
    }
  }
  sb.e0[lane] = last;
  sb.len[lane] = len;
  const int kmax = wave_max(len);
  T chi2 = T(0);
  int nval = 0, prev = 0;
  bool live = run;
  const int64_t nh = a.n_hits;
  wave_sync();
  for (int j0 = 0; j0 < kmax; j0 += J) {
    // all J rows are loaded before any is written to LDS (one memory round
    // trip per chunk); a slot past the end of its pass loads the pass's last
    // entry (the track's first valid one) and is never read; kmax > 0 means
    // some track has an entry, so entry 0 exists for the slots of no track
    int32_t lvr[J];
    T vr[J][9];
#pragma unroll
    for (int r = 0; r < J; ++r) {
      const int idx = r * 64 + lane;
      const int l = idx / J, jj = idx % J;
      const int ln = sb.len[l];
      const int64_t e = ln > 0 ? sb.e0[l] - min(j0 + jj, ln - 1) : 0;
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
      if (k == 0) prev = lay;
      T m[3], V[6];
#pragma unroll
      for (int x = 0; x < 3; ++x) m[x] = sb.v[x][jj][lane];
#pragma unroll
      for (int x = 0; x < 6; ++x) V[x] = sb.v[3 + x][jj][lane];
      const int r = n_e - 1 - k;   // entry index within the track
      if (SMOOTH)
        live = smooth_step(b, g, t, k, r, lay, prev, valid, m, V, p, c, q, st, chi2, nval, bk, bk_stride);
      else
        live = fit_entry(a, g, static_cast<const T*>(nullptr), t, k, lay, prev, valid, m, V, p, c, q, st, chi2,
                         nval, bk, bk_stride);
      if (SMOOTH && !live) {
        // the pass stops here: the entries it will not reach get no
        // prediction (NaN), so that the combination skips them; a step that
        // failed in its update had stored its prediction already; a failed
        // first step or a bad layer id leaves the track unsmoothed
        const int first = (k == 0 || (st & TRK_BAD_INPUT)) ? n_e - 2 : ((st & TRK_NONFINITE) ? r - 1 : r);
        for (int rr = first; rr >= k0; --rr) b.smooth_state[int64_t(rr) * a.ld + t] = k_nan<T>();
      }
    }
    wave_sync();   // every lane has read the chunk before the next one is staged
  }
  if (in_range) {
    if (run) reverse_direction(p, c, q);
    store_fit(a, t, p, c, q, chi2, nval, st);
  }
}

// WAVES: waves per SIMD the register allocation must allow (2 in FP32, 1 in
// FP64, the forward fit's tuned choices).
template <typename T, int WAVES, int MODE>
__global__ void __launch_bounds__(kBwdBlock, WAVES) backward_kernel(BwdArgs<T> b, GeomArgs g) {
  constexpr int J = stage_entries<T, WAVES>();
  __shared__ GeomLds<T> sg;
  __shared__ T bk[28 * kBwdBlock];
  __shared__ StageBuf<T, J> sb[kBwdBlock / 64];
  stage_geometry(sg, g);
  const int64_t w0 = int64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u);
  backward_wave_staged<T, J, MODE>(b, TrackGeom<T>{sg.kind, sg.pos, sg.x0, g.n_layers, T(g.bz), T(g.mass)}, w0,
                             sb[threadIdx.x >> 6], bk + threadIdx.x, int(blockDim.x));
}

// The final fit's unbiased chi2, entry-parallel: thread (r, t) judges hit r
// of open track t (a used hit) against the estimate from the track's other
// hits: the forward prediction at r (the filtered state after entry r - 1,
// from the checkpoints, propagated to r's layer with its material; on the
// first used entry the seed with that layer's material) combined with the
// backward pass's prediction there (combine_on_surface), or the forward
// prediction alone on the last entry and where the backward pass did not
// reach.  With x, C that estimate, chi2 = r^T (V + H C H^T)^-1 r with
// r = m - H x (FP64 from here on; NaN when the forward prediction fails or
// the combination is not positive definite).
template <typename T>
__global__ void __launch_bounds__(256, KF_FINAL_CHI2_WAVES) final_chi2_kernel(FinalRoundArgs<T> a, GeomArgs g) {
  __shared__ GeomLds<T> sg;
  stage_geometry(sg, g);
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int r = int(blockIdx.y);
  if (t >= a.n) return;
  if (a.open && !(a.open[t] & kFinalOpen)) return;
  const int64_t e0 = a.hit_offsets[t];
  int n_e = int(a.hit_offsets[t + 1] - e0);
  if (n_e > a.max_len) n_e = a.max_len;
  if (r >= n_e) return;
  const int64_t e = e0 + r;
  if (!a.used[e]) return;
  T res = k_nan<T>();
  if (!(a.b_status[t] & TRK_BAD_INPUT)) {
    int k0 = 0;
    while (k0 < r && !a.used[e0 + k0]) ++k0;
    const int lay = a.hit_layer[e];
    if (lay >= 0 && lay < g.n_layers) {
      const int kind = sg.kind[lay];
      const T pos = sg.pos[lay], x0 = sg.x0[lay];
      // what the entry reads besides the forward prediction (the backward
      // prediction, the hit), loaded before the prediction is computed
      const int64_t os = a.n * int64_t(a.max_len), at = int64_t(r) * a.n + t;
      const bool two = r < n_e - 1;
      T pb[6], cb[21];
      if (two) {
#pragma unroll
        for (int i = 0; i < 6; ++i) pb[i] = a.pred_state[i * os + at];
#pragma unroll
        for (int i = 0; i < 21; ++i) cb[i] = a.pred_cov[i * os + at];
      }
      const int64_t nh = a.n_hits;
      T hm[3], hv[6];
#pragma unroll
      for (int i = 0; i < 3; ++i) hm[i] = a.hit_pos[i * nh + e];
#pragma unroll
      for (int i = 0; i < 6; ++i) hv[i] = a.hit_cov[i * nh + e];
      T p[6], c[21];
      int q;
      uint32_t st = 0;
      bool ok = true;
      if (r == k0) {
#pragma unroll
        for (int i = 0; i < 6; ++i) p[i] = a.seed_state[i * a.n + t];
        q = a.seed_charge[t];
        seed_covariance(c);
        add_material_here(p, c, kind, x0, T(g.mass), st);
      } else {
        const int64_t cs = a.n * int64_t(a.max_len > 1 ? a.max_len - 1 : 1);
        const T* f = a.ckpt + int64_t(r - 1 - k0) * a.n + t;
#pragma unroll
        for (int i = 0; i < 6; ++i) p[i] = f[i * cs];
#pragma unroll
        for (int i = 0; i < 21; ++i) c[i] = f[(6 + i) * cs];
        q = int(f[27 * cs]);
        const int prev = a.hit_layer[e - 1];
        ok = propagate(p, c, q, kind, pos, x0, lay == prev, true, T(g.bz), T(g.mass), st);
      }
      if (ok) {
        T px[6], cx[21];
        bool have = false;
        if (two && pb[0] == pb[0]) {
          ok = combine_on_surface(p, c, pb, cb, kind, pos, px, cx);
          have = true;
        }
        if (!have) {
#pragma unroll
          for (int i = 0; i < 6; ++i) px[i] = p[i];
#pragma unroll
          for (int i = 0; i < 21; ++i) cx[i] = c[i];
        }
        if (ok) {
          const double r0 = double(hm[0]) - double(px[0]);
          const double r1 = double(hm[1]) - double(px[1]);
          const double r2 = double(hm[2]) - double(px[2]);
          const double sa = double(hv[0]) + double(cx[0]);
          const double sb = double(hv[1]) + double(cx[1]);
          const double sc = double(hv[2]) + double(cx[2]);
          const double sd = double(hv[3]) + double(cx[3]);
          const double se = double(hv[4]) + double(cx[4]);
          const double sf = double(hv[5]) + double(cx[5]);
          const double i00 = sc * sf - se * se, i10 = sd * se - sb * sf, i20 = sb * se - sc * sd;
          const double i11 = sa * sf - sd * sd, i21 = sb * sd - sa * se, i22 = sa * sc - sb * sb;
          const double det = sa * i00 + sb * i10 + sd * i20;
          const double qf = r0 * (i00 * r0 + i10 * r1 + i20 * r2) + r1 * (i10 * r0 + i11 * r1 + i21 * r2) +
                            r2 * (i20 * r0 + i21 * r1 + i22 * r2);
          res = T(qf / det);
        }
      }
    }
  }
  a.chi2_work[e] = res;
}

}  // namespace

template <typename T>
hipError_t launch_backward(const BwdArgs<T>& a, const GeomArgs& g, hipStream_t s) {
  if (a.f.n == 0) return hipSuccess;
  const int64_t grid = (a.f.n + kBwdBlock - 1) / kBwdBlock;
  if (a.smooth_state) {
    hipLaunchKernelGGL((backward_kernel<T, sizeof(T) == 4 ? 2 : 1, kSmooth>), dim3(unsigned(grid)), dim3(kBwdBlock), 0,
                       s, a, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(smooth_combine_kernel<T>, dim3(unsigned((a.f.n + 255) / 256), unsigned(a.f.max_len)), dim3(256),
                       0, s, a, g);
  } else
    hipLaunchKernelGGL((backward_kernel<T, sizeof(T) == 4 ? 2 : 1, kPlain>), dim3(unsigned(grid)), dim3(kBwdBlock), 0,
                       s, a, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_backward_predictions(const BwdArgs<T>& a, const GeomArgs& g, hipStream_t s, int block) {
  if (a.f.n == 0) return hipSuccess;
  // the kernel's LDS is sized for kBwdBlock threads; smaller blocks of whole waves use part of it
  const int bs = block >= 64 && block <= kBwdBlock && block % 64 == 0 ? block : kBwdBlock;
  const int64_t grid = (a.f.n + bs - 1) / bs;
  hipLaunchKernelGGL((backward_kernel<T, sizeof(T) == 4 ? 2 : 1, kSmooth>), dim3(unsigned(grid)), dim3(bs), 0, s, a,
                     g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_final_chi2(const FinalRoundArgs<T>& a, const GeomArgs& g, hipStream_t s) {
  if (a.n == 0) return hipSuccess;
  hipLaunchKernelGGL(final_chi2_kernel<T>, dim3(unsigned((a.n + 255) / 256), unsigned(a.max_len)), dim3(256), 0, s,
                     a, g);
  return hipGetLastError();
}

template hipError_t launch_backward<float>(const BwdArgs<float>&, const GeomArgs&, hipStream_t);
template hipError_t launch_backward<double>(const BwdArgs<double>&, const GeomArgs&, hipStream_t);
template hipError_t launch_backward_predictions<float>(const BwdArgs<float>&, const GeomArgs&, hipStream_t, int);
template hipError_t launch_backward_predictions<double>(const BwdArgs<double>&, const GeomArgs&, hipStream_t, int);
template hipError_t launch_final_chi2<float>(const FinalRoundArgs<float>&, const GeomArgs&, hipStream_t);
template hipError_t launch_final_chi2<double>(const FinalRoundArgs<double>&, const GeomArgs&, hipStream_t);

}  // namespace kf
