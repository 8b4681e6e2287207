// The per-track layer loop of the forward fit, callable from device and host
// code: the kernels run it with one track per lane.
#pragma once

#include "kf_kernels.hpp"
#include "kf_math.hpp"

namespace kf {

// Seed of track t from three of its valid hits (mode 0: the first three;
// mode 1: the first, then each next one >= 3 cm away in the transverse plane
// from the previously chosen one).
template <typename T>
KF_HD inline void seed_track(const SeedArgs<T>& a, int64_t t) {
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
struct TrackGeom {
  const int* kind;
  const T* pos;
  const T* x0;
  int n_layers;
  T bz;
  T mass;
};

template <typename T>
KF_HD inline void write_checkpoint(const FitArgs<T>& a, int64_t t, int slot, const T p[6], const T c[21], int q) {
  const int64_t stride = a.ld * int64_t(a.n_seg);
  T* base = a.ckpt + int64_t(slot) * a.ld + t;
#pragma unroll
  for (int i = 0; i < 6; ++i) base[i * stride] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) base[(6 + i) * stride] = c[i];
  base[27 * stride] = T(q);
}

// Forward fit of track t.  sal: alignment staged as [rphi x kMaxLayers][z x kMaxLayers] or null.
// bk: room for 28 values at bk[k * bk_stride] (k = 0..27) holding the state
// before the current entry, read back only if that entry turns non-finite
// (kept out of registers: in LDS on the device).
template <typename T>
KF_HD inline void fit_track(const FitArgs<T>& a, const TrackGeom<T>& g, const T* __restrict__ sal, int64_t t,
                            T* bk, int bk_stride) {
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
  if (k0 >= e1) {
    st |= TRK_BAD_INPUT;
  } else {
    int prev = a.hit_layer[k0];
    // entry data are loaded one entry ahead so that the loads of entry e+1
    // overlap the arithmetic of entry e
    int lay_n = prev;
    bool valid_n = true;
    T m_n[3], V_n[6];
    m_n[0] = a.hit_pos[k0];
    m_n[1] = a.hit_pos[nh + k0];
    m_n[2] = a.hit_pos[2 * nh + k0];
#pragma unroll
    for (int i = 0; i < 6; ++i) V_n[i] = a.hit_cov[i * nh + k0];
    for (int64_t e = k0; e < e1; ++e) {
      const int lay = lay_n;
      const bool valid = valid_n;
      T m[3], V[6];
#pragma unroll
      for (int i = 0; i < 3; ++i) m[i] = m_n[i];
#pragma unroll
      for (int i = 0; i < 6; ++i) V[i] = V_n[i];
      if (e + 1 < e1) {
        const int64_t f = e + 1;
        lay_n = a.hit_layer[f];
        valid_n = a.hit_valid[f] != 0;
        m_n[0] = a.hit_pos[f];
        m_n[1] = a.hit_pos[nh + f];
        m_n[2] = a.hit_pos[2 * nh + f];
#pragma unroll
        for (int i = 0; i < 6; ++i) V_n[i] = a.hit_cov[i * nh + f];
      }
      if (lay < 0 || lay >= g.n_layers) {
        st |= TRK_BAD_INPUT;
        break;
      }
      const int j = int(e - k0);
      if (a.ckpt && j >= 1 && ((j - 1) % a.seg) == 0) write_checkpoint(a, t, (j - 1) / a.seg, p, c, q);
#pragma unroll
      for (int i = 0; i < 6; ++i) bk[i * bk_stride] = p[i];
#pragma unroll
      for (int i = 0; i < 21; ++i) bk[(6 + i) * bk_stride] = c[i];
      const int qq = q;
      uint32_t sst = 0;
      const int kind = g.kind[lay];
      if (j > 0) {
        if (!propagate(p, c, q, kind, g.pos[lay], g.x0[lay], lay == prev, true, g.bz, g.mass, sst)) {
          st |= sst;
          break;
        }
      } else {
        add_material_here(p, c, kind, g.x0[lay], g.mass, sst);
      }
      T c2 = T(0);
      if (valid) {
        if (sal && kind == 0) {
          const T ang = sal[lay] * k_rcp(g.pos[lay]);
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
        for (int i = 0; i < 6; ++i) p[i] = bk[i * bk_stride];
#pragma unroll
        for (int i = 0; i < 21; ++i) c[i] = bk[(6 + i) * bk_stride];
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

}  // namespace kf
