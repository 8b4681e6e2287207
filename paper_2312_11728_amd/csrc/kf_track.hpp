// The per-track layer loop of the forward fit, callable from device and host
// code: the kernels run it with one track per lane.
#pragma once

#include "kf_kernels.hpp"
#include "kf_math.hpp"

namespace kf {

// Spacing of the hits of a spaced seed (mode 1), cm in the transverse plane:
// wide enough to give closely spaced disk hits a usable lever arm, and below
// the 3 cm between the two innermost barrel layers of the toy detectors, so
// that whether a barrel hit pair qualifies is never decided by rounding.
constexpr double kSeedSpacing = 2.5;

// Seed of track t from three of its valid hits (mode 0: the first three;
// mode 1: the first, then each next one >= kSeedSpacing away in the
// transverse plane from the previously chosen one), with the charge and the
// status (KF_TRK_BAD_INPUT without three such hits; the state is then zero).
template <typename T>
struct SeedOut {
  T p[6];
  int q;
  uint32_t st;
};

// Not inlined: the seeding kernel and the fits that seed their own tracks
// call one compiled copy, so both give the same bits.
template <typename T>
KF_HD __attribute__((noinline)) SeedOut<T> seed_of_track(const int32_t* __restrict__ off,
                                                        const uint8_t* __restrict__ valid,
                                                        const T* __restrict__ pos, int64_t nh, int64_t t, int mode,
                                                        T bz) {
  const int64_t e0 = off[t], e1 = off[t + 1];
  int64_t pick[3] = {-1, -1, -1};
  int cnt = 0;
  T lx = T(0), ly = T(0);
  for (int64_t e = e0; e < e1 && cnt < 3; ++e) {
    if (!valid[e]) continue;
    const T hx = pos[e], hy = pos[nh + e];
    bool take = (cnt == 0);
    if (!take) {
      if (mode == 0) {
        take = true;
      } else {
        const T dx = hx - lx, dy = hy - ly;
        take = k_sqrt(dx * dx + dy * dy) >= T(kSeedSpacing);
      }
    }
    if (take) {
      pick[cnt++] = e;
      lx = hx;
      ly = hy;
    }
  }
  SeedOut<T> o;
#pragma unroll
  for (int i = 0; i < 6; ++i) o.p[i] = T(0);
  o.q = 1;
  o.st = 0;
  if (cnt == 3) {
    T h[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) h[k][c] = pos[c * nh + pick[k]];
    seed_from_hits(h[0], h[1], h[2], bz, o.p, o.q);
  } else {
    o.st |= TRK_BAD_INPUT;
  }
  return o;
}

// the seed covariance: wide and diagonal, so that the first hits decide
template <typename T>
KF_HD inline void seed_covariance(T c[21]) {
  const T diag[6] = {T(1), T(1), T(1), T(1), T(0.01), T(0.01)};
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) c[sym(i, j)] = (i == j) ? diag[i] : T(0);
}

template <typename T>
KF_HD inline void seed_track(const SeedArgs<T>& a, int64_t t) {
  const SeedOut<T> o = seed_of_track(a.hit_offsets, a.hit_valid, a.hit_pos, a.n_hits, t, int(a.mode), T(a.bz));
  T c[21];
  seed_covariance(c);
#pragma unroll
  for (int i = 0; i < 6; ++i) a.seed_state[i * a.ld + t] = o.p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) a.seed_cov[i * a.ld + t] = c[i];
  a.seed_charge[t] = int8_t(o.q);
  a.trk_status[t] = o.st;
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

// Entry access for the per-track loop: the caller's CSR arrays ...
template <typename T>
struct CsrTrack {
  const FitArgs<T>& a;
  int64_t e0;
  KF_HD inline bool valid(int k) const { return a.hit_valid[e0 + k] != 0; }
  KF_HD inline void load(int k, int& lay, bool& val, T m[3], T V[6]) const {
    const int64_t e = e0 + k, nh = a.n_hits;
    lay = a.hit_layer[e];
    val = a.hit_valid[e] != 0;
    m[0] = a.hit_pos[e];
    m[1] = a.hit_pos[nh + e];
    m[2] = a.hit_pos[2 * nh + e];
#pragma unroll
    for (int i = 0; i < 6; ++i) V[i] = a.hit_cov[i * nh + e];
  }
};

// ... or the packed tile-transposed copy (slot s of its tile).
template <typename T>
struct PackedTrack {
  const PackedHits<T>& pk;
  int64_t base;  // tile_base + s % kTile
  KF_HD inline bool valid(int k) const { return (pk.lv[base + int64_t(k) * kTile] >> 16) != 0; }
  KF_HD inline void load(int k, int& lay, bool& val, T m[3], T V[6]) const {
    const int64_t i = base + int64_t(k) * kTile, st = pk.stride;
    const int32_t lv = pk.lv[i];
    lay = int16_t(lv & 0xffff);
    val = (lv >> 16) != 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) m[c] = pk.hit[c * st + i];
#pragma unroll
    for (int c = 0; c < 6; ++c) V[c] = pk.hit[(3 + c) * st + i];
  }
};

// One entry of the forward fit: transport to layer `lay` (entry j > 0; the
// first entry only adds its own layer's material), then, for a valid hit, the
// alignment correction of the hit (barrel layers: rotation by a_rphi / R about
// the beam axis and a shift a_z along it) and the update.  m is overwritten
// with the aligned hit.  Returns false when the crossing fails; c2 is the
// entry's chi2 contribution (0 for a hole).
template <typename T>
KF_HD inline bool step_forward(T p[6], T c[21], int& q, int j, int lay, int prev, bool valid, T m[3], const T V[6],
                               const TrackGeom<T>& g, const T* __restrict__ sal, T& c2, uint32_t& sst) {
  const int kind = g.kind[lay];
  if (j > 0) {
    if (!propagate(p, c, q, kind, g.pos[lay], g.x0[lay], lay == prev, true, g.bz, g.mass, sst)) return false;
  } else {
    add_material_here(p, c, kind, g.x0[lay], g.mass, sst);
  }
  c2 = T(0);
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
  return true;
}

// The work of one entry of the forward fit, shared by every entry source:
// layer check, checkpoint, backup of the state (bk: room for 28 values at
// bk[k * bk_stride], kept out of registers -- in LDS on the device), the step,
// and the roll-back to the backup when the step turns non-finite.  j: index
// relative to the first valid entry.  Returns false when the track stops here
// (the reason is in st).
template <typename T>
KF_HD inline bool fit_entry(const FitArgs<T>& a, const TrackGeom<T>& g, const T* __restrict__ sal, int64_t t, int j,
                            int lay, int& prev, bool valid, T m[3], const T V[6], T p[6], T c[21], int& q,
                            uint32_t& st, T& chi2, int& nval, T* bk, int bk_stride) {
  if (lay < 0 || lay >= g.n_layers) {
    st |= TRK_BAD_INPUT;
    return false;
  }
  if (a.ckpt && j >= 1 && ((j - 1) % a.seg) == 0) write_checkpoint(a, t, (j - 1) / a.seg, p, c, q);
#pragma unroll
  for (int i = 0; i < 6; ++i) bk[i * bk_stride] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) bk[(6 + i) * bk_stride] = c[i];
  const int qq = q;
  uint32_t sst = 0;
  T c2;
  if (!step_forward(p, c, q, j, lay, prev, valid, m, V, g, sal, c2, sst)) {
    st |= sst;
    return false;
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

// The starting state of track t: the given seed, or (make_seeds) the seed
// made from its hits, whose status bits go to st.
template <typename T>
KF_HD inline void load_seed(const FitArgs<T>& a, int64_t t, T bz, T p[6], T c[21], int& q, uint32_t& st) {
  if (a.make_seeds == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) p[i] = a.seed_state[i * a.ld + t];
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = a.seed_cov[i * a.ld + t];
    q = a.seed_charge[t];
    return;
  }
  const SeedOut<T> o = seed_of_track(a.hit_offsets, a.hit_valid, a.hit_pos, a.n_hits, t, a.make_seeds - 1, bz);
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = o.p[i];
  q = o.q;
  st |= o.st;
  seed_covariance(c);
  if (a.seed_state_out) {
#pragma unroll
    for (int i = 0; i < 6; ++i) a.seed_state_out[i * a.ld + t] = p[i];
  }
  if (a.seed_cov_out) {
#pragma unroll
    for (int i = 0; i < 21; ++i) a.seed_cov_out[i * a.ld + t] = c[i];
  }
  if (a.seed_charge_out) a.seed_charge_out[t] = int8_t(q);
}

template <typename T>
KF_HD inline void store_fit(const FitArgs<T>& a, int64_t t, const T p[6], const T c[21], int q, T chi2, int nval,
                            uint32_t st) {
#pragma unroll
  for (int i = 0; i < 6; ++i) a.state_out[i * a.ld + t] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) a.cov_out[i * a.ld + t] = c[i];
  a.charge_out[t] = int8_t(q);
  a.chi2[t] = chi2;
  a.ndf[t] = 2 * nval - 5;
  a.trk_status[t] = st;
}

// Forward fit of track t whose entries are read through `acc` (len entries).
// sal: alignment staged as [rphi x kMaxLayers][z x kMaxLayers] or null.
// Leading holes are skipped: the fit starts at the first valid entry.
template <typename T, typename Acc>
KF_HD inline void fit_track(const FitArgs<T>& a, const TrackGeom<T>& g, const T* __restrict__ sal, int64_t t,
                            const Acc& acc, int len, T* bk, int bk_stride) {
  T p[6], c[21];
  int q;
  uint32_t st = 0;
  load_seed(a, t, g.bz, p, c, q, st);
  if (len > a.max_len) {
    st |= TRK_BAD_INPUT;
    len = a.max_len;
  }
  int k0 = 0;
  while (k0 < len && !acc.valid(k0)) ++k0;
  T chi2 = T(0);
  int nval = 0;
  if (k0 >= len) {
    st |= TRK_BAD_INPUT;
  } else {
    // entry data are loaded one entry ahead so that the loads of entry k+1
    // overlap the arithmetic of entry k
    int lay_n;
    bool valid_n;
    T m_n[3], V_n[6];
    acc.load(k0, lay_n, valid_n, m_n, V_n);
    int prev = lay_n;
    for (int k = k0; k < len; ++k) {
      const int lay = lay_n;
      const bool valid = valid_n;
      T m[3], V[6];
#pragma unroll
      for (int i = 0; i < 3; ++i) m[i] = m_n[i];
#pragma unroll
      for (int i = 0; i < 6; ++i) V[i] = V_n[i];
      if (k + 1 < len) acc.load(k + 1, lay_n, valid_n, m_n, V_n);
      if (!fit_entry(a, g, sal, t, k - k0, lay, prev, valid, m, V, p, c, q, st, chi2, nval, bk, bk_stride)) break;
    }
  }
  store_fit(a, t, p, c, q, chi2, nval, st);
}

// Fit of the track in slot / index `i`: LAYOUT 2 reads the packed layout,
// LAYOUT 1 the CSR arrays in length-sorted slot order, LAYOUT 0 the CSR arrays
// with slot = track.
template <typename T, int LAYOUT>
KF_HD inline void fit_slot(const FitArgs<T>& a, const TrackGeom<T>& g, const T* __restrict__ sal, int64_t i, T* bk,
                           int bk_stride) {
  if constexpr (LAYOUT == 1) {
    const int64_t t = a.pk.order[i];
    const int64_t e0 = a.hit_offsets[t];
    const int len = int(a.hit_offsets[t + 1] - e0);
    CsrTrack<T> acc{a, e0};
    fit_track(a, g, sal, t, acc, len, bk, bk_stride);
  } else if constexpr (LAYOUT == 2) {
    const int64_t t = a.pk.order[i];
    const int len = int(a.hit_offsets[t + 1] - a.hit_offsets[t]);
    PackedTrack<T> acc{a.pk, a.pk.tile_base[i / kTile] + (i % kTile)};
    fit_track(a, g, sal, t, acc, len, bk, bk_stride);
  } else {
    const int64_t e0 = a.hit_offsets[i];
    const int len = int(a.hit_offsets[i + 1] - e0);
    CsrTrack<T> acc{a, e0};
    fit_track(a, g, sal, i, acc, len, bk, bk_stride);
  }
}

}  // namespace kf
