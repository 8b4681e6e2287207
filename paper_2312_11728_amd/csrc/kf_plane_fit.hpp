// The per-track loop of the forward fit over tilted modules, callable from
// device and host code (the kernel runs it with one track per lane).
#pragma once

#include "kf_plane.hpp"
#include "kf_plane_launch.hpp"

namespace kf {

// Forward fit over the modules of each track's entries: the fit starts at
// the first valid entry (leading holes are skipped), where the seed sits on
// the hit; every entry, the first included (a step of length ~0 onto the
// plane), is propagated to with its module's material and, if valid, gets
// the local update.  A failed crossing, a module id out of range, or a step
// that turns the state non-finite (rolled back) stops the track.
template <typename T>
KF_HD void fit_plane_track(const PlaneFitArgs<T>& a, const PlaneGeomArgs<T>& g, int64_t t) {
  T p[6], c[21];
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = a.seed_state[i * a.ld + t];
#pragma unroll
  for (int i = 0; i < 21; ++i) c[i] = a.seed_cov[i * a.ld + t];
  int q = a.seed_charge[t];
  const int64_t e0 = a.hit_offsets[t], e1 = a.hit_offsets[t + 1];
  const int64_t nh = a.n_hits;
  const T bz = T(g.bz), mass = T(g.mass);
  int64_t k0 = e0;
  while (k0 < e1 && !a.hit_valid[k0]) ++k0;
  uint32_t st = 0;
  T chi2 = T(0);
  int nval = 0;
  if (k0 >= e1) st |= TRK_BAD_INPUT;
  for (int64_t e = k0; e < e1; ++e) {
    const int64_t mod = a.hit_module[e];
    if (mod < 0 || mod >= g.n_modules) {
      st |= TRK_BAD_INPUT;
      break;
    }
    Plane<T> pl;
    load_plane(g.table, g.n_modules, mod, pl);
    const bool valid = a.hit_valid[e] != 0;
    T bp[6], bc[21];
#pragma unroll
    for (int i = 0; i < 6; ++i) bp[i] = p[i];
#pragma unroll
    for (int i = 0; i < 21; ++i) bc[i] = c[i];
    const int bq = q;
    uint32_t sst = 0;
    if (!propagate_plane(p, c, q, pl, true, bz, mass, sst)) {
      st |= sst;
      break;
    }
    T c2 = T(0);
    if (valid) {
      const T m[2] = {a.hit_uv[e], a.hit_uv[nh + e]};
      const T V[3] = {a.hit_cov_uv[e], a.hit_cov_uv[nh + e], a.hit_cov_uv[2 * nh + e]};
      update_plane(p, c, q, pl, m, V, c2, sst);
    }
    if (!all_finite(p, c, c2)) {
      st |= sst | TRK_NONFINITE;
#pragma unroll
      for (int i = 0; i < 6; ++i) p[i] = bp[i];
#pragma unroll
      for (int i = 0; i < 21; ++i) c[i] = bc[i];
      q = bq;
      break;
    }
    st |= sst;
    chi2 += c2;
    nval += valid ? 1 : 0;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) a.state_out[i * a.ld + t] = p[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) a.cov_out[i * a.ld + t] = c[i];
  a.charge_out[t] = int8_t(q);
  a.chi2[t] = chi2;
  a.ndf[t] = 2 * nval - 5;
  a.trk_status[t] = st;
}

}  // namespace kf
