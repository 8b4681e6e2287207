// Tilted planar modules (the Phase-2 layout of the paper's Sec. 3.1, where a
// module is given by its position, its normal and its phi-direction vector):
// helix propagation to a module's plane with the surface-to-surface Jacobian,
// the module's material at the crossing, and the Kalman update with the two
// local coordinates of a hit on the module.  Per-lane code for one track, like
// kf_math.hpp, whose helix point, covariance transport and Highland angle it
// uses.
#pragma once

#include "kf_math.hpp"

namespace kf {

// Rows of the module table [kModuleRows][n_modules] (SoA, the call's float
// type): centre, unit normal, unit phi-direction (in the plane), x/X0.
constexpr int kModuleRows = 10;

template <typename T>
struct Plane {
  T cx, cy, cz;   // centre
  T nx, ny, nz;   // unit normal
  T ux, uy, uz;   // unit phi-direction
  T vx, vy, vz;   // v = n x u
  T x0;           // x / X0 at normal incidence
};

template <typename T>
KF_HD inline void load_plane(const T* __restrict__ tab, int64_t n_mod, int64_t id, Plane<T>& pl) {
  pl.cx = tab[id];
  pl.cy = tab[n_mod + id];
  pl.cz = tab[2 * n_mod + id];
  pl.nx = tab[3 * n_mod + id];
  pl.ny = tab[4 * n_mod + id];
  pl.nz = tab[5 * n_mod + id];
  pl.ux = tab[6 * n_mod + id];
  pl.uy = tab[7 * n_mod + id];
  pl.uz = tab[8 * n_mod + id];
  pl.x0 = tab[9 * n_mod + id];
  pl.vx = pl.ny * pl.uz - pl.nz * pl.uy;
  pl.vy = pl.nz * pl.ux - pl.nx * pl.uz;
  pl.vz = pl.nx * pl.uy - pl.ny * pl.ux;
}

// Bound on the steps of the crossing search: a simple root takes 3-5, a
// crossing within 0.05 of tangency a few tens.
constexpr int kPlaneSteps = 64;

// First crossing of the plane: the smallest root s > -kSBack of
// h(s) = n.(x(s) - c) within one turn of the helix (s <= -kSBack + 2 pi/|w|).
// Along the helix h'(s) = n.d(s), d = (cos phi(s), sin phi(s), cot theta),
// and |h''(s)| <= M = |w| |n_xy|.  From a point where sigma h > 0 (sigma the
// sign of h there) no root lies closer than the smallest positive root of
// sigma h + sigma h' t - M t^2 / 2, t = 2 sigma h / (sqrt(h'^2 + 2 M sigma h)
// - sigma h'), so steps of that length, starting at s = -kSBack, reach the
// first root without passing it; near a simple root they are Newton steps to
// second order.  The search stops when a step no longer moves s by more than
// a few units in the last place, when h changes sign (the root, to
// rounding) or when s leaves the turn.  The crossing is accepted within
// 1e-9 cm of the plane in FP64; in FP32 within 64 units of 2^-23 of the
// module centre's distance from the origin (the rounding of the positions
// involved).  In FP32 small steps move the helix point to first order
// (helix_nudge, as in the cylinder crossing); larger ones and every FP64 step
// evaluate it afresh.
template <typename T>
KF_HD bool plane_crossing(const T p[6], T sphi, T cphi, T cot, T w, const Plane<T>& pl, T& s_out, HelixPt<T>& hp) {
  const T lo = T(-kSBack);
  const T aw = k_abs(w);
  const T M = aw * k_sqrt(pl.nx * pl.nx + pl.ny * pl.ny);
  const T s_max = aw > T(0) ? lo + T(kTwoPi) * k_rcp(aw) : k_inf<T>();
  constexpr bool kNudge = sizeof(T) == 4;
  const T eps = T(sizeof(T) == 4 ? kEpsF32 : 1.1102230246251565e-16);
  const T tiny = T(0.01) * eps;
  const T scale = k_abs(pl.cx) + k_abs(pl.cy) + k_abs(pl.cz);
  T s = lo;
  helix_eval(p, sphi, cphi, cot, w, s, hp);
  T h = (hp.x - pl.cx) * pl.nx + (hp.y - pl.cy) * pl.ny + (hp.z - pl.cz) * pl.nz;
  const T sig = h < T(0) ? T(-1) : T(1);
  for (int it = 0; it < kPlaneSteps; ++it) {
    const T hs = sig * h;
    if (!(hs > T(0))) break;   // on the root, or past it by rounding
    const T dh = sig * (hp.cphm * pl.nx + hp.sphm * pl.ny + cot * pl.nz);
    const T den = k_sqrt(dh * dh + T(2) * M * hs) - dh;
    if (!(den > T(0))) return false;   // a straight line moving away from the plane
    const T ds = T(2) * hs * k_rcp(den);
    if (!k_finite(ds)) return false;
    s += ds;
    if (!(s <= s_max)) return false;
    const T wd = w * ds;
    if (kNudge && wd * wd <= tiny && aw * ds * ds <= tiny * scale)
      helix_nudge(hp, w, cot, ds);
    else
      helix_eval(p, sphi, cphi, cot, w, s, hp);
    h = (hp.x - pl.cx) * pl.nx + (hp.y - pl.cy) * pl.ny + (hp.z - pl.cz) * pl.nz;
    if (ds <= T(4) * eps * (k_abs(s) + T(1))) break;
  }
  const T tol = sizeof(T) == 4 ? T(64) * eps * (scale + T(1)) : T(1e-9);
  if (!(k_abs(h) <= tol) || !(s > lo)) return false;
  s_out = s;
  return true;
}

// C <- (I - n n^T) C (I - n n^T) on the position block: the plane normal n
// (unit) becomes a null vector of the covariance.
template <typename T>
KF_HD inline void project_out_normal(T c[21], T nx, T ny, T nz) {
  T cn[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) cn[i] = c[sym(i, 0)] * nx + c[sym(i, 1)] * ny + c[sym(i, 2)] * nz;
  const T nn = cn[0] * nx + cn[1] * ny + cn[2] * nz;
  const T nv[6] = {nx, ny, nz, T(0), T(0), T(0)};
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) c[sym(i, j)] += -cn[i] * nv[j] - nv[i] * cn[j] + nn * nv[i] * nv[j];
}

// Propagate (p, c) to the module plane pl: crossing, state at the crossing,
// C <- F C F^T with F = G + g (ds/dp), ds/dp = -(n^T G_pos) / (n . g_pos),
// the normal imposed as a null vector, then (material) the Highland noise of
// x/X0 / |n . direction|.  Returns false, p and c untouched, when there is no
// admissible crossing.
template <typename T>
KF_HD bool propagate_plane(T p[6], T c[21], int q, const Plane<T>& pl, bool material, T bz, T mass, uint32_t& st,
                           T* path = nullptr) {
  const T dw_dipt = -T(q) * T(kCLight) * bz;
  const T w = dw_dipt * p[3];
  T sphi, cphi, sth, cth;
  k_sincos(p[4], &sphi, &cphi);
  k_sincos(p[5], &sth, &cth);
  const T isth = k_rcp(sth);
  const T cot = cth * isth;
  T s;
  HelixPt<T> hp;
  if (!plane_crossing(p, sphi, cphi, cot, w, pl, s, hp)) {
    st |= TRK_NO_CROSSING;
    return false;
  }
  if (path) *path = s;
  const T sphm = hp.sphm, cphm = hp.cphm;
  const T f1 = u_minus_sin_over_u2(hp.u);
  const T f2 = T(0.5) * hp.shc * hp.shc;
  const T s2 = s * s;
  const T dxdw = s2 * (cphm * f1 - sphm * f2);
  const T dydw = s2 * (sphm * f1 + cphm * f2);
  const T G03 = dxdw * dw_dipt, G04 = -hp.dy;
  const T G13 = dydw * dw_dipt, G14 = hp.dx;
  const T G25 = -s * isth * isth;
  const T G43 = s * dw_dipt;
  const T inv = -k_rcp(pl.nx * cphm + pl.ny * sphm + pl.nz * cot);
  T d[6];
  d[0] = pl.nx * inv;
  d[1] = pl.ny * inv;
  d[2] = pl.nz * inv;
  d[3] = (pl.nx * G03 + pl.ny * G13) * inv;
  d[4] = (pl.nx * G04 + pl.ny * G14) * inv;
  d[5] = pl.nz * G25 * inv;
  transport_cov(c, d, G03, G04, G13, G14, G25, G43, cphm, sphm, cot, w);
  project_out_normal(c, pl.nx, pl.ny, pl.nz);
  p[0] = hp.x;
  p[1] = hp.y;
  p[2] = hp.z;
  p[4] = wrap_phi(hp.phi);
  if (material) {
    const T ca = k_abs(sth * (cphm * pl.nx + sphm * pl.ny) + cth * pl.nz);
    const T var = highland_var(p[3], sth, ca, pl.x0, mass, st);
    add_q(c, p[3], sth, cot, var);
  }
  return true;
}

// The local update in type T: H = [u^T 0; v^T 0], B = C H^T (6 x 2),
// S = H B + V (2 x 2), r = m - H (x - c), K = B S^-1, chi2 = r^T S^-1 r,
// p += K r, and the Joseph form expanded as C - K B^T - E K^T with
// E = B - K S (equal to (I - KH) C (I - KH)^T + K V K^T for any gain, the
// rounding of K entering at second order); then the charge flip, the phi
// wrap and the positivity check of kf_math.hpp's update.  Si: S^-1 packed
// (00, 10, 11), computed by the caller.
template <typename T>
KF_HD inline void update_plane_core(T p[6], T c[21], int& q, const Plane<T>& pl, const T m[2], const T V[3],
                                    const T B[6][2], const T S[3], const T Si[3], T& chi2, uint32_t& st) {
  const T tr_prior = c[0] + c[2] + c[5];
  const T dx = p[0] - pl.cx, dy = p[1] - pl.cy, dz = p[2] - pl.cz;
  const T r0 = m[0] - (dx * pl.ux + dy * pl.uy + dz * pl.uz);
  const T r1 = m[1] - (dx * pl.vx + dy * pl.vy + dz * pl.vz);
  const T z0 = Si[0] * r0 + Si[1] * r1;
  const T z1 = Si[1] * r0 + Si[2] * r1;
  chi2 = r0 * z0 + r1 * z1;
  T K[6][2], E[6][2];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    K[i][0] = B[i][0] * Si[0] + B[i][1] * Si[1];
    K[i][1] = B[i][0] * Si[1] + B[i][1] * Si[2];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] += B[i][0] * z0 + B[i][1] * z1;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    E[i][0] = B[i][0] - K[i][0] * S[0] - K[i][1] * S[1];
    E[i][1] = B[i][1] - K[i][0] * S[1] - K[i][1] * S[2];
  }
#pragma unroll
  for (int j = 0; j < 6; ++j)
#pragma unroll
    for (int i = j; i < 6; ++i) {
      T v = c[sym(i, j)];
      v = v - K[i][0] * B[j][0];
      v = v - K[i][1] * B[j][1];
      v = v - E[i][0] * K[j][0];
      v = v - E[i][1] * K[j][1];
      c[sym(i, j)] = v;
    }
  if (p[3] < T(0)) {
    p[3] = -p[3];
    q = -q;
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (j != 3) c[sym(3, j)] = -c[sym(3, j)];
    st |= TRK_CHARGE_FLIP;
  }
  p[4] = wrap_phi(p[4]);
  const T tr = c[0] + c[2] + c[5];
  const T tol = T(1e-3) * tr + T(kPsdUlps * (sizeof(T) == 4 ? kEpsF32 : 0.0)) * tr_prior;
  if (!(c[sym(3, 3)] > T(0)) || !(c[sym(4, 4)] > T(0)) || !(c[sym(5, 5)] > T(0)) || c[0] < -tol ||
      c[2] < -tol || c[5] < -tol)
    st |= TRK_COV_NOT_PSD;
}

// B = C H^T and S = H C H^T + V for the plane's (u, v).
template <typename T>
KF_HD inline void plane_gain_inputs(const T c[21], const Plane<T>& pl, const T V[3], T B[6][2], T S[3]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    B[i][0] = c[sym(i, 0)] * pl.ux + c[sym(i, 1)] * pl.uy + c[sym(i, 2)] * pl.uz;
    B[i][1] = c[sym(i, 0)] * pl.vx + c[sym(i, 1)] * pl.vy + c[sym(i, 2)] * pl.vz;
  }
  S[0] = pl.ux * B[0][0] + pl.uy * B[1][0] + pl.uz * B[2][0] + V[0];
  S[1] = pl.vx * B[0][0] + pl.vy * B[1][0] + pl.vz * B[2][0] + V[1];
  S[2] = pl.vx * B[0][1] + pl.vy * B[1][1] + pl.vz * B[2][1] + V[2];
}

template <typename T>
KF_HD inline T inv2(const T S[3], T Si[3]) {
  const T det = S[0] * S[2] - S[1] * S[1];
  const T r = k_rcp(det);
  Si[0] = S[2] * r;
  Si[1] = -S[1] * r;
  Si[2] = S[0] * r;
  return det;
}

// The whole local update of one FP32 lane carried out in FP64.
KF_HD inline void update_plane_lane_fp64(float p[6], float c[21], int& q, const Plane<float>& pl, const float m[2],
                                         const float V[3], float& chi2, uint32_t& st) {
  double pd[6], cd[21], md[2] = {double(m[0]), double(m[1])}, Vd[3] = {double(V[0]), double(V[1]), double(V[2])};
#pragma unroll
  for (int i = 0; i < 6; ++i) pd[i] = double(p[i]);
#pragma unroll
  for (int i = 0; i < 21; ++i) cd[i] = double(c[i]);
  Plane<double> pd_pl{pl.cx, pl.cy, pl.cz, pl.nx, pl.ny, pl.nz, pl.ux, pl.uy, pl.uz, pl.vx, pl.vy, pl.vz, pl.x0};
  double B[6][2], S[3], Si[3], c2;
  plane_gain_inputs(cd, pd_pl, Vd, B, S);
  inv2(S, Si);
  update_plane_core(pd, cd, q, pd_pl, md, Vd, B, S, Si, c2, st);
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = float(pd[i]);
#pragma unroll
  for (int i = 0; i < 21; ++i) c[i] = float(cd[i]);
  chi2 = float(c2);
  st |= TRK_FP64_FALLBACK;
}

// Kalman update with the local measurement (m_u, m_v), covariance V packed
// (uu, vu, vv), on the plane pl.  FP32 lanes move to FP64 when the projected
// prior H C H^T exceeds the hit covariance by more than kRatioMax (tested on
// tr(V^-1 H C H^T), as the 3-D update does), and take an FP64 inverse of S
// when det S <= 0 or its condition estimate exceeds kKappaMax.
template <typename T>
KF_HD void update_plane(T p[6], T c[21], int& q, const Plane<T>& pl, const T m[2], const T V[3], T& chi2,
                        uint32_t& st) {
  T B[6][2], S[3], Si[3];
  plane_gain_inputs(c, pl, V, B, S);
  if constexpr (std::is_same<T, float>::value) {
    const float P0 = S[0] - V[0], P1 = S[1] - V[1], P2 = S[2] - V[2];
    const float detv = V[0] * V[2] - V[1] * V[1];
    const float tr = V[2] * P0 - 2.f * V[1] * P1 + V[0] * P2;
    if (!(tr <= float(kRatioMax) * detv)) {
      update_plane_lane_fp64(p, c, q, pl, m, V, chi2, st);
      return;
    }
    const float det = inv2(S, Si);
    const float nS = fmaxf(k_abs(S[0]) + k_abs(S[1]), k_abs(S[1]) + k_abs(S[2]));
    const float nSi = fmaxf(k_abs(Si[0]) + k_abs(Si[1]), k_abs(Si[1]) + k_abs(Si[2]));
    if (!(det > 0.f) || !(nS * nSi <= float(kKappaMax))) {
      const double Sd[3] = {double(S[0]), double(S[1]), double(S[2])};
      double Sid[3];
      inv2(Sd, Sid);
      Si[0] = float(Sid[0]);
      Si[1] = float(Sid[1]);
      Si[2] = float(Sid[2]);
      st |= TRK_FP64_FALLBACK;
    }
  } else {
    inv2(S, Si);
  }
  update_plane_core(p, c, q, pl, m, V, B, S, Si, chi2, st);
}

}  // namespace kf
