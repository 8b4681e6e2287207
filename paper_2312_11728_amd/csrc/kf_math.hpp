// Per-lane Kalman-filter step for one track: helix propagation to a layer
// surface, transport Jacobian, covariance propagation with multiple
// scattering, and the Kalman update.  Templated on the arithmetic type (float
// or double); every function works on registers of one lane.
//
// The paper (Sec. 3.1) lists these as the vectorised key computations
// (track-candidate propagation, hit selection, Kalman-filter calculations);
// the formulas are the standard ones for a helix in a uniform solenoidal field,
// the Highland scattering angle and the linear Kalman filter, written here in
// forms that keep FP32 accurate (chord forms, a half-angle quadratic for the
// crossing, series for small turning angles).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <type_traits>

// Every function is callable from device code and from host code (the
// latter lets the same per-track arithmetic be exercised on a CPU).
#define KF_HD __host__ __device__

namespace kf {

constexpr double kCLight = 0.00299792458;  // GeV/c per (T cm)
constexpr double kGrazingCos = 0.05;
constexpr double kSBack = 1.0;    // cm: a different layer may be this far behind
constexpr double kSSame = 0.01;   // cm: minimum path to re-cross the current layer
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;
constexpr double kKappaMax = 1e6;  // condition estimate that triggers the FP64 inverse
// prior-to-hit variance ratio above which an FP32 update loses too many digits
// (the posterior variance is a difference of nearly equal numbers) and the
// lane's update is done in FP64 instead
constexpr double kRatioMax = 1e4;
// A position variance counts as negative (TRK_COV_NOT_PSD) below -1e-3 of the
// position trace.  An FP32 covariance also carries rounding of the order of
// its own scale before the update; a prior far larger than the posterior (the
// first steps after a restart from a scaled-up covariance) leaves residues of
// that order along the surface normal, whose true variance is zero.  In FP32
// the threshold is therefore widened by kPsdUlps units of 2^-23 of the prior's
// position trace; in FP64 that term is negligible and left out.
constexpr double kPsdUlps = 16.0;
constexpr double kEpsF32 = 1.1920928955078125e-7;   // 2^-23

enum : uint32_t {
  TRK_NO_CROSSING = 1u,
  TRK_GRAZING = 2u,
  TRK_NONFINITE = 4u,
  TRK_FP64_FALLBACK = 8u,
  TRK_CHARGE_FLIP = 16u,
  TRK_COV_NOT_PSD = 32u,
  TRK_BAD_INPUT = 64u,
};

// packed lower-triangular index of a symmetric matrix
KF_HD constexpr int sym(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// ---- type-generic math -----------------------------------------------------
KF_HD inline float k_sqrt(float x) { return sqrtf(x); }
KF_HD inline double k_sqrt(double x) { return sqrt(x); }
KF_HD inline float k_abs(float x) { return fabsf(x); }
KF_HD inline double k_abs(double x) { return fabs(x); }
KF_HD inline void k_sincos(float x, float* s, float* c) { sincosf(x, s, c); }
KF_HD inline void k_sincos(double x, double* s, double* c) { sincos(x, s, c); }
KF_HD inline float k_atan2(float y, float x) { return atan2f(y, x); }
KF_HD inline double k_atan2(double y, double x) { return atan2(y, x); }
KF_HD inline float k_atan(float x) { return atanf(x); }
KF_HD inline double k_atan(double x) { return atan(x); }
KF_HD inline float k_log(float x) { return logf(x); }
KF_HD inline double k_log(double x) { return log(x); }
KF_HD inline float k_floor(float x) { return floorf(x); }
KF_HD inline double k_floor(double x) { return floor(x); }
KF_HD inline float k_ceil(float x) { return ceilf(x); }
KF_HD inline double k_ceil(double x) { return ceil(x); }
// The class test, not x - x == 0: with floating-point contraction, the
// compiler turns x - x for a product x = a b into fma(a, b, -x), the
// product's rounding error, which is non-zero for most finite x.
KF_HD inline bool k_finite(float x) { return __builtin_isfinite(x); }
KF_HD inline bool k_finite(double x) { return __builtin_isfinite(x); }
template <typename T>
KF_HD inline T k_inf() { return T(__builtin_huge_val()); }
template <typename T>
KF_HD inline T k_nan() { return T(__builtin_nan("")); }
KF_HD inline float k_copysign(float a, float b) { return copysignf(a, b); }
KF_HD inline double k_copysign(double a, double b) { return copysign(a, b); }

// Reciprocal: the hardware approximation (1 ulp) for FP32 on the device,
// the correctly rounded quotient otherwise.
KF_HD inline float k_rcp(float x) {
#ifdef __HIP_DEVICE_COMPILE__
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
KF_HD inline double k_rcp(double x) { return 1.0 / x; }

template <typename T>
KF_HD inline T wrap_phi(T phi) {
  // to (-pi, pi]
  return phi - T(kTwoPi) * k_ceil((phi - T(kPi)) * T(1.0 / kTwoPi));
}

// The same track moving the opposite way along its helix: direction
// (phi, theta) -> (phi + pi, pi - theta) and charge -q, position and ipt
// unchanged (omega = -q c_B B_z ipt and cot(theta) change sign, so the helix
// is traced backwards).  The map's Jacobian is diag(1, 1, 1, 1, 1, -1): the
// covariance terms of theta with the other five change sign.
template <typename T>
KF_HD inline void reverse_direction(T p[6], T c[21], int& q) {
  p[4] = wrap_phi(p[4] + T(kPi));
  p[5] = T(kPi) - p[5];
  q = -q;
#pragma unroll
  for (int j = 0; j < 5; ++j) c[sym(5, j)] = -c[sym(5, j)];
}

// The covariance of a state on a surface has the surface normal as a null
// vector: C <- (I - n n^T) C (I - n n^T) on the position block, n = (x, y) / R
// for a barrel of radius R, the z row and column cleared for a disk (the same
// projection propagate() applies after a crossing).  A covariance that already
// has the null vector is unchanged up to rounding; a stored and scaled-up one
// loses its rounding residue along n.
template <typename T>
KF_HD inline void impose_surface(T c[21], const T p[6], int kind, T pos) {
  if (kind == 1) {
#pragma unroll
    for (int j = 0; j < 6; ++j) c[sym(2, j)] = T(0);
    return;
  }
  const T rinv = k_rcp(pos);
  const T nx = p[0] * rinv, ny = p[1] * rinv;
  T cn[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) cn[i] = c[sym(i, 0)] * nx + c[sym(i, 1)] * ny;
  const T nn = cn[0] * nx + cn[1] * ny;
  const T nv[6] = {nx, ny, T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) c[sym(i, j)] += -cn[i] * nv[j] - nv[i] * cn[j] + nn * nv[i] * nv[j];
}

// sin(h)/h
template <typename T>
KF_HD inline T sinc(T h) {
  T h2 = h * h;
  if (k_abs(h) < T(0.05)) return T(1) - h2 * (T(1.0 / 6.0) - h2 * (T(1.0 / 120.0) - h2 * T(1.0 / 5040.0)));
  T s, c;
  k_sincos(h, &s, &c);
  return s * k_rcp(h);
}

// (u - sin u)/u^2
template <typename T>
KF_HD inline T u_minus_sin_over_u2(T u) {
  if (k_abs(u) < T(0.5)) {
    T u2 = u * u;
    // u/6 - u^3/120 + u^5/5040 - u^7/362880 + u^9/39916800 - u^11/6227020800 + u^13/1307674368000
    T r = T(1.0 / 1307674368000.0);
    r = T(1.0 / 6227020800.0) - u2 * r;
    r = T(1.0 / 39916800.0) - u2 * r;
    r = T(1.0 / 362880.0) - u2 * r;
    r = T(1.0 / 5040.0) - u2 * r;
    r = T(1.0 / 120.0) - u2 * r;
    r = T(1.0 / 6.0) - u2 * r;
    return u * r;
  }
  T s, c;
  k_sincos(u, &s, &c);
  return (u - s) * k_rcp(u * u);
}

// atan(t)/t
template <typename T>
KF_HD inline T atanc(T t) {
  if (k_abs(t) < T(0.05)) {
    T t2 = t * t;
    return T(1) - t2 * (T(1.0 / 3.0) - t2 * (T(0.2) - t2 * T(1.0 / 7.0)));
  }
  return k_atan(t) * k_rcp(t);
}

// ---- a1: crossing ------------------------------------------------------------

// Map a root s onto the admissible window (lo, lo + 2 pi/|w|].
template <typename T>
KF_HD inline T to_window(T s, T lo, T w) {
  T aw = k_abs(w);
  if (aw == T(0)) return s;  // straight line: caller rejects s <= lo
  T P = T(kTwoPi) * k_rcp(aw);
  T d = s - lo;
  T m = d - P * k_floor(d * aw * T(1.0 / kTwoPi));
  if (m <= T(0)) m += P;
  return lo + m;
}

// Path s (transverse) along the helix through a half-angle quadratic root:
// tan(u/2) = w*sig, s = u/w, evaluated without loss as w -> 0.
template <typename T>
KF_HD inline T path_from_sigma(T num, T den, T w) {
  // sig = num/den; u = 2 atan2(w num, den) taken on the branch through 0
  T t = w * num;
  if (k_abs(t) < T(0.1) * k_abs(den)) {
    T sig = num * k_rcp(den);
    return T(2) * sig * atanc(w * sig);
  }
  return T(2) * k_atan2(t, den) * k_rcp(w);
}

// Point of the helix at transverse path s, from the trigonometry of the start
// direction (sphi, cphi = sin, cos phi0) and of the half turning angle only:
// with u = w s and h = u/2, the chord is s sinc(h) along phi0 + h, and every
// other angle follows from the addition identities (1 - cos u = 2 sin^2 h
// exactly, so nothing cancels).
template <typename T>
struct HelixPt {
  T x, y, z, phi;   // position and direction at s
  T sphm, cphm;     // sin, cos of phi
  T dx, dy;         // chord components
  T u, sh, ch, shc; // turning angle, sin(u/2), cos(u/2), sinc(u/2)
  T smid, cmid;     // sin, cos of phi0 + u/2
};

template <typename T>
KF_HD inline void helix_eval(const T p[6], T sphi, T cphi, T cot, T w, T s, HelixPt<T>& o) {
  const T u = w * s;
  const T h = T(0.5) * u;
  T sh, ch;
  k_sincos(h, &sh, &ch);
  T shc;
  if (k_abs(h) < T(0.05)) {
    const T h2 = h * h;
    shc = T(1) - h2 * (T(1.0 / 6.0) - h2 * (T(1.0 / 120.0) - h2 * T(1.0 / 5040.0)));
  } else {
    shc = sh * k_rcp(h);
  }
  const T smid = sphi * ch + cphi * sh;
  const T cmid = cphi * ch - sphi * sh;
  const T sin_u = T(2) * sh * ch;
  const T cos_u = T(1) - T(2) * sh * sh;
  o.dx = s * cmid * shc;
  o.dy = s * smid * shc;
  o.x = p[0] + o.dx;
  o.y = p[1] + o.dy;
  o.z = p[2] + s * cot;
  o.phi = p[4] + u;
  o.sphm = sphi * cos_u + cphi * sin_u;
  o.cphm = cphi * cos_u - sphi * sin_u;
  o.u = u;
  o.sh = sh;
  o.ch = ch;
  o.shc = shc;
  o.smid = smid;
  o.cmid = cmid;
}

// Move a helix point by a small extra path ds, to first order in w ds: the
// position and chord move along the direction at s, the direction turns by
// w ds, and the half-angle quantities (h = u/2) turn by w ds / 2, so every
// identity between the fields keeps holding to second order.  The dropped
// terms are (w ds)^2 / 2 in the angles and |w| ds^2 / 2 in the position.
template <typename T>
KF_HD inline void helix_nudge(HelixPt<T>& o, T w, T cot, T ds) {
  o.x += ds * o.cphm;
  o.y += ds * o.sphm;
  o.dx += ds * o.cphm;
  o.dy += ds * o.sphm;
  o.z += ds * cot;
  const T dphi = w * ds;
  const T h = T(0.5) * o.u;
  o.phi += dphi;
  o.u += dphi;
  const T sp = o.sphm, cp = o.cphm;
  o.sphm = sp + dphi * cp;
  o.cphm = cp - dphi * sp;
  const T dh = T(0.5) * dphi;
  // d sinc(h) / dh = (cos h - sinc h) / h, = -h/3 to O(h^3) near 0
  const T dshc = k_abs(h) < T(0.05) ? -h * T(1.0 / 3.0) : (o.ch - o.shc) * k_rcp(h);
  const T sh = o.sh, ch = o.ch, sm = o.smid, cm = o.cmid;
  o.sh = sh + dh * ch;
  o.ch = ch - dh * sh;
  o.smid = sm + dh * cm;
  o.cmid = cm - dh * sm;
  o.shc += dh * dshc;
}

// First admissible crossing of the layer surface.  Barrel: roots of
// r(s)^2 = R^2 written as alpha sig^2 + 2 A sig - D/2 = 0 with tan(u/2) = w sig,
// A = x cos phi + y sin phi, B = x sin phi - y cos phi, D = R^2 - r^2,
// alpha = 2 (1 - w B) - w^2 D / 2; then one Newton step on r^2 - R^2.
// Disk: s = (Z - z)/cot(theta).  On success fills the helix point at s.
template <typename T>
KF_HD bool crossing(const T p[6], T sphi, T cphi, T cot, T w, int kind, T pos, bool same, T& s_out,
                    HelixPt<T>& hp) {
  T lo = same ? T(kSSame) : T(-kSBack);
  if (kind == 1) {
    if (!(k_abs(cot) > T(1e-12))) return false;
    T s = (pos - p[2]) * k_rcp(cot);
    if (!(s > lo)) return false;
    s_out = s;
    helix_eval(p, sphi, cphi, cot, w, s, hp);
    hp.z = pos;
    return true;
  }
  T x = p[0], y = p[1];
  T A = x * cphi + y * sphi;
  T B = x * sphi - y * cphi;
  T r0 = k_sqrt(x * x + y * y);
  T D = (pos - r0) * (pos + r0);
  T alpha = T(2) * (T(1) - w * B) - T(0.5) * w * w * D;
  T disc = A * A + T(0.5) * alpha * D;
  if (!(disc >= T(0))) return false;
  T sq = k_sqrt(disc);
  T qq = -(A + k_copysign(sq, A));
  T best = T(0);
  bool found = false;
  // root 1: sig = qq / alpha
  if (qq != T(0) || alpha != T(0)) {
    T s1 = path_from_sigma(qq, alpha, w);
    if (k_finite(s1)) {
      s1 = to_window(s1, lo, w);
      if (s1 > lo) {
        best = s1;
        found = true;
      }
    }
  }
  // root 2: sig = -D / (2 qq)
  if (qq != T(0)) {
    T s2 = path_from_sigma(T(-0.5) * D, qq, w);
    if (k_finite(s2)) {
      s2 = to_window(s2, lo, w);
      if (s2 > lo && (!found || s2 < best)) {
        best = s2;
        found = true;
      }
    }
  }
  if (!found) return false;
  // Newton polish on h(s) = r(s)^2 - R^2: two steps (the second matters near
  // tangency, where h'(s) is small and the closed-form root is least
  // accurate).  In FP32 a correction whose second-order terms stay below a
  // hundredth of a unit in the last place, (w ds)^2 in the angles and
  // |w| ds^2 against R in the position, moves the point to first order
  // (helix_nudge); otherwise, and always in FP64, the point is evaluated
  // afresh.
  helix_eval(p, sphi, cphi, cot, w, best, hp);
  constexpr bool kNudge = sizeof(T) == 4;
  const T tiny = T(0.01 * 1.1920929e-7);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const T f = (hp.x * hp.x + hp.y * hp.y - pos * pos);
    const T df = T(2) * (hp.x * hp.cphm + hp.y * hp.sphm);
    if (k_abs(df) > T(1e-20)) {
      const T ds = -f * k_rcp(df);
      best += ds;
      const T wd = w * ds;
      if (kNudge && wd * wd <= tiny && k_abs(w) * ds * ds <= tiny * pos)
        helix_nudge(hp, w, cot, ds);
      else
        helix_eval(p, sphi, cphi, cot, w, best, hp);
    }
  }
  s_out = best;
  return true;
}

// ---- a1-a3: propagate state and covariance ----------------------------------

// Highland angle squared for unit charge at the state (ipt, theta) crossing
// x_over_x0 at |cos(incidence)| = ca (clamped at kGrazingCos, flagged).
template <typename T>
KF_HD inline T highland_var(T ipt, T sth, T ca, T x_over_x0, T mass, uint32_t& st) {
  if (ca < T(kGrazingCos)) {
    st |= TRK_GRAZING;
    ca = T(kGrazingCos);
  }
  const T mis = mass * ipt * sth;              // m / p
  const T xl = x_over_x0 * k_rcp(ca);
  const T one_m = T(1) + mis * mis;            // 1 / beta^2
  const T inv_bp = ipt * sth * k_sqrt(one_m);  // 1 / (beta p)
  const T th0 = T(0.0136) * inv_bp * k_sqrt(xl) * (T(1) + T(0.038) * k_log(xl * one_m));
  return th0 * th0;
}

// Add the scattering noise Q (rank 2 in ipt, phi, theta).
template <typename T>
KF_HD inline void add_q(T c[21], T ipt, T sth, T cot, T var) {
  const T ic = ipt * cot;
  c[sym(3, 3)] += ic * ic * var;
  c[sym(5, 3)] += -ic * var;
  c[sym(4, 4)] += var * k_rcp(sth * sth);
  c[sym(5, 5)] += var;
}

// C <- F C F^T for the surface-to-surface Jacobian F = G + g d^T: G the
// helix partials at fixed path (identity but for G03, G04, G13, G14, G25,
// G43), g = d(state)/ds = (g0, g1, g2, 0, g4, 0) and d = ds/dp.  Expanded as
// G C G^T + g v^T + v g^T + a g g^T with v = G C d and a = d^T C d, which
// uses the sparsity of G and never forms F.
template <typename T>
KF_HD inline void transport_cov(T c[21], const T d[6], T G03, T G04, T G13, T G14, T G25, T G43, T g0, T g1, T g2,
                                T g4) {
  // wv = C d, a = d^T C d, v = G wv
  T wv[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < 6; ++j) acc += c[sym(i, j)] * d[j];
    wv[i] = acc;
  }
  T a = T(0);
#pragma unroll
  for (int i = 0; i < 6; ++i) a += d[i] * wv[i];
  T v[6];
  v[0] = wv[0] + G03 * wv[3] + G04 * wv[4];
  v[1] = wv[1] + G13 * wv[3] + G14 * wv[4];
  v[2] = wv[2] + G25 * wv[5];
  v[3] = wv[3];
  v[4] = G43 * wv[3] + wv[4];
  v[5] = wv[5];
  // M = G C (rows), then N = M G^T (lower triangle)
  T M[6][6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    M[0][j] = c[sym(0, j)] + G03 * c[sym(3, j)] + G04 * c[sym(4, j)];
    M[1][j] = c[sym(1, j)] + G13 * c[sym(3, j)] + G14 * c[sym(4, j)];
    M[2][j] = c[sym(2, j)] + G25 * c[sym(5, j)];
    M[3][j] = c[sym(3, j)];
    M[4][j] = G43 * c[sym(3, j)] + c[sym(4, j)];
    M[5][j] = c[sym(5, j)];
  }
  T N[21];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    N[sym(i, 0)] = M[i][0] + G03 * M[i][3] + G04 * M[i][4];
    if (i >= 1) N[sym(i, 1)] = M[i][1] + G13 * M[i][3] + G14 * M[i][4];
    if (i >= 2) N[sym(i, 2)] = M[i][2] + G25 * M[i][5];
    if (i >= 3) N[sym(i, 3)] = M[i][3];
    if (i >= 4) N[sym(i, 4)] = G43 * M[i][3] + M[i][4];
    if (i >= 5) N[sym(i, 5)] = M[i][5];
  }
  // C' = N + g v^T + v g^T + a g g^T ; g = (g0, g1, g2, 0, g4, 0)
  const T gg[6] = {g0, g1, g2, T(0), g4, T(0)};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      c[sym(i, j)] = N[sym(i, j)] + gg[i] * v[j] + v[i] * gg[j] + a * gg[i] * gg[j];
    }
  }
}

// Intermediates of one propagation, recorded for the reverse pass.
template <typename T>
struct PropTape {
  T s, w, dw_dipt, sphi, cphi, sth, cth, isth, cot, f1, f2, dxdw, dydw;
  T G03, G04, G13, G14, G25, G43, inv;
  T d[6];
  HelixPt<T> hp;
};

// Propagate (p, c) to the surface (kind, pos) and add its scattering noise.
// Returns false (p, c untouched) if there is no admissible crossing.  If
// `tape` is given, the intermediates needed by the reverse pass are stored.
// The hook propagate() calls with the state on the surface just before the
// layer's material is added (the default does nothing).
struct NoPreMaterial {
  template <typename T>
  KF_HD void operator()(const T*, const T*) const {}
};

template <typename T, typename PreMaterial = NoPreMaterial>
KF_HD bool propagate(T p[6], T c[21], int q, int kind, T pos, T x_over_x0, bool same, bool material, T bz,
                     T mass, uint32_t& st, T* path = nullptr, PropTape<T>* tape = nullptr,
                     const PreMaterial& pre = PreMaterial()) {
  const T dw_dipt = -T(q) * T(kCLight) * bz;
  const T w = dw_dipt * p[3];
  T sphi, cphi, sth, cth;
  k_sincos(p[4], &sphi, &cphi);
  k_sincos(p[5], &sth, &cth);
  const T isth = k_rcp(sth);
  const T cot = cth * isth;
  T s;
  HelixPt<T> hp;
  if (!crossing(p, sphi, cphi, cot, w, kind, pos, same, s, hp)) {
    st |= TRK_NO_CROSSING;
    return false;
  }
  if (path) *path = s;
  const T x = hp.x, y = hp.y, sphm = hp.sphm, cphm = hp.cphm;
  const T u = hp.u;
  // helix partials at fixed s (G), with the chord-form derivatives
  const T f1 = u_minus_sin_over_u2(u);
  const T f2 = T(0.5) * hp.shc * hp.shc;   // (1 - cos u)/u^2
  const T s2 = s * s;
  const T dxdw = s2 * (cphm * f1 - sphm * f2);
  const T dydw = s2 * (sphm * f1 + cphm * f2);
  const T G03 = dxdw * dw_dipt, G04 = -hp.dy;
  const T G13 = dydw * dw_dipt, G14 = hp.dx;
  const T G25 = -s * isth * isth;
  const T G43 = s * dw_dipt;
  // ds/dp = -(dh/dp)/(dh/ds)
  T d[6];
  if (kind == 0) {
    const T inv = -k_rcp(x * cphm + y * sphm);
    d[0] = x * inv;
    d[1] = y * inv;
    d[2] = T(0);
    d[3] = (x * G03 + y * G13) * inv;
    d[4] = (x * G04 + y * G14) * inv;
    d[5] = T(0);
  } else {
    const T inv = -k_rcp(cot);
    d[0] = T(0);
    d[1] = T(0);
    d[2] = inv;
    d[3] = T(0);
    d[4] = T(0);
    d[5] = G25 * inv;
  }
  if (tape) {
    tape->s = s;
    tape->w = w;
    tape->dw_dipt = dw_dipt;
    tape->sphi = sphi;
    tape->cphi = cphi;
    tape->sth = sth;
    tape->cth = cth;
    tape->isth = isth;
    tape->cot = cot;
    tape->f1 = f1;
    tape->f2 = f2;
    tape->dxdw = dxdw;
    tape->dydw = dydw;
    tape->G03 = G03;
    tape->G04 = G04;
    tape->G13 = G13;
    tape->G14 = G14;
    tape->G25 = G25;
    tape->G43 = G43;
#pragma unroll
    for (int i = 0; i < 6; ++i) tape->d[i] = d[i];
    tape->inv = (kind == 0) ? -k_rcp(x * cphm + y * sphm) : -k_rcp(cot);
    tape->hp = hp;
  }
  transport_cov(c, d, G03, G04, G13, G14, G25, G43, cphm, sphm, cot, w);
  // The exact C' has the surface normal n (in position) as a null vector: a
  // state confined to the surface cannot move along n.  Rounding in the
  // cancellation F = G + g d^T leaves a residue of order eps * (G C G^T) there,
  // so the null vector is imposed: disk -> z row/column zero; barrel -> the
  // radial direction is projected out, C <- (I - n n^T) C (I - n n^T).
  const T rinv = k_rcp(pos);
  if (kind == 1) {
#pragma unroll
    for (int j = 0; j < 6; ++j) c[sym(2, j)] = T(0);
  } else {
    const T nx = x * rinv, ny = y * rinv;
    T cn[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) cn[i] = c[sym(i, 0)] * nx + c[sym(i, 1)] * ny;
    const T nn = cn[0] * nx + cn[1] * ny;
    const T nv[6] = {nx, ny, T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j) c[sym(i, j)] += -cn[i] * nv[j] - nv[i] * cn[j] + nn * nv[i] * nv[j];
  }
  p[0] = x;
  p[1] = y;
  p[2] = hp.z;
  p[4] = wrap_phi(hp.phi);
  pre(p, c);
  if (material) {
    // Highland angle at the propagated state; x/X0 scaled by 1/|cos(incidence)|
    const T ca = (kind == 0) ? k_abs(sth * (cphm * x + sphm * y) * rinv) : k_abs(cth);
    const T var = highland_var(p[3], sth, ca, x_over_x0, mass, st);
    add_q(c, p[3], sth, cot, var);
  }
  return true;
}

// Material of a layer added at the current state (the seed's own layer).
template <typename T>
KF_HD void add_material_here(const T p[6], T c[21], int kind, T x_over_x0, T mass, uint32_t& st) {
  T sth, cth;
  k_sincos(p[5], &sth, &cth);
  T ca;
  if (kind == 0) {
    T sph, cph;
    k_sincos(p[4], &sph, &cph);
    const T r = k_sqrt(p[0] * p[0] + p[1] * p[1]);
    ca = k_abs(sth * (cph * p[0] + sph * p[1]) * k_rcp(r));
  } else {
    ca = k_abs(cth);
  }
  const T var = highland_var(p[3], sth, ca, x_over_x0, mass, st);
  add_q(c, p[3], sth, cth * k_rcp(sth), var);
}

// ---- a4/a5: residual covariance inverse, chi2, gain, Joseph update ----------

// Inverse of a symmetric 3x3 (packed) by cofactors; returns the determinant.
template <typename T>
KF_HD inline T inv3(const T S[6], T I[6]) {
  const T a = S[0], b = S[1], cc = S[2], d = S[3], e = S[4], f = S[5];
  const T i00 = cc * f - e * e;
  const T i10 = d * e - b * f;
  const T i11 = a * f - d * d;
  const T i20 = b * e - cc * d;
  const T i21 = b * d - a * e;
  const T i22 = a * cc - b * b;
  const T det = a * i00 + b * i10 + d * i20;
  const T r = k_rcp(det);
  I[0] = i00 * r;
  I[1] = i10 * r;
  I[2] = i11 * r;
  I[3] = i20 * r;
  I[4] = i21 * r;
  I[5] = i22 * r;
  return det;
}

template <typename T>
KF_HD inline T norm_inf3(const T S[6]) {
  const T r0 = k_abs(S[0]) + k_abs(S[1]) + k_abs(S[3]);
  const T r1 = k_abs(S[1]) + k_abs(S[2]) + k_abs(S[4]);
  const T r2 = k_abs(S[3]) + k_abs(S[4]) + k_abs(S[5]);
  const T m01 = r0 > r1 ? r0 : r1;
  return m01 > r2 ? m01 : r2;
}

template <typename T>
KF_HD inline void inverse_checked(const T S[6], T Si[6], uint32_t& st);

template <>
KF_HD inline void inverse_checked<double>(const double S[6], double Si[6], uint32_t& st) {
  inv3(S, Si);
}

template <>
KF_HD inline void inverse_checked<float>(const float S[6], float Si[6], uint32_t& st) {
  const float det = inv3(S, Si);
  const float kappa = norm_inf3(S) * norm_inf3(Si);
  if (!(det > 0.f) || !(kappa <= float(kKappaMax))) {
    double Sd[6], Id[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) Sd[i] = double(S[i]);
    inv3(Sd, Id);
#pragma unroll
    for (int i = 0; i < 6; ++i) Si[i] = float(Id[i]);
    st |= TRK_FP64_FALLBACK;
  }
}

// Kalman update with hit m (3) and covariance V (packed 3x3), in type T.
template <typename T>
KF_HD void update_core(T p[6], T c[21], int& q, const T m[3], const T V[6], T& chi2, uint32_t& st) {
  const T tr_prior = c[0] + c[2] + c[5];
  T S[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) S[sym(i, j)] = c[sym(i, j)] + V[sym(i, j)];
  T Si[6];
  inverse_checked<T>(S, Si, st);
  const T r[3] = {m[0] - p[0], m[1] - p[1], m[2] - p[2]};
  T Sr[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Sr[i] = Si[sym(i, 0)] * r[0] + Si[sym(i, 1)] * r[1] + Si[sym(i, 2)] * r[2];
  chi2 = r[0] * Sr[0] + r[1] * Sr[1] + r[2] * Sr[2];
  // K = C[:, 0:3] S^-1
  T K[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      K[i][j] = c[sym(i, 0)] * Si[sym(0, j)] + c[sym(i, 1)] * Si[sym(1, j)] + c[sym(i, 2)] * Si[sym(2, j)];
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] += K[i][0] * r[0] + K[i][1] * r[1] + K[i][2] * r[2];
  if constexpr (std::is_same<T, float>::value) {
    // The Joseph form (I - K H) C (I - K H)^T + K V K^T, expanded: with
    // B = C H^T (the first three columns of C) and S = H C H^T + V it equals
    // C - K B^T - B K^T + K S K^T = C - K B^T - E K^T, E = B - K S, for any
    // gain K.  E vanishes for the exact optimal gain and carries the rounding
    // of K, which so enters C' at second order only, as in the factored
    // form.  B is copied first (C is overwritten in place).
    T B[6][3], E[6][3];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) B[i][k] = c[sym(i, k)];
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        T e = B[i][k];
        e = e - K[i][0] * S[sym(0, k)];
        e = e - K[i][1] * S[sym(1, k)];
        e = e - K[i][2] * S[sym(2, k)];
        E[i][k] = e;
      }
#pragma unroll
    for (int j = 0; j < 6; ++j)
#pragma unroll
      for (int i = j; i < 6; ++i) {
        T v = c[sym(i, j)];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          v = v - K[i][k] * B[j][k];
          v = v - E[i][k] * K[j][k];
        }
        c[sym(i, j)] = v;
      }
  } else {
  // Joseph form C' = A C A^T + K V K^T with A = I - K H, column by column:
  // (A C)_ij = c_ij - sum_k K_ik c_kj, C'_ij = (A C)_ij - sum_k (A C)_ik K_jk + (K V)_i . K_j.
  // Only (A C)[:, 0:3], K and K V stay live; columns are done from the last
  // to the first so that every c entry is read before it is overwritten.
  T AC3[6][3], KV[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      AC3[i][k] = c[sym(i, k)] - K[i][0] * c[sym(0, k)] - K[i][1] * c[sym(1, k)] - K[i][2] * c[sym(2, k)];
      KV[i][k] = K[i][0] * V[sym(0, k)] + K[i][1] * V[sym(1, k)] + K[i][2] * V[sym(2, k)];
    }
#pragma unroll
  for (int j = 5; j >= 0; --j)
#pragma unroll
    for (int i = 5; i >= j; --i) {
      T acij;
      if (j < 3) {
        acij = AC3[i][j];
      } else {
        acij = c[sym(i, j)] - K[i][0] * c[sym(0, j)] - K[i][1] * c[sym(1, j)] - K[i][2] * c[sym(2, j)];
      }
      const T aca = acij - AC3[i][0] * K[j][0] - AC3[i][1] * K[j][1] - AC3[i][2] * K[j][2];
      const T kvk = KV[i][0] * K[j][0] + KV[i][1] * K[j][1] + KV[i][2] * K[j][2];
      c[sym(i, j)] = aca + kvk;
    }
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

// The same update in FP64 for one FP32 lane, with fewer live values: the
// Joseph form expanded element by element, (I-KH) C (I-KH)^T + K V K^T =
// C - K B^T - B K^T + K S K^T with B = C H^T (it holds for any K), so only K,
// S and the packed C are kept.
KF_HD inline void update_lane_fp64(float p[6], float c[21], int& q, const float m[3], const float V[6], float& chi2,
                                   uint32_t& st) {
  const float tr_prior = c[0] + c[2] + c[5];
  double S[6], Si[6];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) S[sym(i, j)] = double(c[sym(i, j)]) + double(V[sym(i, j)]);
  inv3(S, Si);
  const double r[3] = {double(m[0]) - p[0], double(m[1]) - p[1], double(m[2]) - p[2]};
  double K[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      K[i][k] = double(c[sym(i, 0)]) * Si[sym(0, k)] + double(c[sym(i, 1)]) * Si[sym(1, k)] +
                double(c[sym(i, 2)]) * Si[sym(2, k)];
  double c2 = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) c2 += r[i] * (Si[sym(i, 0)] * r[0] + Si[sym(i, 1)] * r[1] + Si[sym(i, 2)] * r[2]);
  chi2 = float(c2);
  // entry (i, j) of C' needs c(i, j) and rows i, j of B = C[:, 0:3]: B is
  // copied first, then C is overwritten in place
  float B[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) B[i][k] = c[sym(i, k)];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double KSj[3];   // row j of K S
#pragma unroll
    for (int k = 0; k < 3; ++k) KSj[k] = K[j][0] * S[sym(0, k)] + K[j][1] * S[sym(1, k)] + K[j][2] * S[sym(2, k)];
#pragma unroll
    for (int i = j; i < 6; ++i) {
      double v = double(c[sym(i, j)]);
#pragma unroll
      for (int k = 0; k < 3; ++k) v += -K[i][k] * double(B[j][k]) - double(B[i][k]) * K[j][k] + K[i][k] * KSj[k];
      c[sym(i, j)] = float(v);
    }
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = float(double(p[i]) + K[i][0] * r[0] + K[i][1] * r[1] + K[i][2] * r[2]);
  if (p[3] < 0.f) {
    p[3] = -p[3];
    q = -q;
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (j != 3) c[sym(3, j)] = -c[sym(3, j)];
    st |= TRK_CHARGE_FLIP;
  }
  p[4] = wrap_phi(p[4]);
  const float tr = c[0] + c[2] + c[5];
  const float tol = 1e-3f * tr + float(kPsdUlps * kEpsF32) * tr_prior;
  if (!(c[sym(3, 3)] > 0.f) || !(c[sym(4, 4)] > 0.f) || !(c[sym(5, 5)] > 0.f) || c[0] < -tol || c[2] < -tol ||
      c[5] < -tol)
    st |= TRK_COV_NOT_PSD;
  st |= TRK_FP64_FALLBACK;
}

// Kalman update.  The FP32 form moves a lane to FP64 when the prior position
// variance exceeds the hit variance by more than kRatioMax in some direction
// (then the FP32 posterior would keep fewer than ~3 significant digits).  The
// largest such ratio is the largest eigenvalue of V^-1 C_pos, bounded above by
// its trace tr(V^-1 C_pos) (at most three times it), which is what is tested:
// comparing the variances axis by axis misses a prior that is wide along the
// hit's most precise direction when that direction is not a coordinate axis
// (a barrel hit's r-phi direction, where V_xx and V_yy also carry the larger
// thickness term).
template <typename T>
KF_HD void update(T p[6], T c[21], int& q, const T m[3], const T V[6], T& chi2, uint32_t& st) {
  if constexpr (std::is_same<T, float>::value) {
    // cofactors of V (its inverse up to 1/det, det > 0 for a valid hit covariance)
    const float a = V[0], b = V[1], cc = V[2], d = V[3], e = V[4], f = V[5];
    const float i00 = cc * f - e * e, i10 = d * e - b * f, i11 = a * f - d * d;
    const float i20 = b * e - cc * d, i21 = b * d - a * e, i22 = a * cc - b * b;
    const float det = a * i00 + b * i10 + d * i20;
    const float tr = i00 * c[0] + i11 * c[2] + i22 * c[5] + 2.f * (i10 * c[1] + i20 * c[3] + i21 * c[4]);
    if (!(tr <= float(kRatioMax) * det)) {   // also a non-finite or degenerate V
      update_lane_fp64(p, c, q, m, V, chi2, st);
      return;
    }
  }
  update_core<T>(p, c, q, m, V, chi2, st);
}

template <typename T>
KF_HD inline bool all_finite(const T p[6], const T c[21], T chi2) {
  bool ok = k_finite(chi2);
#pragma unroll
  for (int i = 0; i < 6; ++i) ok = ok && k_finite(p[i]);
#pragma unroll
  for (int i = 0; i < 21; ++i) ok = ok && k_finite(c[i]);
  return ok;
}

// ---- seeding from three hits -------------------------------------------------

template <typename T>
KF_HD void seed_from_hits(const T h1[3], const T h2[3], const T h3[3], T bz, T p[6], int& q) {
  const T dx12 = h2[0] - h1[0], dy12 = h2[1] - h1[1];
  const T dx13 = h3[0] - h1[0], dy13 = h3[1] - h1[1];
  const T dx23 = h3[0] - h2[0], dy23 = h3[1] - h2[1];
  const T d12 = k_sqrt(dx12 * dx12 + dy12 * dy12);
  const T d13 = k_sqrt(dx13 * dx13 + dy13 * dy13);
  const T d23 = k_sqrt(dx23 * dx23 + dy23 * dy23);
  const T cr = dx12 * dy13 - dy12 * dx13;
  const T kappa = T(2) * cr / (d12 * d13 * d23);
  q = kappa > T(0) ? -1 : 1;
  const T ak = k_abs(kappa);
  p[0] = h1[0];
  p[1] = h1[1];
  p[2] = h1[2];
  p[3] = ak / (T(kCLight) * bz);
  // half turning angle to hit 2: asin(kappa d12/2) = atan2(k, sqrt(1-k^2))
  T a12 = kappa * d12 * T(0.5);
  a12 = a12 < T(-1) ? T(-1) : (a12 > T(1) ? T(1) : a12);
  const T half = k_atan2(a12, k_sqrt((T(1) - a12) * (T(1) + a12)));
  p[4] = wrap_phi(k_atan2(dy12, dx12) - half);
  // transverse arc 1 -> 3: 2 asin(|kappa| d13/2)/|kappa| = d13 * asin(x)/x
  T a13 = ak * d13 * T(0.5);
  a13 = a13 > T(1) ? T(1) : a13;
  T asin_over;
  if (a13 < T(0.05)) {
    const T x2 = a13 * a13;
    asin_over = T(1) + x2 * (T(1.0 / 6.0) + x2 * (T(3.0 / 40.0) + x2 * T(5.0 / 112.0)));
  } else {
    asin_over = k_atan2(a13, k_sqrt((T(1) - a13) * (T(1) + a13))) / a13;
  }
  const T s13 = d13 * asin_over;
  const T cot = (h3[2] - h1[2]) / s13;
  p[5] = T(kPi * 0.5) - k_atan(cot);
}

}  // namespace kf
