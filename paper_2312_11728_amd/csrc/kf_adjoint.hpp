// Hand-written reverse pass of the forward fit: the gradient of
// L = sum_t w_t chi2_t with respect to the seed states and the hit positions.
//
// The sweep runs over a track's entries from the last to the first.  The
// state entering each entry is recomputed from the nearest checkpoint written
// by the forward fit (every `seg` entries), and each entry's adjoint is the
// reverse of its three parts:
//   update     p' = p + K r, C' = C - K H C (the Joseph form has the same
//              derivative at the optimal gain), chi2 = r^T S^-1 r
//   material   C += Q(p)
//   transport  p' = g(p), C' = F(p) C F(p)^T with F = G + g_s d^T, where the
//              path length s(p) enters through the implicit-function rule
//              ds/dp = d, so the root solve itself is not differentiated.
// Symmetric-matrix adjoints are kept as symmetric full matrices (dL =
// sum_ij Cb_ij dC_ij over all 36 entries), stored packed.
#pragma once

#include "kf_track.hpp"

namespace kf {

template <typename T, typename U>
KF_HD inline void unpack6(const T c[21], U C[6][6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) C[i][j] = c[sym(i, j)];
}

// packed symmetric adjoint of a full (not necessarily symmetric) adjoint
template <typename T>
KF_HD inline void pack6_sym(const T A[6][6], T c[21]) {
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) c[sym(i, j)] = T(0.5) * (A[i][j] + A[j][i]);
}

// Gradient of <Cb, Q(p)> (Cb symmetric full-matrix adjoint, packed) with
// respect to p, added to pb.  Q as in add_q / highland_var; `seed` selects
// the incidence of the seed's own layer (radius from the position) instead of
// the crossing formula (radius = the layer radius, 1/R = rinv).
template <typename T>
KF_HD inline void q_grad(const T p[6], int kind, T x_over_x0, T mass, bool seed, T rinv, const T cb[21], T pb[6]) {
  T sph, cph, sth, cth;
  k_sincos(p[4], &sph, &cph);
  k_sincos(p[5], &sth, &cth);
  const T isth = T(1) / sth;
  const T cot = cth * isth;
  const T ipt = p[3];
  const T x = p[0], y = p[1];
  T A = cph * x + sph * y, r = T(0), ir = rinv;
  if (seed && kind == 0) {
    r = k_sqrt(x * x + y * y);
    ir = T(1) / r;
  }
  const T ca_raw = (kind == 0) ? sth * A * ir : cth;
  T ca = k_abs(ca_raw);
  const bool clamped = ca < T(kGrazingCos);
  if (clamped) ca = T(kGrazingCos);
  const T mis = mass * ipt * sth;
  const T one_m = T(1) + mis * mis;
  const T xl = x_over_x0 / ca;
  const T sq = k_sqrt(xl);
  const T sqm = k_sqrt(one_m);
  const T Lg = T(1) + T(0.038) * k_log(xl * one_m);
  const T inv_bp = ipt * sth * sqm;
  const T th0 = T(0.0136) * inv_bp * sq * Lg;
  const T var = th0 * th0;
  const T ic = ipt * cot;
  const T b33 = cb[sym(3, 3)], b53 = cb[sym(5, 3)], b44 = cb[sym(4, 4)], b55 = cb[sym(5, 5)];
  // Phi = b33 ic^2 var - 2 b53 ic var + b44 var isth^2 + b55 var
  const T bvar = b33 * ic * ic - T(2) * b53 * ic + b44 * isth * isth + b55;
  const T bic = T(2) * b33 * ic * var - T(2) * b53 * var;
  T bisth = T(2) * b44 * var * isth;
  T bipt = bic * cot;
  T bcot = bic * ipt;
  const T bth0 = T(2) * th0 * bvar;
  const T binv_bp = bth0 * T(0.0136) * sq * Lg;
  const T bsq = bth0 * T(0.0136) * inv_bp * Lg;
  const T bL = bth0 * T(0.0136) * inv_bp * sq;
  T bxl = bL * T(0.038) / xl + bsq / (T(2) * sq);
  T bone = bL * T(0.038) / one_m;
  bipt += binv_bp * sth * sqm;
  T bsth = binv_bp * ipt * sqm;
  bone += binv_bp * ipt * sth / (T(2) * sqm);
  const T bmis = bone * T(2) * mis;
  bipt += bmis * mass * sth;
  bsth += bmis * mass * ipt;
  const T bca = clamped ? T(0) : -bxl * x_over_x0 / (ca * ca);
  const T bca_raw = ca_raw < T(0) ? -bca : bca;
  T bcth = T(0), bph = T(0), bx = T(0), by = T(0);
  if (kind == 0) {
    // ca_raw = sth A ir, A = cph x + sph y; for the seed ir = 1/sqrt(x^2 + y^2)
    bsth += bca_raw * A * ir;
    const T bA = bca_raw * sth * ir;
    bx += bA * cph;
    by += bA * sph;
    bph += bA * (-sph * x + cph * y);
    if (seed) {
      const T bir = bca_raw * sth * A;
      // ir = (x^2 + y^2)^(-1/2)
      const T dr = -bir * ir * ir * ir;
      bx += dr * x;
      by += dr * y;
    }
  } else {
    bcth += bca_raw;
  }
  // cot = cth isth, isth = 1/sth
  bcth += bcot * isth;
  bisth += bcot * cth;
  bsth += -bisth * isth * isth;
  pb[0] += bx;
  pb[1] += by;
  pb[3] += bipt;
  pb[4] += bph;
  pb[5] += bsth * cth - bcth * sth;
}

// Contribution of <Fb, F(p, s(p))> to pb (total derivative: partials at
// fixed s plus (d/ds) * ds/dp with ds/dp = tape.d).
template <typename T>
KF_HD inline void jacobian_grad(const PropTape<T>& tp, int kind, const T Fb[6][6], T pb[6]) {
  const HelixPt<T>& hp = tp.hp;
  const T s = tp.s, w = tp.w, dwi = tp.dw_dipt, cot = tp.cot, isth = tp.isth, sth = tp.sth, cth = tp.cth;
  const T x = hp.x, y = hp.y, sphm = hp.sphm, cphm = hp.cphm, u = hp.u, shc = hp.shc, ch = hp.ch;
  const T smid = hp.smid, cmid = hp.cmid;
  const T f1 = tp.f1, f2 = tp.f2, inv = tp.inv;
  const T gv[6] = {cphm, sphm, cot, T(0), w, T(0)};
  T bG03 = Fb[0][3], bG04 = Fb[0][4], bG13 = Fb[1][3], bG14 = Fb[1][4], bG25 = Fb[2][5], bG43 = Fb[4][3];
  T bg[6], bd[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    T acc = T(0);
#pragma unroll
    for (int b = 0; b < 6; ++b) acc += Fb[a][b] * tp.d[b];
    bg[a] = acc;
  }
#pragma unroll
  for (int b = 0; b < 6; ++b) {
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 6; ++a) acc += Fb[a][b] * gv[a];
    bd[b] = acc;
  }
  T bcphm = bg[0], bsphm = bg[1], bcot = bg[2], bw = bg[4];
  T bx = T(0), by = T(0), bs = T(0), bisth = T(0), bsth = T(0), bcth = T(0), bu = T(0), bdx = T(0), bdy = T(0);
  if (kind == 0) {
    const T v3 = x * tp.G03 + y * tp.G13, v4 = x * tp.G04 + y * tp.G14;
    const T binv = bd[0] * x + bd[1] * y + bd[3] * v3 + bd[4] * v4;
    const T bv0 = bd[0] * inv, bv1 = bd[1] * inv, bv3 = bd[3] * inv, bv4 = bd[4] * inv;
    bx += bv0 + bv3 * tp.G03 + bv4 * tp.G04;
    by += bv1 + bv3 * tp.G13 + bv4 * tp.G14;
    bG03 += bv3 * x;
    bG13 += bv3 * y;
    bG04 += bv4 * x;
    bG14 += bv4 * y;
    // inv = -1/den, den = x cphm + y sphm
    const T bden = binv * inv * inv;
    bx += bden * cphm;
    by += bden * sphm;
    bcphm += bden * x;
    bsphm += bden * y;
  } else {
    // d2 = inv, d5 = G25 inv, inv = -1/cot
    const T binv = bd[2] + bd[5] * tp.G25;
    bG25 += bd[5] * inv;
    bcot += binv * inv * inv;
  }
  // G03 = dxdw dwi, G13 = dydw dwi, G04 = -dy, G14 = dx, G25 = -s isth^2, G43 = s dwi
  const T bdxdw = bG03 * dwi, bdydw = bG13 * dwi;
  bdy -= bG04;
  bdx += bG14;
  bs += -bG25 * isth * isth + bG43 * dwi;
  bisth += -bG25 * T(2) * s * isth;
  // dxdw = s^2 (cphm f1 - sphm f2), dydw = s^2 (sphm f1 + cphm f2)
  const T s2 = s * s;
  bs += bdxdw * T(2) * s * (cphm * f1 - sphm * f2) + bdydw * T(2) * s * (sphm * f1 + cphm * f2);
  bcphm += bdxdw * s2 * f1 + bdydw * s2 * f2;
  bsphm += -bdxdw * s2 * f2 + bdydw * s2 * f1;
  const T bf1 = bdxdw * s2 * cphm + bdydw * s2 * sphm;
  const T bf2 = -bdxdw * s2 * sphm + bdydw * s2 * cphm;
  // f2 = shc^2 / 2; f1'(u) = f2 - 2 f1 / u
  T bshc = bf2 * shc;
  const T df1 = k_abs(u) < T(1e-3) ? T(1.0 / 6.0) - u * u * T(1.0 / 40.0) : f2 - T(2) * f1 / u;
  bu += bf1 * df1;
  // x = x0 + dx, y = y0 + dy
  const T bx0 = bx, by0 = by;
  bdx += bx;
  bdy += by;
  // dx = s cmid shc, dy = s smid shc
  bs += bdx * cmid * shc + bdy * smid * shc;
  const T bcmid = bdx * s * shc, bsmid = bdy * s * shc;
  bshc += bdx * s * cmid + bdy * s * smid;
  // (sphm, cphm) = sin, cos (phi0 + u); (smid, cmid) = sin, cos (phi0 + u/2)
  const T bphim = bsphm * cphm - bcphm * sphm;
  const T bphimid = bsmid * cmid - bcmid * smid;
  const T bphi0 = bphim + bphimid;
  bu += bphim;
  T bh = bphimid;
  const T h = T(0.5) * u;
  const T dsinc = k_abs(h) < T(1e-2) ? -h * T(1.0 / 3.0) + h * h * h * T(1.0 / 30.0) : (ch - shc) / h;
  bh += bshc * dsinc;
  bu += T(0.5) * bh;
  // u = w s, w = dwi ipt
  bw += bu * s;
  bs += bu * w;
  const T bipt = bw * dwi;
  // cot = cth isth, isth = 1/sth
  bcth += bcot * isth;
  bisth += bcot * cth;
  bsth += -bisth * isth * isth;
  const T btheta = bsth * cth - bcth * sth;
  pb[0] += bx0 + bs * tp.d[0];
  pb[1] += by0 + bs * tp.d[1];
  pb[2] += bs * tp.d[2];
  pb[3] += bipt + bs * tp.d[3];
  pb[4] += bphi0 + bs * tp.d[4];
  pb[5] += btheta + bs * tp.d[5];
}

// Reverse of the update (computed in U), given the predicted state pp, its
// covariance C (full), the aligned hit m and V.  In: pb, Gb = adjoints of the
// updated state/covariance (after the charge flip, if it happened).  Out: pb,
// Gb = adjoints of the predicted state/covariance; mb = adjoint of m.
template <typename U>
KF_HD inline void update_vjp(const U pp[6], const U C[6][6], const U m[3], const U V[6], U wchi, U pb[6], U Gb[6][6],
                             U mb[3]) {
  U S[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) S[k][l] = C[k][l] + V[sym(k, l)];
  U Sp[6] = {S[0][0], S[1][0], S[1][1], S[2][0], S[2][1], S[2][2]}, Ip[6];
  uint32_t ist = 0;
  inverse_checked<U>(Sp, Ip, ist);
  U Si[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) Si[k][l] = Ip[sym(k, l)];
  const U r[3] = {m[0] - pp[0], m[1] - pp[1], m[2] - pp[2]};
  U K[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) K[i][k] = C[i][0] * Si[0][k] + C[i][1] * Si[1][k] + C[i][2] * Si[2][k];
  // flip (sign of the updated ipt) is decided by the caller
  U Sir[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) Sir[k] = Si[k][0] * r[0] + Si[k][1] * r[1] + Si[k][2] * r[2];
  U Kb[6][3], rb[3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) Kb[i][k] = pb[i] * r[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    U acc = U(2) * wchi * Sir[k];
#pragma unroll
    for (int i = 0; i < 6; ++i) acc += K[i][k] * pb[i];
    rb[k] = acc;
  }
  // GK = Gb K (6x3), used for B-bar and Si-bar
  U GK[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      U acc = U(0);
#pragma unroll
      for (int j = 0; j < 6; ++j) acc += Gb[i][j] * K[j][k];
      GK[i][k] = acc;
    }
  // Sib = wchi r r^T + B^T Kb - B^T Gb B  (B = C[:, 0:3])
  U Sib[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      U acc = wchi * r[k] * r[l];
#pragma unroll
      for (int i = 0; i < 6; ++i) acc += C[i][k] * Kb[i][l];
      U bgb = U(0);
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        U gbl = U(0);
#pragma unroll
        for (int j = 0; j < 6; ++j) gbl += Gb[i][j] * C[j][l];
        bgb += C[i][k] * gbl;
      }
      Sib[k][l] = acc - bgb;
    }
  // Bb = Kb Si - 2 Gb K
  U Bb[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k)
      Bb[i][k] = Kb[i][0] * Si[0][k] + Kb[i][1] * Si[1][k] + Kb[i][2] * Si[2][k] - U(2) * GK[i][k];
  // Sb = -Si Sib Si
  U T1[3][3], Sb[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) T1[k][l] = Sib[k][0] * Si[0][l] + Sib[k][1] * Si[1][l] + Sib[k][2] * Si[2][l];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) Sb[k][l] = -(Si[k][0] * T1[0][l] + Si[k][1] * T1[1][l] + Si[k][2] * T1[2][l]);
  // C-bar = Gb + embed(Sb) + embed(Bb), symmetrised
  U Cb[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) Cb[i][j] = Gb[i][j];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int l = 0; l < 3; ++l) Cb[k][l] += Sb[k][l];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int k = 0; k < 3; ++k) Cb[i][k] += Bb[i][k];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      const U v = U(0.5) * (Cb[i][j] + Cb[j][i]);
      Gb[i][j] = v;
      Gb[j][i] = v;
    }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    pb[k] -= rb[k];
    mb[k] = rb[k];
  }
}

// Intermediates of a propagation converted to the reverse pass's type.
template <typename U, typename T>
KF_HD inline PropTape<U> tape_as(const PropTape<T>& t) {
  PropTape<U> o;
  o.s = t.s;
  o.w = t.w;
  o.dw_dipt = t.dw_dipt;
  o.sphi = t.sphi;
  o.cphi = t.cphi;
  o.sth = t.sth;
  o.cth = t.cth;
  o.isth = t.isth;
  o.cot = t.cot;
  o.f1 = t.f1;
  o.f2 = t.f2;
  o.dxdw = t.dxdw;
  o.dydw = t.dydw;
  o.G03 = t.G03;
  o.G04 = t.G04;
  o.G13 = t.G13;
  o.G14 = t.G14;
  o.G25 = t.G25;
  o.G43 = t.G43;
  o.inv = t.inv;
#pragma unroll
  for (int i = 0; i < 6; ++i) o.d[i] = t.d[i];
  o.hp.x = t.hp.x;
  o.hp.y = t.hp.y;
  o.hp.z = t.hp.z;
  o.hp.phi = t.hp.phi;
  o.hp.sphm = t.hp.sphm;
  o.hp.cphm = t.hp.cphm;
  o.hp.dx = t.hp.dx;
  o.hp.dy = t.hp.dy;
  o.hp.u = t.hp.u;
  o.hp.sh = t.hp.sh;
  o.hp.ch = t.hp.ch;
  o.hp.shc = t.hp.shc;
  o.hp.smid = t.hp.smid;
  o.hp.cmid = t.hp.cmid;
  return o;
}

// Adjoint of one entry (see the file comment).  p_in, c_in, q_in: the state
// entering the entry (recomputed in the forward path's type T, so the
// transport, crossing and flip decisions are the forward's own); q_out: the
// charge after the entry (it differs from q_in iff the update flipped it);
// m_raw: the hit before alignment.  pb, cb: in, adjoints of the state leaving
// the entry; out, adjoints of the state entering it.  hb: adjoint of the raw
// hit position.  The reverse arithmetic runs in FP64 for both precisions: the
// covariance adjoint is of order 1/sigma^4 of the hits while the gradient
// with respect to the earlier states is of order one, so the products in the
// transport and update reverse cancel by five to six orders of magnitude,
// which FP32 cannot resolve.
template <typename T>
KF_HD inline void step_vjp(const T p_in[6], const T c_in[21], int q_in, int q_out, int j, int lay, int prev,
                           bool valid, const T m_raw[3], const T V[6], const TrackGeom<T>& g,
                           const T* __restrict__ sal, double wchi, double pb[6], double cb[21], double hb[3]) {
  using R = double;
  const int kind = g.kind[lay];
  T p[6], c[21];
#pragma unroll
  for (int i = 0; i < 6; ++i) p[i] = p_in[i];
#pragma unroll
  for (int i = 0; i < 21; ++i) c[i] = c_in[i];
  int q = q_in;
  uint32_t sst = 0;
  PropTape<T> tp;
  if (j > 0) {
    propagate(p, c, q, kind, g.pos[lay], g.x0[lay], lay == prev, true, g.bz, g.mass, sst, static_cast<T*>(nullptr),
              &tp);
  } else {
    add_material_here(p, c, kind, g.x0[lay], g.mass, sst);
  }
  // p, c: the predicted state and covariance (material included)
  R P[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) P[i] = p[i];
  hb[0] = hb[1] = hb[2] = R(0);
  R Gb[6][6];
  unpack6(cb, Gb);
  if (valid) {
    R m[3] = {m_raw[0], m_raw[1], m_raw[2]};
    R sa = R(0), ca = R(1);
    const bool al = sal && kind == 0;
    if (al) {
      T sat, cat;
      k_sincos(sal[lay] * k_rcp(g.pos[lay]), &sat, &cat);
      sa = sat;
      ca = cat;
      m[0] = ca * R(m_raw[0]) - sa * R(m_raw[1]);
      m[1] = sa * R(m_raw[0]) + ca * R(m_raw[1]);
      m[2] = R(m_raw[2]) + R(sal[kMaxLayers + lay]);
    }
    if (q_out != q) {
      // the update flipped the charge: ipt, q and row/column 3 changed sign
      pb[3] = -pb[3];
#pragma unroll
      for (int i = 0; i < 6; ++i)
        if (i != 3) {
          Gb[3][i] = -Gb[3][i];
          Gb[i][3] = -Gb[i][3];
        }
    }
    R C[6][6], Vd[6], mb[3];
    unpack6(c, C);
#pragma unroll
    for (int i = 0; i < 6; ++i) Vd[i] = V[i];
    update_vjp<R>(P, C, m, Vd, wchi, pb, Gb, mb);
    // m = R(a) h (barrel alignment): h-bar = R^T m-bar
    hb[0] = ca * mb[0] + sa * mb[1];
    hb[1] = -sa * mb[0] + ca * mb[1];
    hb[2] = mb[2];
  }
  // material: C_pred = C_prop + Q(p_pred)
  R cbp[21];
  pack6_sym(Gb, cbp);
  if (j > 0) {
    q_grad<R>(P, kind, R(g.x0[lay]), R(g.mass), false, R(1) / R(g.pos[lay]), cbp, pb);
    // transport: p = g(p_in), C_prop = F C_in F^T
    const PropTape<R> td = tape_as<R>(tp);
    R F[6][6];
    const R gv[6] = {td.hp.cphm, td.hp.sphm, td.cot, R(0), td.w, R(0)};
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) F[a][b] = (a == b ? R(1) : R(0)) + gv[a] * td.d[b];
    F[0][3] += td.G03;
    F[0][4] += td.G04;
    F[1][3] += td.G13;
    F[1][4] += td.G14;
    F[2][5] += td.G25;
    F[4][3] += td.G43;
    // GF = Gb F; C-bar_in = F^T Gb F; F-bar = 2 Gb F C_in
    R GF[6][6];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        R acc = R(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) acc += Gb[a][k] * F[k][b];
        GF[a][b] = acc;
      }
    R Fb[6][6];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) {
        R acc = R(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) acc += GF[a][k] * R(c_in[sym(k, b)]);
        Fb[a][b] = R(2) * acc;
      }
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b <= a; ++b) {
        R acc = R(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) acc += F[k][a] * GF[k][b];
        cb[sym(a, b)] = acc;
      }
    // p-bar_in = F^T p-bar + d<Fb, F>/dp
    R pbi[6];
#pragma unroll
    for (int b = 0; b < 6; ++b) {
      R acc = R(0);
#pragma unroll
      for (int a = 0; a < 6; ++a) acc += F[a][b] * pb[a];
      pbi[b] = acc;
    }
    jacobian_grad(td, kind, Fb, pbi);
#pragma unroll
    for (int i = 0; i < 6; ++i) pb[i] = pbi[i];
  } else {
    // the seed's own layer: C = C_in + Q(p_in), p unchanged
    R Pin[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) Pin[i] = p_in[i];
    q_grad<R>(Pin, kind, R(g.x0[lay]), R(g.mass), true, R(0), cbp, pb);
#pragma unroll
    for (int i = 0; i < 21; ++i) cb[i] = cbp[i];
  }
}

// State entering entry j (relative to the first valid entry k0) of track t:
// the seed for j = 0, else the checkpoint before entry 1 + m seg followed by
// the entries up to j - 1.  Also returns the layer of entry j - 1 (prev).
template <typename T, typename Acc>
KF_HD inline void state_before(const AdjArgs<T>& a, const TrackGeom<T>& g, const T* __restrict__ sal, int64_t t,
                               const Acc& acc, int k0, int j, T p[6], T c[21], int& q, int& prev) {
  const FitArgs<T>& f = a.f;
  const int64_t ld = f.ld;
  int jstart;
  if (j == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) p[i] = f.seed_state[i * ld + t];
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = f.seed_cov[i * ld + t];
    q = f.seed_charge[t];
    jstart = 0;
  } else {
    const int64_t cst = ld * int64_t(f.n_seg);
    const int mslot = (j - 1) / f.seg;
    const T* base = f.ckpt + int64_t(mslot) * ld + t;
#pragma unroll
    for (int i = 0; i < 6; ++i) p[i] = base[i * cst];
#pragma unroll
    for (int i = 0; i < 21; ++i) c[i] = base[(6 + i) * cst];
    q = int(base[27 * cst]);
    jstart = 1 + mslot * f.seg;
  }
  int lay;
  bool valid;
  T m[3], V[6];
  acc.load(k0 + (jstart > 0 ? jstart - 1 : 0), lay, valid, m, V);
  prev = lay;
  for (int jj = jstart; jj < j; ++jj) {
    acc.load(k0 + jj, lay, valid, m, V);
    T c2;
    uint32_t sst = 0;
    step_forward(p, c, q, jj, lay, prev, valid, m, V, g, sal, c2, sst);
    prev = lay;
  }
}

// With a state buffer: the states before entries js .. jhi (relative to the
// first valid entry k0, 1 <= js <= jhi) of track t, recomputed from the
// checkpoint of their segment in one pass and stored in slots js - 1 ..
// jhi - 1 ([slot][kSegVals][n]).
template <typename T, typename Acc>
KF_HD inline void fill_segment(const AdjArgs<T>& a, const TrackGeom<T>& g, const T* __restrict__ sal, int64_t t,
                               const Acc& acc, int k0, int js, int jhi) {
  const int64_t n = a.f.n;
  T p[6], c[21];
  int q, prev;
  state_before(a, g, sal, t, acc, k0, js, p, c, q, prev);
  for (int j = js;; ++j) {
    T* slot = a.seg_buf + int64_t(j - 1) * kSegVals * n + t;
#pragma unroll
    for (int i = 0; i < 6; ++i) slot[i * n] = p[i];
#pragma unroll
    for (int i = 0; i < 21; ++i) slot[(6 + i) * n] = c[i];
    slot[27 * n] = T(q);
    slot[28 * n] = T(prev);
    if (j == jhi) break;
    int lay;
    bool valid;
    T m[3], V[6];
    acc.load(k0 + j, lay, valid, m, V);
    T c2;
    uint32_t sst = 0;
    step_forward(p, c, q, j, lay, prev, valid, m, V, g, sal, c2, sst);
    prev = lay;
  }
}

// The states before entries 1 .. n_steps - 1 of track t (len entries) for
// the reverse pass, segment by segment, each from its own checkpoint: the
// same forward steps the reverse pass would take to reach each of them.
// This is the per-track form (host builds); the device kernel takes the same
// steps with the wave's hits staged through LDS.
template <typename T, typename Acc>
KF_HD inline void refill_track(const AdjArgs<T>& a, const TrackGeom<T>& g, const T* __restrict__ sal, int64_t t,
                               const Acc& acc, int len) {
  const FitArgs<T>& f = a.f;
  if (len > f.max_len) len = f.max_len;
  int k0 = 0;
  while (k0 < len && !acc.valid(k0)) ++k0;
  const int n_steps = len - k0;
  for (int js = 1; js < n_steps; js += f.seg) {
    const int jhi = js + f.seg - 1 < n_steps - 1 ? js + f.seg - 1 : n_steps - 1;
    fill_segment(a, g, sal, t, acc, k0, js, jhi);
  }
}

// Reverse sweep of track t (len entries, the first at e0 of the hit arrays),
// read through `acc`.
template <typename T, typename Acc>
KF_HD inline void adjoint_track(const AdjArgs<T>& a, const TrackGeom<T>& g, const T* __restrict__ sal, int64_t t,
                                const Acc& acc, int len, int64_t e0) {
  const FitArgs<T>& f = a.f;
  const int64_t ld = f.ld, nh = f.n_hits;
  // hit gradients of this track start at zero (holes, entries beyond max_len
  // and entries after a stop stay so)
  for (int k = 0; k < len; ++k) {
    a.grad_hit[e0 + k] = T(0);
    a.grad_hit[nh + e0 + k] = T(0);
    a.grad_hit[2 * nh + e0 + k] = T(0);
  }
  if (len > f.max_len) len = f.max_len;
  int k0 = 0;
  while (k0 < len && !acc.valid(k0)) ++k0;
  const int n_steps = len - k0;
  // entries the forward completed (it stops early on a failed crossing, a
  // non-finite step or a bad layer id) and the charge after the last one
  int n_done = n_steps;
  int q_end = 0;
  if (n_steps > 0) {
    const uint32_t stop = TRK_NO_CROSSING | TRK_NONFINITE | TRK_BAD_INPUT;
    const bool stopped = a.fwd_status && (a.fwd_status[t] & stop);
    T p[6], c[21];
    int q, prev;
    const int j0 = stopped ? 0 : n_steps - 1;
    state_before(a, g, sal, t, acc, k0, j0, p, c, q, prev);
    if (stopped) n_done = 0;
    q_end = q;
    for (int j = j0; j < n_steps; ++j) {
      int lay;
      bool valid;
      T m[3], V[6];
      acc.load(k0 + j, lay, valid, m, V);
      if (lay < 0 || lay >= g.n_layers) break;
      if (j == 0) prev = lay;
      T c2;
      uint32_t sst = 0;
      if (!step_forward(p, c, q, j, lay, prev, valid, m, V, g, sal, c2, sst)) break;
      if (!all_finite(p, c, c2)) break;
      prev = lay;
      q_end = q;
      if (stopped) n_done = j + 1;
    }
  }
  const double wchi = a.w ? double(a.w[t]) : 1.0;
  double pb[6], cb[21];
#pragma unroll
  for (int i = 0; i < 6; ++i) pb[i] = 0.0;
#pragma unroll
  for (int i = 0; i < 21; ++i) cb[i] = 0.0;
  int q_after = q_end;
  for (int j = n_done - 1; j >= 0; --j) {
    T p[6], c[21];
    int q, prev;
    if (a.seg_buf && j >= 1) {
      // recomputed by the refill pass
      const T* slot = a.seg_buf + int64_t(j - 1) * kSegVals * f.n + t;
#pragma unroll
      for (int i = 0; i < 6; ++i) p[i] = slot[i * f.n];
#pragma unroll
      for (int i = 0; i < 21; ++i) c[i] = slot[(6 + i) * f.n];
      q = int(slot[27 * f.n]);
      prev = int(slot[28 * f.n]);
    } else {
      state_before(a, g, sal, t, acc, k0, j, p, c, q, prev);
    }
    int lay;
    bool valid;
    T m[3], V[6];
    acc.load(k0 + j, lay, valid, m, V);
    if (j == 0) prev = lay;
    double hb[3];
    step_vjp(p, c, q, q_after, j, lay, prev, valid, m, V, g, sal, wchi, pb, cb, hb);
    if (valid) {
      const int64_t e = e0 + k0 + j;
      a.grad_hit[e] = T(hb[0]);
      a.grad_hit[nh + e] = T(hb[1]);
      a.grad_hit[2 * nh + e] = T(hb[2]);
    }
    q_after = q;
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) a.grad_seed[i * ld + t] = T(pb[i]);
}

}  // namespace kf
