"""FP64 CPU oracle for tilted planar modules.  TEST INFRASTRUCTURE: only the
tests, the smoke check and the benchmark's CPU-baseline leg may import this
module; it shares no code with the HIP kernels.

The paper (Sec. 3.1, the Phase-2 geometry) describes detector modules by a
position, a normal vector and a phi-direction vector, and names propagation
to such modules and Kalman updates on them as what the tilted Phase-2 layout
needs.  It gives no formulas.  The readings here:

* A module is a plane through its centre c with unit normal n; its local
  frame is u (the unit phi-direction, in the plane) and v = n x u.  A hit on
  the module is the pair of local coordinates (m_u, m_v) = ((x - c).u,
  (x - c).v) of its position x, with a 2x2 covariance.
* Propagation: the helix of kf_oracle.helix_at to the plane, the path s the
  first root s > -1 cm (the window of a different layer in kf_oracle) of
  h(s) = n.(x(s) - c) within one turn, found by steps that cannot pass a
  root (crossing_plane).  The Jacobian is the surface-to-surface derivative
  F = G + g_s (ds/dp), ds/dp = -(n.G_pos)/(n.g_pos), with G and g_s the
  helix partials of kf_oracle.helix_partials.  After it the plane normal (in
  position) is a null vector of the covariance.
* Material: a thin scatterer of x/X0 / |cos a| with cos a = n.d, d the unit
  direction of motion, added at the crossing before the update (Q of
  kf_oracle.scattering_q).
* Update: the Kalman update with the 2-D measurement, H = [u^T 0; v^T 0]
  (2x6), r = m - H(x - c), S = H C H^T + V (2x2), K = C H^T S^-1,
  symmetrised Joseph form, the charge flip and phi wrap of kf_oracle.update.
"""
from __future__ import annotations

import math

import torch

from . import kf_oracle as O

DT = torch.float64
SAFE_STEPS = 200    # bound on the steps of the crossing search (a near-tangent crossing needs ~60)
CROSS_TOL = 1e-9   # cm: |h(s)| accepted as on the plane


def _t(a):
    return O._t(a)


def frames(modules):
    """(c, n, u, v, x0) [M,3] x4 and [M] from a module table [10, M]:
    rows cx cy cz nx ny nz ux uy uz x_over_x0; v = n x u."""
    m = _t(modules)
    c, n, u = m[0:3].T, m[3:6].T, m[6:9].T
    v = torch.linalg.cross(n, u)
    return c, n, u, v, m[9]


def crossing_plane(p, q, c, n, bz, lo=-O.S_BACK):
    """Path s to the first crossing of the plane through c with normal n
    ([k,3] each): the smallest root s > lo of h(s) = n.(x(s) - c), within
    one turn of the helix (s <= lo + 2 pi / |w|).

    Along the helix h'(s) = n.d(s), d = (cos phi(s), sin phi(s), cot theta),
    and |h''(s)| <= M = |w| sqrt(n_x^2 + n_y^2).  From a point where
    sigma h > 0 (sigma = the sign of h there), every root lies at least the
    smallest positive root of sigma h + sigma h' t - M t^2 / 2 = 0 ahead, so
    stepping by that amount never passes a root; the steps start at s = lo
    and stop when they no longer move s (or when h changes sign, which in
    exact arithmetic only happens at the root).  Near a simple root they
    are Newton steps to second order.  Returns (s, ok): ok iff the last point
    is within CROSS_TOL of the plane with s > lo."""
    p, q, c, n = _t(p), _t(q), _t(c), _t(n)
    k = p.shape[0]
    w = O._safe_omega(O.omega(q, p[:, 3], bz))
    th = p[:, 5]
    cot = torch.cos(th) / torch.sin(th)
    M = w.abs() * torch.sqrt(n[:, 0] ** 2 + n[:, 1] ** 2)
    s_max = lo + 2 * math.pi / w.abs()
    s = torch.full((k,), float(lo), dtype=DT)

    def h_and_slope(s_):
        x = O.helix_at(p, q, s_, bz)
        h = ((x[:, :3] - c) * n).sum(1)
        d = torch.stack([torch.cos(x[:, 4]), torch.sin(x[:, 4]), cot], dim=1)
        return h, (d * n).sum(1)

    h, dh = h_and_slope(s)
    sig = torch.where(h < 0, -1.0, 1.0).to(DT)
    active = torch.ones(k, dtype=torch.bool)
    for _ in range(SAFE_STEPS):
        if not bool(active.any()):
            break
        hs, ds_ = sig * h, sig * dh
        den = torch.sqrt(ds_ * ds_ + 2 * M * hs.clamp(min=0.0)) - ds_
        step = torch.where(den > 0, 2 * hs.clamp(min=0.0) / torch.where(den > 0, den, torch.ones_like(den)),
                           torch.full_like(den, math.inf))
        step = torch.where(active, step, torch.zeros_like(step))
        s_new = s + step
        moved = active & (s_new != s)
        s = torch.where(active, s_new, s)
        active = moved & (s <= s_max) & torch.isfinite(s)
        h2, dh2 = h_and_slope(torch.where(torch.isfinite(s), s, torch.zeros_like(s)))
        h, dh = torch.where(torch.isfinite(s), h2, h), torch.where(torch.isfinite(s), dh2, dh)
        active = active & (sig * h > 0)
    h, _ = h_and_slope(torch.where(torch.isfinite(s), s, torch.zeros_like(s)))
    ok = torch.isfinite(s) & (h.abs() < CROSS_TOL) & (s > lo) & (s <= s_max)
    return s, ok


def jacobian_plane(p, q, s, n, bz):
    """F = G + g_s (ds/dp) with ds/dp = -(n.G_pos)/(n.g_pos)."""
    G, g = O.helix_partials(p, q, s, bz)
    n = _t(n)
    dh_dp = (n[:, :, None] * G[:, :3, :]).sum(1)
    dh_ds = (n * g[:, :3]).sum(1)
    dh_ds = torch.where(dh_ds.abs() < 1e-30, torch.full_like(dh_ds, 1e-30), dh_ds)
    return G + g[:, :, None] * (-dh_dp / dh_ds[:, None])[:, None, :]


def cos_incidence_plane(p, n):
    """n.d with d the unit direction of motion (sin th cos ph, sin th sin ph, cos th)."""
    p, n = _t(p), _t(n)
    ph, th = p[:, 4], p[:, 5]
    d = torch.stack([torch.sin(th) * torch.cos(ph), torch.sin(th) * torch.sin(ph), torch.cos(th)], dim=1)
    return (d * n).sum(1)


def propagate_plane(p, C, q, c, n, x_over_x0, geom, apply_material=True):
    """The state and covariance carried to the plane (c, n), with the
    module's material.  Returns (p', C', s, status)."""
    p, C, q = _t(p), _t(C), _t(q)
    s, ok = crossing_plane(p, q, c, n, geom.bz)
    s0 = torch.where(ok, s, torch.zeros_like(s))
    p2 = O.helix_at(p, q, s0, geom.bz)
    p2 = torch.cat([p2[:, :4], O.wrap_phi(p2[:, 4:5]), p2[:, 5:]], dim=1)
    F = jacobian_plane(p, q, s0, n, geom.bz)
    C2 = F @ C @ F.transpose(1, 2)
    status = torch.where(ok, 0, O.NO_CROSSING).to(torch.int64)
    if apply_material:
        th0, grazing = O.highland_theta0_at(p2, cos_incidence_plane(p2, n), _t(x_over_x0), geom.mass)
        C2 = C2 + O.scattering_q(p2, th0)
        status = status | torch.where(grazing & ok, O.GRAZING, 0)
    p2 = torch.where(ok[:, None], p2, p)
    C2 = torch.where(ok[:, None, None], C2, C)
    return p2, C2, s, status


def local_to_global(m_uv, c, u, v):
    """Global position of local coordinates (m_u, m_v) [k,2] on the planes."""
    m_uv = _t(m_uv)
    return _t(c) + m_uv[:, 0:1] * _t(u) + m_uv[:, 1:2] * _t(v)


def update_local(p, C, q, m_uv, V_uv, c, u, v):
    """Kalman update with the 2-D local measurement m_uv [k,2], covariance
    V_uv [k,2,2] on the plane (c, u, v): H = [u^T 0; v^T 0],
    r = m - H (x - c), S = H C H^T + V, chi2 = r^T S^-1 r, K = C H^T S^-1,
    p += K r, C = (I - KH) C (I - KH)^T + K V K^T symmetrised, then the
    charge flip and phi wrap of kf_oracle.update.  Returns (p', C', q',
    chi2, status)."""
    p, C, q, m_uv, V_uv = _t(p), _t(C), _t(q), _t(m_uv), _t(V_uv)
    k = p.shape[0]
    H = torch.zeros(k, 2, 6, dtype=DT)
    H[:, 0, :3] = _t(u)
    H[:, 1, :3] = _t(v)
    r = m_uv - (H[:, :, :3] @ (p[:, :3] - _t(c))[:, :, None])[:, :, 0]
    S = H @ C @ H.transpose(1, 2) + V_uv
    Si = torch.linalg.inv(S)
    chi2 = torch.einsum("ni,nij,nj->n", r, Si, r)
    K = C @ H.transpose(1, 2) @ Si
    p2 = p + (K @ r[:, :, None])[:, :, 0]
    IKH = torch.eye(6, dtype=DT) - K @ H
    C2 = IKH @ C @ IKH.transpose(1, 2) + K @ V_uv @ K.transpose(1, 2)
    C2 = 0.5 * (C2 + C2.transpose(1, 2))
    flip = p2[:, 3] < 0
    sgn = torch.where(flip, -1.0, 1.0).to(DT)
    D = torch.ones(k, 6, dtype=DT)
    D[:, 3] = sgn
    p2 = p2 * D
    C2 = C2 * D[:, :, None] * D[:, None, :]
    p2 = torch.cat([p2[:, :4], O.wrap_phi(p2[:, 4:5]), p2[:, 5:]], dim=1)
    d = torch.diagonal(C2, dim1=1, dim2=2)
    tr = d[:, 0] + d[:, 1] + d[:, 2]
    bad = (d[:, 3:] <= 0).any(dim=1) | (d[:, :3] < -1e-3 * tr[:, None]).any(dim=1)
    status = torch.where(flip, O.CHARGE_FLIP, 0) | torch.where(bad, O.COV_NOT_PSD, 0)
    return p2, C2, q * sgn, chi2, status.to(torch.int64)


def unpack2(cov3):
    """[3, k] packed (uu, vu, vv) -> [k, 2, 2]."""
    c = _t(cov3)
    V = torch.zeros(c.shape[1], 2, 2, dtype=DT)
    V[:, 0, 0] = c[0]
    V[:, 1, 0] = V[:, 0, 1] = c[1]
    V[:, 1, 1] = c[2]
    return V


def make_seeds_planes(hit_offsets, hit_module, hit_valid, hit_uv, modules, bz):
    """Three-hit seeds (kf_oracle.make_seeds, first three valid hits) from
    the hits' global positions on their modules."""
    c, n, u, v, _ = frames(modules)
    mod = torch.as_tensor(hit_module, dtype=torch.int64)
    g = local_to_global(_t(hit_uv).T, c[mod], u[mod], v[mod])
    return O.make_seeds(hit_offsets, hit_valid, g.T, bz)


def fit_plane_tracks(seed_p, seed_C, seed_q, hit_offsets, hit_module, hit_valid, hit_uv, hit_cov_uv, modules, geom,
                     state_round=None, state_jitter=None):
    """Forward fit over tilted modules, the rules of kf_oracle.fit_tracks
    with a module per entry: the seed sits on the first valid entry's hit
    and, like every later entry, is propagated to its module's plane
    (propagate_plane, here a step of length ~0 whose Jacobian removes the
    seed covariance's component along the normal), gets the module's
    material and, if valid, the 2-D update; a failed crossing or a non-finite step freezes the track.
    hit_uv [2, nh], hit_cov_uv [3, nh] packed (uu, vu, vv), modules [10, M].
    state_round / state_jitter: the conditioning probes of
    kf_oracle.fit_tracks (the state rounded to a precision, or scaled by
    1 +- state_jitter element by element, after every propagation and
    update).  Returns dict(p, C, q, chi2, ndf, status)."""
    off = torch.as_tensor(hit_offsets, dtype=torch.int64)
    mod_all = torch.as_tensor(hit_module, dtype=torch.int64)
    val_all = torch.as_tensor(hit_valid, dtype=torch.int64)
    m_all = _t(hit_uv).T
    V_all = unpack2(hit_cov_uv)
    c_m, n_m, u_m, v_m, x0_m = frames(modules)
    n = off.shape[0] - 1
    lens = off[1:] - off[:-1]
    k0 = torch.full((n,), -1, dtype=torch.int64)
    maxlen = int(lens.max()) if n > 0 else 0
    for j in range(maxlen - 1, -1, -1):
        e = off[:-1] + j
        has = j < lens
        ev = torch.where(has, e, torch.zeros_like(e))
        k0 = torch.where(has & (val_all[ev] == 1), e, k0)
    p, C, q = _t(seed_p), _t(seed_C), _t(seed_q)
    chi2 = torch.zeros(n, dtype=DT)
    nval = torch.zeros(n, dtype=torch.int64)
    status = torch.zeros(n, dtype=torch.int64)
    alive = k0 >= 0
    end = off[1:]
    for j in range(maxlen):
        e = k0 + j
        act = alive & (e < end)
        idx = torch.nonzero(act)[:, 0]
        if idx.numel() == 0:
            break
        ei = e[idx]
        md = mod_all[ei]
        pp, CC, qq = p[idx], C[idx], q[idx]
        # the seed is carried onto its first module too (a step of length
        # ~0): that projects its covariance onto the plane, so that the
        # normal is a null vector there as after every other step
        pp2, CC2, _, st_p = propagate_plane(pp, CC, qq, c_m[md], n_m[md], x0_m[md], geom)
        if state_round is not None:
            pp2, CC2 = pp2.to(state_round).to(DT), CC2.to(state_round).to(DT)
        if state_jitter is not None:
            pp2, CC2 = O._jitter(pp2, CC2, idx + j, state_jitter)
        good = (st_p & O.NO_CROSSING) == 0
        valid = (val_all[ei] == 1) & good
        pu, Cu, qu, c2, st_u = update_local(pp2, CC2, qq, m_all[ei], V_all[ei], c_m[md], u_m[md], v_m[md])
        pn = torch.where(valid[:, None], pu, pp2)
        Cn = torch.where(valid[:, None, None], Cu, CC2)
        qn = torch.where(valid, qu, qq)
        c2n = torch.where(valid, c2, torch.zeros_like(c2))
        st = st_p | torch.where(valid, st_u, 0)
        finite = torch.isfinite(pn).all(dim=1) & torch.isfinite(Cn).flatten(1).all(dim=1) & torch.isfinite(c2n)
        st = st | torch.where(finite, 0, O.NONFINITE)
        keep = good & finite
        pn = torch.where(keep[:, None], pn, pp)
        Cn = torch.where(keep[:, None, None], Cn, CC)
        qn = torch.where(keep, qn, qq)
        c2n = torch.where(keep, c2n, torch.zeros_like(c2n))
        if state_round is not None:
            pn, Cn = pn.to(state_round).to(DT), Cn.to(state_round).to(DT)
        if state_jitter is not None:
            pn, Cn = O._jitter(pn, Cn, idx + j + 1, state_jitter)
        p = p.index_put((idx,), pn)
        C = C.index_put((idx,), Cn)
        q = q.index_put((idx,), qn)
        chi2 = chi2.index_put((idx,), chi2[idx] + c2n)
        nval = nval.index_put((idx,), nval[idx] + (valid & keep).to(torch.int64))
        status = status.index_put((idx,), status[idx] | st)
        alive = alive.index_put((idx,), keep)
    return dict(p=p, C=C, q=q, chi2=chi2, ndf=2 * nval - 5, status=status)
