"""FP64 CPU oracle for the per-layer Kalman-filter step.  TEST INFRASTRUCTURE.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It is a plain, slow, step-by-step statement of what the GPU path
computes, in float64 PyTorch CPU ops, batched over tracks only (every per-track
formula is written exactly as stated below; nothing is fused or reordered).
It shares no code with the HIP kernels.

The paper (Sec. 2.2 "Track finding algorithm" and Sec. 3.1 "Geometry &
detector description") names the computations -- propagation of a track
candidate to the next layer, hit selection, Kalman-filter calculations -- but
gives no formulas.  The formulas are the textbook ones for a helix in a uniform
solenoidal field, the Highland multiple-scattering angle and the linear Kalman
filter; each function states the reading it takes.

Units: cm, GeV/c, tesla, radians.  State p = (x, y, z, ipt, phi, theta) with
ipt = 1/pT >= 0 and a separate charge q = +-1.  Covariances are full 6x6 / 3x3
tensors here; packing is done only at the interface.
"""
from __future__ import annotations

import math

import torch

DT = torch.float64
C_LIGHT = 0.00299792458   # GeV/c per (T cm)
GRAZING_COS = 0.05        # |cos(incidence)| below this is flagged and clamped
SEED_COV_DIAG = (1.0, 1.0, 1.0, 1.0, 0.01, 0.01)

# per-track status bits (shared meaning with the C interface)
NO_CROSSING = 1
GRAZING = 2
NONFINITE = 4
FP64_FALLBACK = 8
CHARGE_FLIP = 16
COV_NOT_PSD = 32

BARREL = 0
DISK = 1


def _t(a):
    """Any input as a float64 tensor (differentiable when it already is one)."""
    return a.to(DT) if torch.is_tensor(a) else torch.as_tensor(a, dtype=DT)


def wrap_phi(phi):
    """Wrap to (-pi, pi]."""
    return phi - 2.0 * math.pi * torch.ceil((phi - math.pi) / (2.0 * math.pi))


def omega(q, ipt, bz):
    """Signed curvature (rad per cm of transverse path): omega = -q c_B B_z / pT.
    Positive charge in a positive field turns clockwise."""
    return -q * C_LIGHT * bz * ipt


def _safe_omega(w):
    tiny = 1e-12
    return torch.where(w.abs() < tiny, torch.where(w < 0, -tiny, tiny) + 0.0 * w, w)


# --------------------------------------------------------------------------
# a1: helix propagation
# --------------------------------------------------------------------------

def helix_at(p, q, s, bz):
    """State after transverse path s along the helix (plain closed form):
    phi(s) = phi0 + w s,  x(s) = x0 + [sin(phi0 + w s) - sin phi0]/w,
    y(s) = y0 - [cos(phi0 + w s) - cos phi0]/w,  z(s) = z0 + s cot(theta).
    ipt and theta are unchanged."""
    p, q, s = _t(p), _t(q), _t(s)
    x0, y0, z0, ipt, phi0, th = p.unbind(-1)
    w = _safe_omega(omega(q, ipt, bz))
    ph = phi0 + w * s
    x = x0 + (torch.sin(ph) - torch.sin(phi0)) / w
    y = y0 - (torch.cos(ph) - torch.cos(phi0)) / w
    # for |u| = |w s| < 1e-2 the differences above lose digits; expand
    # sin(phi0+u) = s0 cos u + c0 sin u, cos(phi0+u) = c0 cos u - s0 sin u:
    # x = x0 + s [s0 (cos u - 1)/u + c0 sin(u)/u], y = y0 + s [-c0 (cos u - 1)/u + s0 sin(u)/u]
    u = w * s
    small = u.abs() < 1e-2
    us = torch.where(small, u, torch.zeros_like(u))
    cm1_u = -us / 2.0 + us ** 3 / 24.0 - us ** 5 / 720.0
    sin_u = 1.0 - us ** 2 / 6.0 + us ** 4 / 120.0 - us ** 6 / 5040.0
    s0, c0 = torch.sin(phi0), torch.cos(phi0)
    x = torch.where(small, x0 + s * (s0 * cm1_u + c0 * sin_u), x)
    y = torch.where(small, y0 + s * (-c0 * cm1_u + s0 * sin_u), y)
    z = z0 + s * torch.cos(th) / torch.sin(th)
    return torch.stack([x, y, z, ipt, ph, th], dim=-1)


S_BACK = 1.0     # cm: a different layer may lie at most this far behind the state
S_SAME = 0.01    # cm: re-crossing the layer the state sits on must go at least this far


def _path_window(same):
    """Lower end of the admissible path window: the crossing is the first root
    of the surface equation with s > lo.  For a different layer lo = -S_BACK
    (a surface just behind an estimate that overshot it is reached by a short
    backward step); for the layer the state already sits on (a looper turning
    round) lo = +S_SAME, so the current point itself is skipped."""
    return torch.where(same, torch.full_like(same, S_SAME, dtype=DT), torch.full_like(same, -S_BACK, dtype=DT))


def crossing_barrel(p, q, R, bz, same=None, newton_steps=3):
    """First root s > lo (see _path_window) of x(s)^2 + y(s)^2 = R^2.

    With A = x0 cos phi0 + y0 sin phi0, B = x0 sin phi0 - y0 cos phi0 and the
    turning angle u = w s, the squared radius along the helix is
        r^2(u) = r0^2 + (2A/w) sin u + 2(1 - wB)(1 - cos u)/w^2,
    so the crossing solves (Aw) sin u - (1 - wB) cos u = w^2 (R^2 - r0^2)/2 - (1 - wB),
    i.e. rho sin(u - delta) = rhs.  Both solutions are mapped onto the turn
    (lo, lo + 2 pi/|w|], the smaller is taken and polished by Newton steps on
    h(s) = r^2(s) - R^2.  Returns (s, ok)."""
    p, q = _t(p), _t(q)
    x0, y0, _, ipt, phi0, _ = p.unbind(-1)
    if same is None:
        same = torch.zeros_like(x0, dtype=torch.bool)
    lo = _path_window(same)
    w = omega(q, ipt, bz)
    ws = _safe_omega(w)
    R = _t(R) * torch.ones_like(x0)
    A = x0 * torch.cos(phi0) + y0 * torch.sin(phi0)
    B = x0 * torch.sin(phi0) - y0 * torch.cos(phi0)
    d2 = R * R - (x0 * x0 + y0 * y0)
    a = A * ws
    b = 1.0 - ws * B
    c = 0.5 * ws * ws * d2
    rho = torch.sqrt(a * a + b * b)
    t = (c - b) / rho
    ok = t.abs() <= 1.0
    tc = torch.clamp(t, -1.0, 1.0)
    delta = torch.atan2(b, a)
    u1 = delta + torch.asin(tc)
    u2 = delta + math.pi - torch.asin(tc)
    period = 2.0 * math.pi / ws.abs()
    s1 = lo + torch.remainder(u1 / ws - lo, period)
    s2 = lo + torch.remainder(u2 / ws - lo, period)
    s = torch.minimum(s1, s2)
    # straight-line limit (|w| tiny): s^2 + 2As - (R^2 - r0^2) = 0
    disc = A * A + d2
    sq = torch.sqrt(torch.clamp(disc, min=0.0))
    r1, r2 = -A - sq, -A + sq
    s_line = torch.where(r1 > lo, r1, r2)
    line = w.abs() < 1e-9
    s = torch.where(line, s_line, s)
    ok = torch.where(line, (disc >= 0) & (s_line > lo), ok)
    s = torch.where(ok, s, torch.zeros_like(s))
    for _ in range(newton_steps):
        h = helix_at(p, q, s, bz)
        hx, hy, hph = h[..., 0], h[..., 1], h[..., 4]
        f = hx * hx + hy * hy - R * R
        df = 2.0 * (hx * torch.cos(hph) + hy * torch.sin(hph))
        df = torch.where(df.abs() < 1e-30, torch.ones_like(df), df)
        s = s - torch.where(ok, f / df, torch.zeros_like(f))
    return s, ok


def crossing_disk(p, Z, same=None):
    """z(s) = Z:  s = (Z - z0) / cot(theta); must be > lo (see _path_window).
    Returns (s, ok)."""
    p = _t(p)
    _, _, z0, _, _, th = p.unbind(-1)
    if same is None:
        same = torch.zeros_like(z0, dtype=torch.bool)
    lo = _path_window(same)
    cot = torch.cos(th) / torch.sin(th)
    ok_c = cot.abs() > 1e-15
    cot_s = torch.where(ok_c, cot, torch.ones_like(cot))
    s = (_t(Z) - z0) / cot_s
    ok = ok_c & (s > lo)
    return torch.where(ok, s, torch.zeros_like(s)), ok


def crossing(p, q, kind, pos, bz, same=None):
    """Path to the layer surface (kind/pos per track); ``same`` marks tracks
    whose state already sits on that layer."""
    sb, okb = crossing_barrel(p, q, pos, bz, same)
    sd, okd = crossing_disk(p, pos, same)
    isb = kind == BARREL
    return torch.where(isb, sb, sd), torch.where(isb, okb, okd)


# --------------------------------------------------------------------------
# a2: transport Jacobian (surface to surface)
# --------------------------------------------------------------------------

def helix_partials(p, q, s, bz):
    """The helix map at fixed transverse path s, differentiated: G = dp'/dp
    with s held fixed, and g_s = dp'/ds = (cos phi(s), sin phi(s), cot theta,
    0, w, 0)."""
    p, q, s = _t(p), _t(q), _t(s)
    x0, y0, z0, ipt, phi0, th = p.unbind(-1)
    w = _safe_omega(omega(q, ipt, bz))
    dw_dipt = -q * C_LIGHT * bz
    ph = phi0 + w * s
    sp, cp = torch.sin(ph), torch.cos(ph)
    s0, c0 = torch.sin(phi0), torch.cos(phi0)
    cot = torch.cos(th) / torch.sin(th)
    one = torch.ones_like(x0)
    dx_dphi = (cp - c0) / w
    dy_dphi = (sp - s0) / w
    # dx/dw = [u cos(phi0+u) - sin(phi0+u) + sin phi0]/w^2 with u = w s; the
    # bracket is O(u^2), so for |u| < 1e-2 it is expanded about phi0:
    # dx/dw = s^2 [c0 (-u/3 + u^3/30 - u^5/840) - s0 (1/2 - u^2/8 + u^4/144)]
    # dy/dw = s^2 [s0 (-u/3 + u^3/30 - u^5/840) + c0 (1/2 - u^2/8 + u^4/144)]
    u = w * s
    small = u.abs() < 1e-2
    us = torch.where(small, u, torch.zeros_like(u))
    odd = -us / 3.0 + us ** 3 / 30.0 - us ** 5 / 840.0
    even = 0.5 - us ** 2 / 8.0 + us ** 4 / 144.0
    ser_x = s * s * (c0 * odd - s0 * even)
    ser_y = s * s * (s0 * odd + c0 * even)
    dx_dw = torch.where(small, ser_x, s * cp / w - (sp - s0) / (w * w))
    dy_dw = torch.where(small, ser_y, s * sp / w + (cp - c0) / (w * w))
    rows = [
        [one, 0 * one, 0 * one, dx_dw * dw_dipt, dx_dphi, 0 * one],
        [0 * one, one, 0 * one, dy_dw * dw_dipt, dy_dphi, 0 * one],
        [0 * one, 0 * one, one, 0 * one, 0 * one, -s / torch.sin(th) ** 2],
        [0 * one, 0 * one, 0 * one, one, 0 * one, 0 * one],
        [0 * one, 0 * one, 0 * one, s * dw_dipt, one, 0 * one],
        [0 * one, 0 * one, 0 * one, 0 * one, 0 * one, one],
    ]
    G = torch.stack([torch.stack(r, dim=-1) for r in rows], dim=-2)
    g_s = torch.stack([cp, sp, cot, 0 * one, w, 0 * one], dim=-1)
    return G, g_s


def jacobian(p, q, s, kind, bz):
    """F = dp'/dp of the map 'propagate p to the surface', including the
    dependence of the path length on p:
        F = G + g_s (ds/dp),  ds/dp = -(dh/dp)/(dh/ds),
    G = partials of the helix at fixed s, g_s = d(state)/ds, and h the surface
    equation (barrel: x^2 + y^2 - R^2, disk: z - Z)."""
    p, q, s = _t(p), _t(q), _t(s)
    G, g_s = helix_partials(p, q, s, bz)
    cp, sp = g_s[..., 0], g_s[..., 1]
    cot = g_s[..., 2]
    h = helix_at(p, q, s, bz)
    xs, ys = h[..., 0], h[..., 1]
    dh_dp_b = 2.0 * xs[:, None] * G[:, 0, :] + 2.0 * ys[:, None] * G[:, 1, :]
    dh_ds_b = 2.0 * (xs * cp + ys * sp)
    dh_dp_d = G[:, 2, :]
    dh_ds_d = cot
    isb = (kind == BARREL)
    dh_dp = torch.where(isb[:, None], dh_dp_b, dh_dp_d)
    dh_ds = torch.where(isb, dh_ds_b, dh_ds_d)
    dh_ds = torch.where(dh_ds.abs() < 1e-30, torch.full_like(dh_ds, 1e-30), dh_ds)
    ds_dp = -dh_dp / dh_ds[:, None]
    return G + g_s[:, :, None] * ds_dp[:, None, :]


# --------------------------------------------------------------------------
# a3: material (multiple scattering) and covariance propagation
# --------------------------------------------------------------------------

def cos_incidence(p, kind):
    """Cosine of the angle between the momentum and the surface normal:
    barrel sin(theta) cos(phi - phi_pos), disk |cos(theta)|."""
    x, y, _, _, ph, th = p.unbind(-1)
    cb = torch.sin(th) * torch.cos(ph - torch.atan2(y, x))
    cd = torch.cos(th).abs()
    return torch.where(kind == BARREL, cb, cd)


def highland_theta0(p, kind, x_over_x0, mass):
    """Highland / PDG plane angle for unit charge:
    theta0 = 0.0136/(beta p) sqrt(x) (1 + 0.038 ln(x / beta^2)),
    x = t / |cos(incidence)|.  Returns (theta0, grazing)."""
    return highland_theta0_at(p, cos_incidence(p, kind), x_over_x0, mass)


def highland_theta0_at(p, cos_a, x_over_x0, mass):
    """highland_theta0 for a given cosine of the incidence angle (any
    surface): |cos_a| clamped at GRAZING_COS and flagged."""
    ipt, th = p[..., 3], p[..., 5]
    ca = _t(cos_a).abs()
    grazing = ca < GRAZING_COS
    ca = torch.clamp(ca, min=GRAZING_COS)
    pmag = 1.0 / (ipt * torch.sin(th))
    beta = pmag / torch.sqrt(pmag * pmag + mass * mass)
    x = x_over_x0 / ca
    th0 = 0.0136 / (beta * pmag) * torch.sqrt(x) * (1.0 + 0.038 * torch.log(x / (beta * beta)))
    return th0, grazing


def process_noise(p, kind, x_over_x0, mass):
    """Q in (ipt, phi, theta) for two independent deflections of rms theta0
    that keep |p|: Q_thth = th0^2, Q_phph = th0^2/sin^2(theta),
    Q_ipt,ipt = (ipt cot)^2 th0^2, Q_ipt,th = -ipt cot th0^2 (rank 2)."""
    p = _t(p)
    th0, grazing = highland_theta0(p, kind, x_over_x0, mass)
    return scattering_q(p, th0), grazing


def scattering_q(p, th0):
    """Q of process_noise for a given plane angle theta0 [n]."""
    ipt, th = p[..., 3], p[..., 5]
    v = th0 * th0
    cot = torch.cos(th) / torch.sin(th)
    n = p.shape[0]
    zero = torch.zeros_like(v)
    q33 = (ipt * cot) ** 2 * v
    q35 = -ipt * cot * v
    q44 = v / torch.sin(th) ** 2
    q55 = v
    rows = [[zero] * 6 for _ in range(6)]
    rows[3][3] = q33
    rows[3][5] = q35
    rows[5][3] = q35
    rows[4][4] = q44
    rows[5][5] = q55
    return torch.stack([torch.stack(r, dim=-1) for r in rows], dim=-2)


def propagate(p, C, q, kind, pos, x_over_x0, geom, apply_material=True, same=None):
    """kf_propagate: move (p, C) to the layer surface.  ``same`` (bool per
    track, default False) marks a re-crossing of the layer the state is on.
    Returns (p', C', s, status)."""
    p, C, q = _t(p), _t(C), _t(q)
    s, ok = crossing(p, q, kind, pos, geom.bz, same)
    p2 = helix_at(p, q, s, geom.bz)
    p2 = torch.cat([p2[..., :4], wrap_phi(p2[..., 4:5]), p2[..., 5:]], dim=-1)
    F = jacobian(p, q, s, kind, geom.bz)
    C2 = F @ C @ F.transpose(-1, -2)
    status = torch.where(ok, 0, NO_CROSSING).to(torch.int64)
    if apply_material:
        Q, grazing = process_noise(p2, kind, x_over_x0, geom.mass)
        C2 = C2 + Q
        status = status | torch.where(grazing & ok, GRAZING, 0)
    return p2, C2, s, status


# --------------------------------------------------------------------------
# a4/a5: residual, S, chi2, gain, Joseph update
# --------------------------------------------------------------------------

def update(p, C, q, m, V):
    """kf_update: Kalman update with a 3-D hit m and its 3x3 covariance V.
    r = m - Hp, S = H C H^T + V, chi2 = r^T S^-1 r, K = C H^T S^-1,
    p <- p + K r, C <- (I - KH) C (I - KH)^T + K V K^T, then symmetrized.
    If ipt turns negative the charge is flipped (ipt, q and row/column 3 of C
    change sign) so that the curvature is unchanged; phi is wrapped.
    Returns (p', C', q', chi2, status)."""
    p, C, q, m, V = _t(p), _t(C), _t(q), _t(m), _t(V)
    n = p.shape[0]
    r = m - p[..., :3]
    S = C[..., :3, :3] + V
    Sinv = torch.linalg.inv(S)
    chi2 = torch.einsum("ni,nij,nj->n", r, Sinv, r)
    K = C[..., :, :3] @ Sinv
    p2 = p + (K @ r[..., None])[..., 0]
    H = torch.zeros(3, 6, dtype=DT)
    H[0, 0] = H[1, 1] = H[2, 2] = 1.0
    I = torch.eye(6, dtype=DT)
    IKH = I - K @ H
    C2 = IKH @ C @ IKH.transpose(-1, -2) + K @ V @ K.transpose(-1, -2)
    C2 = 0.5 * (C2 + C2.transpose(-1, -2))
    flip = p2[..., 3] < 0
    sgn = torch.where(flip, -1.0, 1.0).to(DT)
    D = torch.ones(n, 6, dtype=DT)
    D = torch.cat([D[:, :3], sgn[:, None], D[:, 4:]], dim=1)
    p2 = p2 * D
    C2 = C2 * D[:, :, None] * D[:, None, :]
    q2 = q * sgn
    p2 = torch.cat([p2[..., :4], wrap_phi(p2[..., 4:5]), p2[..., 5:]], dim=-1)
    # the 6x6 covariance of a state on a surface has the surface normal as a
    # null vector (rank 5), so a zero position variance is legitimate: flag
    # only non-positive angle/curvature variances or clearly negative position
    # ones (below -1e-3 of the position trace)
    d = torch.diagonal(C2, dim1=-2, dim2=-1)
    tr_pos = d[..., 0] + d[..., 1] + d[..., 2]
    diag_bad = (d[..., 3:] <= 0).any(dim=-1) | (d[..., :3] < -1e-3 * tr_pos[..., None]).any(dim=-1)
    status = torch.where(flip, CHARGE_FLIP, 0) | torch.where(diag_bad, COV_NOT_PSD, 0)
    return p2, C2, q2, chi2, status.to(torch.int64)


# --------------------------------------------------------------------------
# seeding from three hits
# --------------------------------------------------------------------------

def seed_from_hits(h1, h2, h3, bz):
    """Helix through three hits (transverse Menger curvature, then the polar
    angle from the arc length between hits 1 and 3); position = hit 1.
    kappa = 2 ((h2-h1) x (h3-h1))_z / (d12 d13 d23), q = -sign(kappa) (+1 at 0),
    ipt = |kappa|/(c_B B_z), phi1 = atan2(h2-h1) - asin(kappa d12 / 2),
    s13 = 2 asin(|kappa| d13/2)/|kappa|, cot(theta) = (z3 - z1)/s13.
    Returns (p, C0, q)."""
    h1, h2, h3 = _t(h1), _t(h2), _t(h3)
    dx12, dy12 = h2[..., 0] - h1[..., 0], h2[..., 1] - h1[..., 1]
    dx13, dy13 = h3[..., 0] - h1[..., 0], h3[..., 1] - h1[..., 1]
    dx23, dy23 = h3[..., 0] - h2[..., 0], h3[..., 1] - h2[..., 1]
    d12 = torch.sqrt(dx12 ** 2 + dy12 ** 2)
    d13 = torch.sqrt(dx13 ** 2 + dy13 ** 2)
    d23 = torch.sqrt(dx23 ** 2 + dy23 ** 2)
    cross = dx12 * dy13 - dy12 * dx13
    kappa = 2.0 * cross / (d12 * d13 * d23)
    q = torch.where(kappa > 0, -1.0, 1.0).to(DT)
    ipt = kappa.abs() / (C_LIGHT * bz)
    phi1 = torch.atan2(dy12, dx12) - torch.asin(torch.clamp(kappa * d12 / 2.0, -1.0, 1.0))
    ak = kappa.abs()
    ak_s = torch.where(ak > 0, ak, torch.ones_like(ak))
    s13 = torch.where(ak > 0, 2.0 * torch.asin(torch.clamp(ak_s * d13 / 2.0, -1.0, 1.0)) / ak_s, d13)
    cot = (h3[..., 2] - h1[..., 2]) / s13
    theta = 0.5 * math.pi - torch.atan(cot)
    p = torch.stack([h1[..., 0], h1[..., 1], h1[..., 2], ipt, wrap_phi(phi1), theta], dim=-1)
    C0 = torch.diag(_t(SEED_COV_DIAG)).expand(p.shape[0], 6, 6).clone()
    return p, C0, q


def first_three_valid(hit_offsets, hit_valid):
    """Indices of the first three valid entries of every track (-1 if absent)."""
    off = torch.as_tensor(hit_offsets, dtype=torch.int64)
    valid = torch.as_tensor(hit_valid, dtype=torch.int64)
    n = off.shape[0] - 1
    lens = off[1:] - off[:-1]
    track = torch.repeat_interleave(torch.arange(n), lens)
    csum = torch.cumsum(valid, 0) - valid            # valid entries before e (global)
    rank = csum - torch.cat([torch.zeros(1, dtype=torch.int64), torch.cumsum(valid, 0)])[off[:-1]][track]
    out = torch.full((n, 3), -1, dtype=torch.int64)
    sel = (valid == 1) & (rank < 3)
    e = torch.nonzero(sel)[:, 0]
    out[track[e], rank[e]] = e
    return out


# cm, transverse distance between chosen seed hits (mode 1): below the 3 cm
# between the two innermost barrel layers, so that no barrel hit pair sits at
# the threshold, where rounding would decide the choice
SEED_MIN_SPACING = 2.5


def spaced_three_valid(hit_offsets, hit_valid, hit_pos, spacing=SEED_MIN_SPACING, return_margin=False):
    """Greedy choice along each track: the first valid entry, then each next
    valid entry whose transverse distance from the previously chosen hit is at
    least ``spacing``; three entries, or -1 everywhere if fewer qualify.
    return_margin: also return, per track, the smallest |d - spacing| /
    spacing over the distances the choice compared (inf if none): a track
    whose margin is at the rounding level of a precision can be seeded
    either way in that precision."""
    off = torch.as_tensor(hit_offsets, dtype=torch.int64)
    valid = torch.as_tensor(hit_valid, dtype=torch.int64)
    hp = _t(hit_pos)
    n = off.shape[0] - 1
    lens = off[1:] - off[:-1]
    out = torch.full((n, 3), -1, dtype=torch.int64)
    cnt = torch.zeros(n, dtype=torch.int64)
    lastx = torch.zeros(n, dtype=DT)
    lasty = torch.zeros(n, dtype=DT)
    maxlen = int(lens.max()) if n else 0
    ar = torch.arange(n)
    margin = torch.full((n,), math.inf, dtype=DT)
    for j in range(maxlen):
        has = j < lens
        e = torch.where(has, off[:-1] + j, torch.zeros_like(lens))
        hx, hy = hp[0, e], hp[1, e]
        d = torch.sqrt((hx - lastx) ** 2 + (hy - lasty) ** 2)
        far = d >= spacing
        compared = has & (valid[e] == 1) & (cnt > 0) & (cnt < 3)
        margin = torch.where(compared, torch.minimum(margin, (d - spacing).abs() / spacing), margin)
        take = has & (valid[e] == 1) & (cnt < 3) & ((cnt == 0) | far)
        t = ar[take]
        out[t, cnt[t]] = e[t]
        lastx = torch.where(take, hx, lastx)
        lasty = torch.where(take, hy, lasty)
        cnt = cnt + take.to(torch.int64)
    out[cnt < 3] = -1
    return (out, margin) if return_margin else out


SEED_FIRST_THREE = 0
SEED_SPACED = 1


def make_seeds(hit_offsets, hit_valid, hit_pos, bz, mode=SEED_FIRST_THREE):
    """Seed every track from three of its valid hits: the first three
    (mode 0) or three hits at least SEED_MIN_SPACING apart in the transverse
    plane (mode 1, a longer lever arm for tracks whose first hits are close
    together there, such as forward tracks crossing barrel and disk layers).
    The seed sits on the first valid hit.  Returns (p, C0, q, ok)."""
    if mode == SEED_FIRST_THREE:
        idx = first_three_valid(hit_offsets, hit_valid)
    else:
        idx = spaced_three_valid(hit_offsets, hit_valid, hit_pos)
    ok = (idx >= 0).all(dim=1)
    hp = _t(hit_pos)
    safe = torch.where(idx >= 0, idx, torch.zeros_like(idx))
    h = [hp[:, safe[:, i]].T for i in range(3)]
    p, C0, q = seed_from_hits(h[0], h[1], h[2], bz)
    return p, C0, q, ok


# --------------------------------------------------------------------------
# alignment of barrel hits
# --------------------------------------------------------------------------

def aligned_hits(hit_pos, hit_layer, geom, align):
    """Apply per-layer corrections to barrel hits: rotate about z by a_rphi/R
    (R = the layer radius) and shift z by a_z.  Disk hits are unchanged.
    hit_pos: [3, nh] tensor; align: [2, L] tensor or None.  Returns [nh, 3]."""
    h = hit_pos.T
    if align is None:
        return h
    lay = torch.as_tensor(hit_layer, dtype=torch.int64)
    kind = torch.as_tensor(geom.kind, dtype=torch.int64)[lay]
    R = _t(geom.pos)[lay]
    isb = kind == BARREL
    ang = torch.where(isb, align[0][lay] / R, torch.zeros_like(R))
    dz = torch.where(isb, align[1][lay], torch.zeros_like(R))
    c, s = torch.cos(ang), torch.sin(ang)
    x = c * h[:, 0] - s * h[:, 1]
    y = s * h[:, 0] + c * h[:, 1]
    z = h[:, 2] + dz
    return torch.stack([x, y, z], dim=-1)


# --------------------------------------------------------------------------
# a6: the per-track layer loop
# --------------------------------------------------------------------------

def unpack_sym(packed, n):
    """[k, N] packed lower triangle (row-major, idx(i,j) = i(i+1)/2 + j) -> [N, n, n]."""
    P = torch.as_tensor(packed, dtype=DT)
    N = P.shape[1]
    M = torch.zeros(N, n, n, dtype=DT)
    k = 0
    for i in range(n):
        for j in range(i + 1):
            M[:, i, j] = P[k]
            M[:, j, i] = P[k]
            k += 1
    return M


def pack_sym(M):
    n = M.shape[-1]
    out = []
    for i in range(n):
        for j in range(i + 1):
            out.append(M[..., i, j])
    return torch.stack(out, dim=0)


def _jitter(p, C, key, r):
    """Scale every element by 1 + r or 1 - r with a sign pattern that
    alternates with the element index and with ``key`` (C stays symmetric)."""
    i6 = torch.arange(6)
    sp = 1.0 - 2.0 * ((key[:, None] + i6[None, :]) % 2).to(DT)
    sc = 1.0 - 2.0 * ((key[:, None, None] + i6[None, :, None] + i6[None, None, :]) % 2).to(DT)
    return p * (1.0 + r * sp), C * (1.0 + r * sc)


def fit_tracks(seed_p, seed_C, seed_q, hit_offsets, hit_layer, hit_valid, hit_pos, hit_cov, geom,
               align=None, state_round=None, state_jitter=None, record=False):
    """kf_fit_tracks: forward Kalman fit of every track.

    Each track starts at its seed, which sits on its first valid entry k0
    (entries before k0 are skipped).  At k0 the material of that layer is added
    at the seed; at every later entry the state is propagated to the entry's
    layer and the layer's material is added; valid entries are then used in an
    update and their chi2 summed.  The crossing of entry k is searched with the
    re-crossing window when entry k-1 was on the same layer (a looper turning
    round), otherwise with the window that admits a short backward step.  A
    failed crossing or a non-finite result freezes the track at its last good
    state.

    seed_p [n,6], seed_C [n,6,6], seed_q [n] tensors (may require grad);
    hit_pos [3,nh] tensor (may require grad); hit_cov [6,nh] packed;
    align [2,L] tensor or None.
    state_round: None, or a dtype (float32) to which the state and covariance
    are rounded after every propagation and every update -- a conditioning
    probe for the tests (how far the float64 result moves under
    storage-precision perturbations).
    state_jitter: None, or a relative size r; after every propagation and
    update every element of the state and covariance is scaled by (1 + r) or
    (1 - r) (alternating by element, track and entry) -- the same probe at
    float64 rounding.
    record: also return the filtered state after every entry (pe [nh,6],
    Ce [nh,6,6], qe [nh]; NaN for entries the fit did not reach) and the
    predicted state of every entry, after its propagation and material and
    before its update (pp [nh,6], Cp [nh,6,6]).
    Returns dict(p, C, q, chi2, ndf, status[, pe, Ce, qe])."""
    off = torch.as_tensor(hit_offsets, dtype=torch.int64)
    lay_all = torch.as_tensor(hit_layer, dtype=torch.int64)
    val_all = torch.as_tensor(hit_valid, dtype=torch.int64)
    V_all = unpack_sym(hit_cov, 3)
    hp = hit_pos if torch.is_tensor(hit_pos) else _t(hit_pos)
    m_all = aligned_hits(hp, lay_all, geom, align)
    kind_l = torch.as_tensor(geom.kind, dtype=torch.int64)
    pos_l = _t(geom.pos)
    x0_l = _t(geom.x_over_x0)
    n = off.shape[0] - 1

    # first valid entry of each track
    k0 = torch.full((n,), -1, dtype=torch.int64)
    lens = off[1:] - off[:-1]
    maxlen = int(lens.max()) if n > 0 else 0
    for j in range(maxlen - 1, -1, -1):
        e = off[:-1] + j
        has = (j < lens)
        ev = torch.where(has, e, torch.zeros_like(e))
        k0 = torch.where(has & (val_all[ev] == 1), e, k0)

    p = seed_p
    C = seed_C
    q = seed_q.to(DT)
    chi2 = torch.zeros(n, dtype=DT) + 0.0 * seed_p[:, 0]
    nval = torch.zeros(n, dtype=torch.int64)
    status = torch.zeros(n, dtype=torch.int64)
    alive = k0 >= 0
    end = off[1:]

    prev_e = k0.clone()
    nh = lay_all.shape[0]
    if record:
        pe = torch.full((nh, 6), float("nan"), dtype=DT)
        Ce = torch.full((nh, 6, 6), float("nan"), dtype=DT)
        qe = torch.full((nh,), float("nan"), dtype=DT)
        ppe = torch.full((nh, 6), float("nan"), dtype=DT)
        Cpe = torch.full((nh, 6, 6), float("nan"), dtype=DT)
    for j in range(maxlen):
        e = k0 + j
        act = alive & (e < end)
        idx = torch.nonzero(act)[:, 0]
        if idx.numel() == 0:
            break
        ei = e[idx]
        lay = lay_all[ei]
        kind = kind_l[lay]
        pp, CC, qq = p[idx], C[idx], q[idx]
        st = torch.zeros(idx.numel(), dtype=torch.int64)
        if j > 0:
            same = lay == lay_all[prev_e[idx]]
            pp2, CC2, _, st_p = propagate(pp, CC, qq, kind, pos_l[lay], x0_l[lay], geom, apply_material=True,
                                          same=same)
        else:
            Q, grazing = process_noise(pp, kind, x0_l[lay], geom.mass)
            pp2, CC2 = pp, CC + Q
            st_p = torch.where(grazing, GRAZING, 0).to(torch.int64)
        if state_round is not None:
            pp2 = pp2.to(state_round).to(DT)
            CC2 = CC2.to(state_round).to(DT)
        if state_jitter is not None:
            pp2, CC2 = _jitter(pp2, CC2, idx + j, state_jitter)
        st = st | st_p
        good = (st_p & NO_CROSSING) == 0
        valid = (val_all[ei] == 1) & good
        pu, Cu, qu, c2, st_u = update(pp2, CC2, qq, m_all[ei], V_all[ei])
        vmask = valid
        pn = torch.where(vmask[:, None], pu, pp2)
        Cn = torch.where(vmask[:, None, None], Cu, CC2)
        qn = torch.where(vmask, qu, qq)
        c2n = torch.where(vmask, c2, torch.zeros_like(c2))
        st = st | torch.where(vmask, st_u, 0)
        finite = torch.isfinite(pn).all(dim=1) & torch.isfinite(Cn).flatten(1).all(dim=1) & torch.isfinite(c2n)
        st = st | torch.where(finite, 0, NONFINITE)
        keep = good & finite
        # frozen tracks keep their previous state
        pn = torch.where(keep[:, None], pn, pp)
        Cn = torch.where(keep[:, None, None], Cn, CC)
        qn = torch.where(keep, qn, qq)
        c2n = torch.where(keep, c2n, torch.zeros_like(c2n))
        if state_round is not None:
            pn = pn.to(state_round).to(DT)
            Cn = Cn.to(state_round).to(DT)
        if state_jitter is not None:
            pn, Cn = _jitter(pn, Cn, idx + j + 1, state_jitter)
        p = p.index_put((idx,), pn)
        C = C.index_put((idx,), Cn)
        q = q.index_put((idx,), qn)
        chi2 = chi2.index_put((idx,), chi2[idx] + c2n)
        nval = nval.index_put((idx,), nval[idx] + (vmask & keep).to(torch.int64))
        status = status.index_put((idx,), status[idx] | st)
        alive = alive.index_put((idx,), keep)
        prev_e = prev_e.index_put((idx,), ei)
        if record:
            k = torch.nonzero(keep)[:, 0]
            pe = pe.index_put((ei[k],), pn[k])
            Ce = Ce.index_put((ei[k],), Cn[k])
            qe = qe.index_put((ei[k],), qn[k])
            ppe = ppe.index_put((ei[k],), pp2[k])
            Cpe = Cpe.index_put((ei[k],), CC2[k])
    out = dict(p=p, C=C, q=q, chi2=chi2, ndf=2 * nval - 5, status=status)
    if record:
        out.update(pe=pe, Ce=Ce, qe=qe, pp=ppe, Cp=Cpe)
    return out


def fit_event(ev, align=None, seed_mode=SEED_FIRST_THREE):
    """Convenience: seed (first three valid hits, or spaced hits), then fit."""
    sp, sC, sq, ok = make_seeds(ev.hit_offsets, ev.hit_valid, ev.hit_pos, ev.geometry.bz, mode=seed_mode)
    out = fit_tracks(sp, sC, sq, ev.hit_offsets, ev.hit_layer, ev.hit_valid, _t(ev.hit_pos), ev.hit_cov,
                     ev.geometry, align=align)
    out["seed_p"], out["seed_q"], out["seed_ok"] = sp, sq, ok
    return out


# --------------------------------------------------------------------------
# f1: backward fit
# --------------------------------------------------------------------------

# The backward pass restarts from the forward fit's last state with its
# covariance scaled up by this factor, so that the hits the forward pass
# already used count (almost) once only.  The paper gives no value.
BACKWARD_COV_SCALE = 100.0
# forward status bits after which a track is not refitted (the forward pass
# stopped before its last entry); such a track keeps its input and gets
# NOT_REFITTED, the value of the C interface's bad-input bit
NOT_REFITTED = 64
# final fit: at least one hit was rejected as an outlier
OUTLIER = 128
# the final fit's chi2 cut for one hit (3 measured coordinates, one of them
# the layer's thickness; the paper gives no value)
FINAL_CHI2_CUT = 30.0
# rounds in which the final fit may reject a hit, and the number of used hits
# a track keeps at the least (ndf = 2 * 4 - 5 = 3); the paper gives neither
FINAL_MAX_REJECT = 3
FINAL_MIN_KEEP = 4


def reverse_direction(p, C, q):
    """The same track moving the opposite way along its helix: direction
    (phi, theta) -> (phi + pi, pi - theta) and charge -q, position and ipt
    unchanged.  The helix then turns the other way (omega = -q c_B B_z ipt
    changes sign) and climbs the other way (cot theta changes sign), so it
    traces the same curve backwards.  The Jacobian of the map is
    J = diag(1, 1, 1, 1, 1, -1), hence C' = J C J.  p [n,6], C [n,6,6],
    q [n]."""
    p2 = torch.cat([p[:, :4], wrap_phi(p[:, 4:5] + math.pi), math.pi - p[:, 5:6]], dim=1)
    J = torch.diag(torch.tensor([1.0, 1.0, 1.0, 1.0, 1.0, -1.0], dtype=DT))
    return p2, J @ C @ J, -q


def impose_surface(p, C, kind, pos):
    """The covariance of a state on a surface has the surface normal as a null
    vector (a state confined to the surface cannot move along it): C <- P C P
    with P = I - n n^T on the position block, n = (x, y, 0) / R for a barrel
    of radius R = pos, n = (0, 0, 1) for a disk.  Exact arithmetic leaves such
    a covariance unchanged; it removes the rounding residue along n that a
    stored covariance carries."""
    p, C = _t(p), _t(C)
    n = p.shape[0]
    isb = torch.as_tensor(kind) == BARREL
    R = _t(pos)
    nx = torch.where(isb, p[:, 0] / R, torch.zeros_like(R))
    ny = torch.where(isb, p[:, 1] / R, torch.zeros_like(R))
    nz = torch.where(isb, torch.zeros_like(R), torch.ones_like(R))
    nv = torch.zeros(n, 6, dtype=DT)
    nv[:, 0], nv[:, 1], nv[:, 2] = nx, ny, nz
    P = torch.eye(6, dtype=DT).expand(n, 6, 6) - nv[:, :, None] * nv[:, None, :]
    return P @ C @ P


def surface_frame(p, kind, pos):
    """[n,6,5] orthonormal basis of the directions a state on its surface can
    move in: (tangent, z) for a barrel of radius pos (tangent = (-y, x)/R),
    (x, y) for a disk, then ipt, phi, theta."""
    p = _t(p)
    n = p.shape[0]
    isb = torch.as_tensor(kind) == BARREL
    R = _t(pos)
    B = torch.zeros(n, 6, 5, dtype=DT)
    B[:, 0, 0] = torch.where(isb, -p[:, 1] / R, torch.ones_like(R))
    B[:, 1, 0] = torch.where(isb, p[:, 0] / R, torch.zeros_like(R))
    B[:, 2, 1] = torch.where(isb, torch.ones_like(R), torch.zeros_like(R))
    B[:, 1, 1] = torch.where(isb, torch.zeros_like(R), torch.ones_like(R))
    B[:, 3, 2] = B[:, 4, 3] = B[:, 5, 4] = 1.0
    return B


def combine_on_surface(pf, Cf, pb, Cb, kind, pos):
    """Two estimates of one state on a surface, from disjoint sets of hits,
    combined (the two-filter smoother): with the gain K = C_f (C_f + C_b)^+,
    x = x_f + K (x_b - x_f) and C = (I - K) C_f (I - K)^T + K C_b K^T, where
    ^+ inverts on the 5-dimensional space the state can move in (the surface
    normal is a null vector of both covariances):
    (C_f + C_b)^+ = B (B^T (C_f + C_b) B)^-1 B^T with the frame B of
    surface_frame.  C equals C_f - C_f (C_f + C_b)^+ C_f; the symmetric form
    is used because that difference loses digits where C_f is much larger
    than the result (the first layers, where the forward state is still near
    its diffuse seed).  phi differences are wrapped."""
    B = surface_frame(pf, kind, pos)
    Bt = B.transpose(1, 2)
    d = pb - pf
    d = torch.cat([d[:, :4], wrap_phi(d[:, 4:5]), d[:, 5:]], dim=1)
    M = Bt @ (Cf + Cb) @ B
    K = Cf @ B @ torch.linalg.inv(M) @ Bt
    ps = pf + (K @ d[:, :, None])[:, :, 0]
    ps = torch.cat([ps[:, :4], wrap_phi(ps[:, 4:5]), ps[:, 5:]], dim=1)
    A = torch.eye(6, dtype=DT) - K
    Cs = A @ Cf @ A.transpose(1, 2) + K @ Cb @ K.transpose(1, 2)
    return ps, 0.5 * (Cs + Cs.transpose(1, 2))


def backward_fit(fwd_p, fwd_C, fwd_q, fwd_status, hit_offsets, hit_layer, hit_valid, hit_pos, hit_cov, geom,
                 cov_scale=BACKWARD_COV_SCALE, state_round=None, state_jitter=None, smooth_from=None):
    """Backward fit (Sec. 2.2, step 4): every track is traversed again, from
    its last entry back to its first valid entry, and refitted.

    Input: the forward fit's result (fwd_p [n,6], fwd_C [n,6,6], fwd_q [n],
    fwd_status [n]), which sits on the track's last entry.  Its covariance is
    multiplied by cov_scale, the surface of the last entry's layer imposed on
    it (impose_surface: scaled up, the rounding residue along the normal of a
    stored covariance would no longer be negligible) and the direction of
    motion reversed (reverse_direction); the entries are then taken in reverse order with the
    forward pass's rules: the first (the last entry) adds its layer's material
    at the current state, every later one is propagated to (the re-crossing
    window when the entry before it in this order was on the same layer),
    gets its layer's material and, if valid, an update; a failed crossing or a
    non-finite result freezes the track.  The result, on the first valid
    entry, is turned back to the outward direction.  Tracks the forward pass
    stopped (NO_CROSSING or NONFINITE in fwd_status) or with no valid entry
    keep their input, with status NOT_REFITTED.  state_round, state_jitter:
    the conditioning probes of fit_tracks, applied after every propagation
    and update.

    smooth_from: None, or the forward fit's filtered state after every entry
    (dict(pe, Ce) of fit_tracks(record=True)); then the smoothed state of
    every entry from the first valid one to the last is returned as well
    (ps [nh,6], Cs [nh,6,6], NaN elsewhere).  The forward filtered state of an
    entry holds its layer's scattering and hit and those before; the
    backward pass's state on arriving at the entry, before that layer's
    material, holds the hits after it; both describe the track just outside
    the layer, and combine_on_surface combines them.  The last entry's
    smoothed state is its forward filtered state.  With smoothing, the
    backward pass propagates without material, combines, then adds the
    layer's material (the same arithmetic as propagate with material).

    Returns dict(p, C, q, chi2, ndf, status): chi2 and ndf
    (= 2 * used hits - 5) of the backward pass."""
    off = torch.as_tensor(hit_offsets, dtype=torch.int64)
    lay_all = torch.as_tensor(hit_layer, dtype=torch.int64)
    val_all = torch.as_tensor(hit_valid, dtype=torch.int64)
    V_all = unpack_sym(hit_cov, 3)
    m_all = hit_pos if torch.is_tensor(hit_pos) else _t(hit_pos)
    m_all = m_all.T
    kind_l = torch.as_tensor(geom.kind, dtype=torch.int64)
    pos_l = _t(geom.pos)
    x0_l = _t(geom.x_over_x0)
    n = off.shape[0] - 1
    fwd_status = torch.as_tensor(fwd_status, dtype=torch.int64)

    # first valid entry of each track (forward order); the pass runs from the
    # last entry down to it
    k0 = torch.full((n,), -1, dtype=torch.int64)
    lens = off[1:] - off[:-1]
    maxlen = int(lens.max()) if n > 0 else 0
    for j in range(maxlen - 1, -1, -1):
        e = off[:-1] + j
        has = j < lens
        ev = torch.where(has, e, torch.zeros_like(e))
        k0 = torch.where(has & (val_all[ev] == 1), e, k0)
    last = off[1:] - 1
    run = (k0 >= 0) & ((fwd_status & (NO_CROSSING | NONFINITE | NOT_REFITTED)) == 0)

    lay_last = lay_all[torch.clamp(last, min=0)] if n > 0 else lay_all[:0]
    C0 = impose_surface(fwd_p, _t(fwd_C) * cov_scale, kind_l[lay_last], pos_l[lay_last])
    p, C, q = reverse_direction(_t(fwd_p), C0, _t(fwd_q))
    smooth = smooth_from is not None
    if smooth:
        nh = lay_all.shape[0]
        ps_all = torch.full((nh, 6), float("nan"), dtype=DT)
        Cs_all = torch.full((nh, 6, 6), float("nan"), dtype=DT)
        pb_all = torch.full((nh, 6), float("nan"), dtype=DT)
        Cb_all = torch.full((nh, 6, 6), float("nan"), dtype=DT)
        pe_f, Ce_f = _t(smooth_from["pe"]), _t(smooth_from["Ce"])
    chi2 = torch.zeros(n, dtype=DT)
    nval = torch.zeros(n, dtype=torch.int64)
    status = torch.zeros(n, dtype=torch.int64)
    alive = run.clone()
    prev_e = last.clone()
    for j in range(maxlen):
        e = last - j
        act = alive & (e >= k0)
        idx = torch.nonzero(act)[:, 0]
        if idx.numel() == 0:
            break
        ei = e[idx]
        lay = lay_all[ei]
        kind = kind_l[lay]
        pp, CC, qq = p[idx], C[idx], q[idx]
        if j > 0 and smooth:
            same = lay == lay_all[prev_e[idx]]
            pp2, CC2, _, st = propagate(pp, CC, qq, kind, pos_l[lay], x0_l[lay], geom, apply_material=False,
                                        same=same)
            reach = (st & NO_CROSSING) == 0
            pb, Cb, _ = reverse_direction(pp2, CC2, qq)
            ps, Cs = combine_on_surface(pe_f[ei], Ce_f[ei], pb, Cb, kind, pos_l[lay])
            r = torch.nonzero(reach)[:, 0]
            ps_all = ps_all.index_put((ei[r],), ps[r])
            Cs_all = Cs_all.index_put((ei[r],), Cs[r])
            pb_all = pb_all.index_put((ei[r],), pb[r])
            Cb_all = Cb_all.index_put((ei[r],), Cb[r])
            Q, grazing = process_noise(pp2, kind, x0_l[lay], geom.mass)
            CC2 = CC2 + Q
            st = st | torch.where(grazing & reach, GRAZING, 0)
        elif j > 0:
            same = lay == lay_all[prev_e[idx]]
            pp2, CC2, _, st = propagate(pp, CC, qq, kind, pos_l[lay], x0_l[lay], geom, apply_material=True, same=same)
        else:
            if smooth:
                ps_all = ps_all.index_put((ei,), pe_f[ei])
                Cs_all = Cs_all.index_put((ei,), Ce_f[ei])
            Q, grazing = process_noise(pp, kind, x0_l[lay], geom.mass)
            pp2, CC2 = pp, CC + Q
            st = torch.where(grazing, GRAZING, 0).to(torch.int64)
        if state_round is not None:
            pp2 = pp2.to(state_round).to(DT)
            CC2 = CC2.to(state_round).to(DT)
        if state_jitter is not None:
            pp2, CC2 = _jitter(pp2, CC2, idx + j, state_jitter)
        good = (st & NO_CROSSING) == 0
        valid = (val_all[ei] == 1) & good
        pu, Cu, qu, c2, st_u = update(pp2, CC2, qq, m_all[ei], V_all[ei])
        pn = torch.where(valid[:, None], pu, pp2)
        Cn = torch.where(valid[:, None, None], Cu, CC2)
        qn = torch.where(valid, qu, qq)
        c2n = torch.where(valid, c2, torch.zeros_like(c2))
        st = st | torch.where(valid, st_u, 0)
        finite = torch.isfinite(pn).all(dim=1) & torch.isfinite(Cn).flatten(1).all(dim=1) & torch.isfinite(c2n)
        st = st | torch.where(finite, 0, NONFINITE)
        keep = good & finite
        pn = torch.where(keep[:, None], pn, pp)
        Cn = torch.where(keep[:, None, None], Cn, CC)
        qn = torch.where(keep, qn, qq)
        c2n = torch.where(keep, c2n, torch.zeros_like(c2n))
        if state_round is not None:
            pn = pn.to(state_round).to(DT)
            Cn = Cn.to(state_round).to(DT)
        if state_jitter is not None:
            pn, Cn = _jitter(pn, Cn, idx + j + 1, state_jitter)
        p = p.index_put((idx,), pn)
        C = C.index_put((idx,), Cn)
        q = q.index_put((idx,), qn)
        chi2 = chi2.index_put((idx,), chi2[idx] + c2n)
        nval = nval.index_put((idx,), nval[idx] + (valid & keep).to(torch.int64))
        status = status.index_put((idx,), status[idx] | st)
        alive = alive.index_put((idx,), keep)
        prev_e = prev_e.index_put((idx,), ei)
    p, C, q = reverse_direction(p, C, q)
    # tracks not refitted keep their input
    p = torch.where(run[:, None], p, _t(fwd_p))
    C = torch.where(run[:, None, None], C, _t(fwd_C))
    q = torch.where(run, q, _t(fwd_q))
    status = torch.where(run, status, torch.full_like(status, NOT_REFITTED))
    out = dict(p=p, C=C, q=q, chi2=chi2, ndf=2 * nval - 5, status=status)
    if smooth:
        # the entries the backward pass reached
        out.update(ps=ps_all, Cs=Cs_all, pb=pb_all, Cb=Cb_all)
    return out


# --------------------------------------------------------------------------
# f4: final fit with outlier rejection
# --------------------------------------------------------------------------

def unbiased_chi2(pp, Cp, pb, Cb, kind, pos, m, V):
    """chi2 of a hit against the estimate of its track made from all the other
    hits: that estimate is the forward prediction at the hit's entry (its
    propagation and material, before its update: the hits before it)
    combined with the backward pass's prediction there (the hits after it)
    by combine_on_surface, or the forward prediction alone on the last entry
    (pb NaN: the backward pass starts there from a result that holds the
    hit).  With x, C that estimate: r = m - H x, S = V + H C H^T,
    chi2 = r^T S^-1 r.  In the linear model this equals r_s^T (V - H C_s H^T)^-1
    r_s of the smoothed residual r_s = m - H x_s, but it is formed from a sum
    and a residual of full size, so it keeps its digits where the hit
    dominates the smoothed state.  pp, pb [k,6], Cp, Cb [k,6,6], kind, pos [k]
    (the entry's surface), m [k,3], V [k,3,3].  NaN where the forward
    prediction is missing or the combination fails."""
    pp, Cp, pb, Cb, m, V = _t(pp), _t(Cp), _t(pb), _t(Cb), _t(m), _t(V)
    kind, pos = torch.as_tensor(kind), _t(pos)
    have_f = torch.isfinite(pp).all(dim=1) & torch.isfinite(Cp).flatten(1).all(dim=1)
    have_b = torch.isfinite(pb).all(dim=1) & torch.isfinite(Cb).flatten(1).all(dim=1)
    px, Cx = pp.clone(), Cp.clone()            # the last entry: the forward prediction alone
    both = torch.nonzero(have_f & have_b)[:, 0]
    if both.numel():
        B = surface_frame(pp[both], kind[both], pos[both])
        M = B.transpose(1, 2) @ (Cp[both] + Cb[both]) @ B
        _, info = torch.linalg.cholesky_ex(M)
        good = info == 0
        pc, Cc = combine_on_surface(pp[both], Cp[both], pb[both], Cb[both], kind[both], pos[both]) \
            if bool(good.all()) else _combine_guarded(pp[both], Cp[both], pb[both], Cb[both], kind[both],
                                                       pos[both], good)
        px[both], Cx[both] = pc, Cc
    r = m - px[:, :3]
    S = V + Cx[:, :3, :3]
    fin = have_f & torch.isfinite(r).all(dim=1) & torch.isfinite(S).flatten(1).all(dim=1)
    Ss = torch.where(fin[:, None, None], S, torch.eye(3, dtype=DT).expand_as(S))
    rs = torch.where(fin[:, None], r, torch.zeros_like(r))
    chi2 = torch.einsum("ni,nij,nj->n", rs, torch.linalg.inv(Ss), rs)
    return torch.where(fin, chi2, torch.full_like(chi2, float("nan")))


def _combine_guarded(pf, Cf, pb, Cb, kind, pos, good):
    """combine_on_surface where its 5x5 system is positive definite (good),
    NaN elsewhere."""
    n = pf.shape[0]
    ps = torch.full((n, 6), float("nan"), dtype=DT)
    Cs = torch.full((n, 6, 6), float("nan"), dtype=DT)
    g = torch.nonzero(good)[:, 0]
    if g.numel():
        ps[g], Cs[g] = combine_on_surface(pf[g], Cf[g], pb[g], Cb[g], kind[g], pos[g])
    return ps, Cs


def final_fit(hit_offsets, hit_layer, hit_valid, hit_pos, hit_cov, geom, seed_mode=SEED_FIRST_THREE,
              chi2_cut=FINAL_CHI2_CUT, max_reject=FINAL_MAX_REJECT, min_keep=FINAL_MIN_KEEP,
              cov_scale=BACKWARD_COV_SCALE, state_round=None, state_jitter=None):
    """Final fit with outlier rejection (the final fit the paper names in
    Sec. 2.2 and Sec. 4, with a hit-rejection rule of this reading): rounds of
    refit and reject-the-worst.

    Round i (i = 0 .. max_reject), for every track still open: seed from its
    used hits (its valid hits not yet rejected; seed_mode as make_seeds), the
    forward fit over them recording the filtered state after every entry,
    then the backward fit with the two-filter smoother (backward_fit with
    smooth_from), which gives the backward predictions.  Each used hit gets
    its unbiased chi2 (unbiased_chi2: against the estimate from the track's
    other hits, the combination of the two predictions at its entry); the
    hits of a track that the backward pass did not refit (NOT_REFITTED: its
    forward fit stopped or could not be seeded) get NaN, as there is no such
    estimate.  If i < max_reject, the track
    was refitted, its worst used hit (largest chi2, the first entry among
    equals; NaN never counts) has chi2 > chi2_cut and the track keeps at least
    min_keep used hits without it, that hit is rejected (marked in outlier,
    no longer used) and the track stays open; otherwise the track is closed
    with this round's backward-fit result (state on its first used entry,
    chi2 and ndf = 2 * used - 5 of the backward pass, its status, plus OUTLIER
    if any hit was rejected).

    Returns dict(p, C, q, chi2, ndf, status, outlier [nh] bool, hit_chi2 [nh]
    (a used hit: its chi2 in the round its track closed; a rejected hit: its
    chi2 in the round it was rejected; NaN for the rest), rounds [n] (the
    round each track closed in)).  state_round / state_jitter: the
    conditioning probes of fit_tracks, applied to the seeds and every pass."""
    off = torch.as_tensor(hit_offsets, dtype=torch.int64)
    n = off.shape[0] - 1
    lay_all = torch.as_tensor(hit_layer, dtype=torch.int64)
    nh = lay_all.shape[0]
    lens = off[1:] - off[:-1]
    track_of = torch.repeat_interleave(torch.arange(n), lens)
    hp = hit_pos if torch.is_tensor(hit_pos) else _t(hit_pos)
    m_all = hp.T
    V_all = unpack_sym(hit_cov, 3)
    used = torch.as_tensor(hit_valid, dtype=torch.int64).clone()
    outlier = torch.zeros(nh, dtype=torch.bool)
    hit_chi2 = torch.full((nh,), float("nan"), dtype=DT)
    is_open = torch.ones(n, dtype=torch.bool)
    rejected_any = torch.zeros(n, dtype=torch.bool)
    res = dict(p=torch.zeros(n, 6, dtype=DT), C=torch.zeros(n, 6, 6, dtype=DT), q=torch.zeros(n, dtype=DT),
               chi2=torch.zeros(n, dtype=DT), ndf=torch.zeros(n, dtype=torch.int64),
               status=torch.zeros(n, dtype=torch.int64), rounds=torch.zeros(n, dtype=torch.int64))
    idx = torch.arange(nh)
    for rnd in range(max_reject + 1):
        if not bool(is_open.any()):
            break
        sp, sC, sq, _ = make_seeds(hit_offsets, used, hp.detach(), geom.bz, mode=seed_mode)
        if state_round is not None:
            sp = sp.to(state_round).to(DT)
        fwd = fit_tracks(sp, sC, sq, hit_offsets, hit_layer, used, hp, hit_cov, geom, state_round=state_round,
                         state_jitter=state_jitter, record=True)
        bwd = backward_fit(fwd["p"], fwd["C"], fwd["q"], fwd["status"], hit_offsets, hit_layer, used, hp, hit_cov,
                           geom, cov_scale=cov_scale, state_round=state_round, state_jitter=state_jitter,
                           smooth_from=fwd)
        kind_e = torch.as_tensor(geom.kind, dtype=torch.int64)[lay_all]
        pos_e = _t(geom.pos)[lay_all]
        c2 = unbiased_chi2(fwd["pp"], fwd["Cp"], bwd["pb"], bwd["Cb"], kind_e, pos_e, m_all, V_all)
        # a track the backward pass did not refit (its forward fit stopped or
        # could not be seeded) has no estimate from its other hits
        refitted = (bwd["status"] & NOT_REFITTED) == 0
        c2 = torch.where(refitted[track_of], c2, torch.full_like(c2, float("nan")))
        in_open = is_open[track_of] & (used == 1)
        hit_chi2 = torch.where(in_open, c2, hit_chi2)
        # the worst used hit of each track: the largest chi2, the first entry among equals
        val = torch.where(in_open & torch.isfinite(c2), c2, torch.full_like(c2, -math.inf))
        worst = torch.full((n,), -math.inf, dtype=DT).scatter_reduce(0, track_of, val, reduce="amax")
        first = torch.where(val == worst[track_of], idx, torch.full_like(idx, nh))
        e_w = torch.full((n,), nh, dtype=torch.int64).scatter_reduce(0, track_of, first, reduce="amin")
        n_used = torch.zeros(n, dtype=torch.int64).index_add(0, track_of, (used == 1).to(torch.int64))
        rej = is_open & refitted & (worst > chi2_cut) & (n_used - 1 >= min_keep) & (rnd < max_reject)
        close = is_open & ~rej
        for k in ("p", "C", "q", "chi2", "ndf", "status"):
            sel = close.view(-1, *([1] * (bwd[k].dim() - 1)))
            res[k] = torch.where(sel, bwd[k], res[k])
        res["rounds"] = torch.where(close, rnd, res["rounds"])
        t_rej = torch.nonzero(rej)[:, 0]
        outlier[e_w[t_rej]] = True
        used[e_w[t_rej]] = 0
        rejected_any |= rej
        is_open &= ~close
    res["status"] = res["status"] | torch.where(rejected_any, OUTLIER, 0)
    res.update(outlier=outlier, hit_chi2=hit_chi2)
    return res


# --------------------------------------------------------------------------
# a8: gradient of sum_t w_t chi2_t (reverse-mode autodiff of the oracle)
# --------------------------------------------------------------------------

def fit_gradients(seed_p, seed_C, seed_q, hit_offsets, hit_layer, hit_valid, hit_pos, hit_cov, geom,
                  align=None, weights=None, state_round=None):
    """d(sum_t w_t chi2_t)/d(seed state, hit positions, alignment), by autograd
    through fit_tracks (a mechanism independent of any hand-written reverse).
    state_round is passed to fit_tracks (a conditioning probe: the rounding
    is the identity for the gradient).
    Returns (loss, g_seed [n,6], g_hits [3,nh], g_align [2,L], fit_out)."""
    sp = _t(seed_p).detach().clone().requires_grad_(True)
    hp = _t(hit_pos).detach().clone().requires_grad_(True)
    L = len(geom.kind)
    al = (torch.zeros(2, L, dtype=DT) if align is None else _t(align)).detach().clone().requires_grad_(True)
    out = fit_tracks(sp, _t(seed_C), _t(seed_q), hit_offsets, hit_layer, hit_valid, hp, hit_cov, geom, align=al,
                     state_round=state_round)
    w = torch.ones_like(out["chi2"]) if weights is None else _t(weights)
    loss = (w * out["chi2"]).sum()
    gs, gh, ga = torch.autograd.grad(loss, [sp, hp, al], allow_unused=True)
    gs = torch.zeros_like(sp) if gs is None else gs
    gh = torch.zeros_like(hp) if gh is None else gh
    ga = torch.zeros_like(al) if ga is None else ga
    return loss.detach(), gs, gh, ga, {k: (v.detach() if torch.is_tensor(v) else v) for k, v in out.items()}
