"""Seeded synthetic events for the Kalman-filter workloads.

The paper measures on simulated CMS events, which are not available; these
toys stand in for them.  Charged particles follow exact helices in a uniform
B_z, scatter once at every crossed layer, and leave one smeared hit per
crossing.  The helix is computed here in a rotation form (the momentum
direction and the position turn about the circle centre) with crossings found
by circle-circle intersection.  That code is this module's own; the filter
implementations (the CPU oracle and the GPU kernels) each carry their own
propagation and share nothing with it.

Random streams: ``numpy.random.Generator(PCG64)`` seeded from
``SeedSequence(seed)`` spawned into five children: tracks, smearing, kicks,
holes, noise.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .detector import BARREL, DISK, Geometry, Workload

C_LIGHT = 0.00299792458  # GeV/c per (T cm)
S_EPS = 1e-6             # cm; a crossing closer than this to the start is the start itself
GRAZING_COS = 0.05


@dataclass
class Event:
    """One batch of tracks in CSR form (SoA arrays, float64)."""
    geometry: Geometry
    charge: np.ndarray        # int8 [n]
    vertex: np.ndarray        # float64 [n, 6]: x, y, z, 1/pT, phi, theta at production
    hit_offsets: np.ndarray   # int32 [n+1]
    hit_layer: np.ndarray     # int16 [nh]
    hit_valid: np.ndarray     # uint8 [nh]
    hit_pos: np.ndarray       # float64 [3, nh]
    hit_cov: np.ndarray       # float64 [6, nh] packed lower triangle (xx, yx, yy, zx, zy, zz)
    truth: np.ndarray         # float64 [nh, 6] true state at the crossing, before the kick
    truth_after: np.ndarray   # float64 [nh, 6] true state just after the kick
    align_true: np.ndarray    # float64 [2, L] injected per-layer offsets (zero if none)

    @property
    def n_tracks(self) -> int:
        return int(self.charge.shape[0])

    @property
    def n_hits(self) -> int:
        return int(self.hit_layer.shape[0])

    def lengths(self) -> np.ndarray:
        return np.diff(self.hit_offsets)


def _wrap(a):
    return np.mod(a + np.pi, 2.0 * np.pi) - np.pi


def _advance(x, y, z, phi, cot, omega, s):
    """Move along the helix by transverse path s: rotate the offset from the
    circle centre by the turning angle omega*s."""
    xc = x - np.sin(phi) / omega
    yc = y + np.cos(phi) / omega
    u = omega * s
    cu, su = np.cos(u), np.sin(u)
    vx, vy = x - xc, y - yc
    nx = xc + cu * vx - su * vy
    ny = yc + su * vx + cu * vy
    return nx, ny, z + s * cot, phi + u


def _barrel_candidates(x, y, phi, omega, R):
    """Both path lengths (in the first turn, > S_EPS) at which the circle of the
    track meets the cylinder r = R; NaN where it does not."""
    xc = x - np.sin(phi) / omega
    yc = y + np.cos(phi) / omega
    d = np.hypot(xc, yc)
    d2_minus_rho2 = x * x + y * y - 2.0 * (x * np.sin(phi) - y * np.cos(phi)) / omega
    a = (R * R + d2_minus_rho2) / (2.0 * d)
    h2 = R * R - a * a
    ok = h2 >= 0.0
    h = np.sqrt(np.where(ok, h2, 0.0))
    ex, ey = xc / d, yc / d
    period = 2.0 * np.pi / np.abs(omega)
    out = []
    for sgn in (1.0, -1.0):
        px = a * ex - sgn * h * ey
        py = a * ey + sgn * h * ex
        v0x, v0y = x - xc, y - yc
        v1x, v1y = px - xc, py - yc
        ang = np.arctan2(v0x * v1y - v0y * v1x, v0x * v1x + v0y * v1y)
        s = ang / omega
        s = np.where(s <= S_EPS, s + period, s)
        s = np.where(s <= S_EPS, s + period, s)
        out.append(np.where(ok, s, np.nan))
    return out


def _highland(p, beta, x):
    return 0.0136 / (beta * p) * np.sqrt(x) * (1.0 + 0.038 * np.log(x / (beta * beta)))


def _hit_cov_barrel(phi_h, s_rphi, s_z, s_n):
    sn, cs = np.sin(phi_h), np.cos(phi_h)
    n = phi_h.shape[0]
    cov = np.zeros((6, n))
    cov[0] = s_rphi ** 2 * sn * sn + s_n ** 2 * cs * cs
    cov[1] = (s_n ** 2 - s_rphi ** 2) * sn * cs
    cov[2] = s_rphi ** 2 * cs * cs + s_n ** 2 * sn * sn
    cov[5] = s_z ** 2
    return cov


def _hit_cov_disk(phi_h, s_rphi, s_r, s_n):
    sn, cs = np.sin(phi_h), np.cos(phi_h)
    n = phi_h.shape[0]
    cov = np.zeros((6, n))
    cov[0] = s_rphi ** 2 * sn * sn + s_r ** 2 * cs * cs
    cov[1] = (s_r ** 2 - s_rphi ** 2) * sn * cs
    cov[2] = s_rphi ** 2 * cs * cs + s_r ** 2 * sn * sn
    cov[5] = s_n ** 2
    return cov


def _simulate(wl: Workload, n: int, rng_trk, rng_smear, rng_kick, smear: bool, scatter: bool):
    g = wl.geometry
    L = g.n_layers
    # production
    vx = rng_trk.normal(0.0, 0.01, n)
    vy = rng_trk.normal(0.0, 0.01, n)
    vz = rng_trk.normal(0.0, 5.0, n)
    pt = np.exp(rng_trk.uniform(np.log(wl.pt_min), np.log(wl.pt_max), n))
    eta = rng_trk.uniform(-wl.eta_max, wl.eta_max, n)
    phi = rng_trk.uniform(0.0, 2.0 * np.pi, n)
    q = np.where(rng_trk.uniform(0.0, 1.0, n) < 0.5, 1, -1).astype(np.int8)
    theta = 2.0 * np.arctan(np.exp(-eta))
    vertex = np.stack([vx, vy, vz, 1.0 / pt, _wrap(phi), theta], axis=1)

    x, y, z = vx.copy(), vy.copy(), vz.copy()
    ptot = pt / np.sin(theta)
    alive = np.ones(n, bool)
    nxt = np.zeros(n, np.int64)          # outward mode: index of the next barrel
    rec_layer = np.full((n, wl.max_entries), -1, np.int64)
    rec_hit = np.zeros((n, wl.max_entries, 3))
    rec_cov = np.zeros((n, wl.max_entries, 6))
    rec_truth = np.zeros((n, wl.max_entries, 6))
    rec_after = np.zeros((n, wl.max_entries, 6))
    count = np.zeros(n, np.int64)
    idx_all = np.arange(n)

    for _step in range(wl.max_entries):
        act = np.nonzero(alive)[0]
        if act.size == 0:
            break
        xa, ya, za, pha = x[act], y[act], z[act], phi[act]
        tha = theta[act]
        pta = ptot[act] * np.sin(tha)
        cot = np.cos(tha) / np.sin(tha)
        om = -q[act].astype(np.float64) * C_LIGHT * g.bz / pta
        best_s = np.full(act.size, np.inf)
        best_l = np.full(act.size, -1, np.int64)
        if wl.mode == "outward":
            cand_layers = [None]
        else:
            cand_layers = range(L)
        for lay in cand_layers:
            if lay is None:
                lidx = nxt[act]
                valid_l = lidx < L
                lsafe = np.where(valid_l, lidx, 0)
                R = g.pos[lsafe]
                s1, s2 = _barrel_candidates(xa, ya, pha, om, R)
                s = np.fmin(s1, s2)  # first crossing only (outgoing)
                s = np.where(valid_l, s, np.nan)
                sv = np.where(np.isnan(s), 0.0, s)
                _, _, zz, _ = _advance(xa, ya, za, pha, cot, om, sv)
                inside = (zz >= g.lo[lsafe]) & (zz <= g.hi[lsafe])
                s = np.where(inside, s, np.nan)
                take = np.isfinite(s)
                best_s = np.where(take, s, best_s)
                best_l = np.where(take, lsafe, best_l)
                continue
            if g.kind[lay] == BARREL:
                cands = _barrel_candidates(xa, ya, pha, om, g.pos[lay])
                for s in cands:
                    sv = np.where(np.isnan(s), 0.0, s)
                    _, _, zz, _ = _advance(xa, ya, za, pha, cot, om, sv)
                    ok = np.isfinite(s) & (zz >= g.lo[lay]) & (zz <= g.hi[lay])
                    better = ok & (s < best_s)
                    best_s = np.where(better, s, best_s)
                    best_l = np.where(better, lay, best_l)
            else:
                with np.errstate(divide="ignore", invalid="ignore"):
                    s = (g.pos[lay] - za) / cot
                s = np.where(np.isfinite(s) & (s > S_EPS), s, np.nan)
                sv = np.where(np.isnan(s), 0.0, s)
                xx, yy, _, _ = _advance(xa, ya, za, pha, cot, om, sv)
                rr = np.hypot(xx, yy)
                ok = np.isfinite(s) & (rr >= g.lo[lay]) & (rr <= g.hi[lay])
                better = ok & (s < best_s)
                best_s = np.where(better, s, best_s)
                best_l = np.where(better, lay, best_l)

        # the track ends once it leaves the tracker volume (r > r_env or
        # |z| > z_env) before reaching the next surface: nothing outside can
        # bend it back in
        r_env = float(np.max(np.where(g.kind == BARREL, g.pos, g.hi)))
        z_env = float(np.max(np.where(g.kind == BARREL, np.maximum(np.abs(g.lo), np.abs(g.hi)), np.abs(g.pos))))
        e1, e2 = _barrel_candidates(xa, ya, pha, om, np.full(act.size, r_env))
        rr0 = np.hypot(xa, ya)
        outward = (xa * np.cos(pha) + ya * np.sin(pha)) > 0
        s_env = np.where((rr0 >= r_env - 1e-9) & outward, 0.0, np.fmin(e1, e2))
        s_env = np.where(np.isnan(s_env), np.inf, s_env)
        with np.errstate(divide="ignore", invalid="ignore"):
            s_z = np.where(cot > 0, (z_env - za) / cot, np.where(cot < 0, (-z_env - za) / cot, np.inf))
        s_z = np.where(np.abs(za) >= z_env - 1e-9, np.where(za * cot > 0, 0.0, s_z), s_z)
        best_s = np.where(best_s > np.minimum(s_env, s_z) + 1e-7, np.inf, best_s)
        found = np.isfinite(best_s)
        sv = np.where(found, best_s, 0.0)
        nx, ny, nz, nphi = _advance(xa, ya, za, pha, cot, om, sv)
        lsafe = np.where(found, best_l, 0)
        is_barrel = g.kind[lsafe] == BARREL
        # snap onto the surface (removes the last ulp of drift)
        rr = np.hypot(nx, ny)
        Rl = g.pos[lsafe]
        nx = np.where(is_barrel, nx * Rl / rr, nx)
        ny = np.where(is_barrel, ny * Rl / rr, ny)
        nz = np.where(is_barrel, nz, Rl)
        pos_phi = np.arctan2(ny, nx)
        cos_a = np.where(is_barrel, np.sin(tha) * np.cos(nphi - pos_phi), np.abs(np.cos(tha)))
        grazing = np.abs(cos_a) < GRAZING_COS
        ok = found & ~grazing
        dead = act[~ok]
        alive[dead] = False
        act2 = act[ok]
        if act2.size == 0:
            break
        sel = ok
        nx, ny, nz, nphi = nx[sel], ny[sel], nz[sel], nphi[sel]
        lay2 = best_l[sel]
        is_b = is_barrel[sel]
        th2 = tha[sel]
        pt2 = pta[sel]
        cos_a2 = np.abs(cos_a[sel])
        k = count[act2]
        truth = np.stack([nx, ny, nz, 1.0 / pt2, _wrap(nphi), th2], axis=1)
        rec_layer[act2, k] = lay2
        rec_truth[act2, k] = truth

        # hit: smear along the surface so the hit stays exactly on it
        m = act2.size
        g_rphi = rng_smear.normal(0.0, 1.0, m) if smear else np.zeros(m)
        g_2 = rng_smear.normal(0.0, 1.0, m) if smear else np.zeros(m)
        r_true = np.hypot(nx, ny)
        phi_true = np.arctan2(ny, nx)
        phi_h = phi_true + wl.sigma_rphi * g_rphi / r_true
        hx = np.where(is_b, g.pos[lay2] * np.cos(phi_h), 0.0)
        hy = np.where(is_b, g.pos[lay2] * np.sin(phi_h), 0.0)
        hz = np.where(is_b, nz + wl.sigma_z * g_2, g.pos[lay2])
        r_h = r_true + wl.sigma_r * g_2
        hx = np.where(is_b, hx, r_h * np.cos(phi_h))
        hy = np.where(is_b, hy, r_h * np.sin(phi_h))
        rec_hit[act2, k] = np.stack([hx, hy, hz], axis=1)
        covb = _hit_cov_barrel(phi_h, wl.sigma_rphi, wl.sigma_z, wl.sigma_n)
        covd = _hit_cov_disk(phi_h, wl.sigma_rphi, wl.sigma_r, wl.sigma_n)
        rec_cov[act2, k] = np.where(is_b[None, :], covb, covd).T

        # multiple scattering kick at this crossing
        p2 = ptot[act2]
        beta = p2 / np.sqrt(p2 * p2 + g.mass ** 2)
        xl = g.x_over_x0[lay2] / cos_a2
        th0 = _highland(p2, beta, xl)
        if scatter:
            d_th = rng_kick.normal(0.0, 1.0, m) * th0
            d_ps = rng_kick.normal(0.0, 1.0, m) * th0
        else:
            d_th = np.zeros(m)
            d_ps = np.zeros(m)
        new_th = np.clip(th2 + d_th, 1e-3, np.pi - 1e-3)
        new_phi = nphi + d_ps / np.sin(th2)
        after = np.stack([nx, ny, nz, 1.0 / (p2 * np.sin(new_th)), _wrap(new_phi), new_th], axis=1)
        rec_after[act2, k] = after
        x[act2], y[act2], z[act2] = nx, ny, nz
        phi[act2] = new_phi
        theta[act2] = new_th
        count[act2] += 1
        if wl.mode == "outward":
            nxt[act2] = lay2 + 1
    return q, vertex, rec_layer, rec_hit, rec_cov, rec_truth, rec_after, count


def generate(wl: Workload, n_tracks: int | None = None, *, smear: bool = True,
             scatter: bool = True, holes: bool = True, min_hits: int = 3) -> Event:
    """Generate ``n_tracks`` tracks (default: the workload size)."""
    n = wl.n_tracks if n_tracks is None else int(n_tracks)
    ss = np.random.SeedSequence(wl.seed)
    r_trk, r_smear, r_kick, r_hole, r_noise, r_stop = [np.random.Generator(np.random.PCG64(c)) for c in ss.spawn(6)]
    g = wl.geometry

    chunks = []
    have = 0
    over = 1.15 if (wl.hole_fraction > 0 or wl.mode != "outward") else 1.02
    while have < n:
        m = max(64, int((n - have) * over) + 16)
        q, vtx, lay, hit, cov, tru, aft, cnt = _simulate(wl, m, r_trk, r_smear, r_kick, smear, scatter)
        if wl.stop_fraction > 0:
            # a central track (|eta| < 1, barrel crossings only) that ends
            # early keeps its first k crossings, k uniform in 3 .. n
            central = np.abs(1.0 / np.tan(tru[:, 0, 5])) < np.sinh(1.0)
            stop = (r_stop.uniform(0.0, 1.0, m) < wl.stop_fraction) & central
            k = r_stop.integers(3, np.maximum(cnt, 3) + 1)
            cnt = np.where(stop & (cnt > 3), np.minimum(k, cnt), cnt)
        valid = np.zeros(lay.shape, np.uint8)
        for i in range(lay.shape[1]):
            valid[:, i] = (i < cnt).astype(np.uint8)
        if holes and wl.hole_fraction > 0:
            drop = r_hole.uniform(0.0, 1.0, lay.shape) < wl.hole_fraction
            valid = np.where(drop & (valid == 1), 0, valid).astype(np.uint8)
        nvalid = valid.sum(axis=1)
        keep = np.nonzero((cnt >= min_hits) & (nvalid >= min_hits))[0]
        keep = keep[: n - have]
        chunks.append((q[keep], vtx[keep], lay[keep], hit[keep], cov[keep], tru[keep], aft[keep],
                       cnt[keep], valid[keep]))
        have += keep.size

    q = np.concatenate([c[0] for c in chunks])
    vtx = np.concatenate([c[1] for c in chunks])
    lay = np.concatenate([c[2] for c in chunks])
    hit = np.concatenate([c[3] for c in chunks])
    cov = np.concatenate([c[4] for c in chunks])
    tru = np.concatenate([c[5] for c in chunks])
    aft = np.concatenate([c[6] for c in chunks])
    cnt = np.concatenate([c[7] for c in chunks])
    valid = np.concatenate([c[8] for c in chunks])

    mask = np.arange(lay.shape[1])[None, :] < cnt[:, None]
    offsets = np.zeros(n + 1, np.int32)
    offsets[1:] = np.cumsum(cnt)
    hit_layer = lay[mask].astype(np.int16)
    hit_valid = valid[mask].astype(np.uint8)
    hit_pos = hit[mask].T.copy()
    hit_cov = cov[mask].T.copy()
    truth = tru[mask]
    truth_after = aft[mask]

    align_true = np.zeros((2, g.n_layers))
    if wl.misalign_rphi > 0 or wl.misalign_z > 0:
        align_true[0] = r_noise.normal(0.0, wl.misalign_rphi, g.n_layers)
        align_true[1] = r_noise.normal(0.0, wl.misalign_z, g.n_layers)
        align_true[:, g.kind != BARREL] = 0.0
        # the measured position is displaced by minus the offset; applying the
        # offset as a correction (rotate by a_rphi/R, shift z by a_z) restores it
        R = g.pos[hit_layer]
        ang = -align_true[0, hit_layer] / R
        c, s = np.cos(ang), np.sin(ang)
        hx, hy = hit_pos[0].copy(), hit_pos[1].copy()
        hit_pos[0] = c * hx - s * hy
        hit_pos[1] = s * hx + c * hy
        hit_pos[2] = hit_pos[2] - align_true[1, hit_layer]

    return Event(geometry=g, charge=q.astype(np.int8), vertex=vtx, hit_offsets=offsets,
                 hit_layer=hit_layer, hit_valid=hit_valid, hit_pos=hit_pos, hit_cov=hit_cov,
                 truth=truth, truth_after=truth_after, align_true=align_true)


def truncate(ev: Event, lengths) -> Event:
    """Keep only the first lengths[t] entries of track t (lengths <= current)."""
    lengths = np.minimum(np.asarray(lengths, np.int64), ev.lengths())
    n = ev.n_tracks
    starts = ev.hit_offsets[:-1].astype(np.int64)
    idx = np.concatenate([np.arange(s, s + l) for s, l in zip(starts, lengths)]) if n else np.zeros(0, np.int64)
    off = np.zeros(n + 1, np.int32)
    off[1:] = np.cumsum(lengths)
    return Event(geometry=ev.geometry, charge=ev.charge, vertex=ev.vertex, hit_offsets=off,
                 hit_layer=ev.hit_layer[idx], hit_valid=ev.hit_valid[idx], hit_pos=ev.hit_pos[:, idx],
                 hit_cov=ev.hit_cov[:, idx], truth=ev.truth[idx], truth_after=ev.truth_after[idx],
                 align_true=ev.align_true)


def subset(ev: Event, tracks) -> Event:
    tracks = np.asarray(tracks, np.int64)
    lens = ev.lengths()[tracks]
    starts = ev.hit_offsets[:-1].astype(np.int64)[tracks]
    idx = np.concatenate([np.arange(s, s + l) for s, l in zip(starts, lens)]) if tracks.size else np.zeros(0, np.int64)
    off = np.zeros(tracks.size + 1, np.int32)
    off[1:] = np.cumsum(lens)
    return Event(geometry=ev.geometry, charge=ev.charge[tracks], vertex=ev.vertex[tracks], hit_offsets=off,
                 hit_layer=ev.hit_layer[idx], hit_valid=ev.hit_valid[idx], hit_pos=ev.hit_pos[:, idx],
                 hit_cov=ev.hit_cov[:, idx], truth=ev.truth[idx], truth_after=ev.truth_after[idx],
                 align_true=ev.align_true)


@dataclass
class HitPools:
    """Per-layer hit pools for the combinatorial search (true hits + noise)."""
    layer_offsets: np.ndarray  # int32 [L+1]; pool hits of layer l are [off[l], off[l+1])
    pos: np.ndarray            # float64 [3, np]
    cov: np.ndarray            # float64 [6, np]
    hit_id: np.ndarray         # int32 [np] (= index into these arrays; generator order)
    track: np.ndarray          # int32 [np] producing track, -1 for noise
    module: np.ndarray = None  # int32 [np] detector module of each hit (with_modules), or None


def make_pools(wl: Workload, ev: Event, first_layer: int = 3, noise: bool = True) -> HitPools:
    """Pools for layers >= first_layer: every true hit of ``ev`` on that layer
    plus uniform noise (wl.noise_density per cm^2 of the barrel surface),
    shuffled within the layer."""
    g = wl.geometry
    ss = np.random.SeedSequence(wl.seed + 7919)
    rng = np.random.Generator(np.random.PCG64(ss))
    trk_of_hit = np.repeat(np.arange(ev.n_tracks, dtype=np.int32), ev.lengths())
    pos_l, cov_l, trk_l, off = [], [], [], [0]
    for lay in range(g.n_layers):
        if lay < first_layer:
            off.append(off[-1])
            continue
        sel = np.nonzero((ev.hit_layer == lay) & (ev.hit_valid == 1))[0]
        tp, tc, tt = ev.hit_pos[:, sel], ev.hit_cov[:, sel], trk_of_hit[sel]
        if noise and wl.noise_density > 0 and g.kind[lay] == BARREL:
            R = g.pos[lay]
            area = 2.0 * np.pi * R * (g.hi[lay] - g.lo[lay])
            m = int(round(wl.noise_density * area))
            ph = rng.uniform(-np.pi, np.pi, m)
            zz = rng.uniform(g.lo[lay], g.hi[lay], m)
            npos = np.stack([R * np.cos(ph), R * np.sin(ph), zz])
            ncov = _hit_cov_barrel(ph, wl.sigma_rphi, wl.sigma_z, wl.sigma_n)
            tp = np.concatenate([tp, npos], axis=1)
            tc = np.concatenate([tc, ncov], axis=1)
            tt = np.concatenate([tt, np.full(m, -1, np.int32)])
        perm = rng.permutation(tt.shape[0])
        pos_l.append(tp[:, perm])
        cov_l.append(tc[:, perm])
        trk_l.append(tt[perm])
        off.append(off[-1] + tt.shape[0])
    pos = np.concatenate(pos_l, axis=1) if pos_l else np.zeros((3, 0))
    cov = np.concatenate(cov_l, axis=1) if cov_l else np.zeros((6, 0))
    trk = np.concatenate(trk_l) if trk_l else np.zeros(0, np.int32)
    return HitPools(layer_offsets=np.asarray(off, np.int32), pos=pos, cov=cov,
                    hit_id=np.arange(trk.shape[0], dtype=np.int32), track=trk.astype(np.int32))


MODULE_WIDTH = 4.0     # cm of r-phi per barrel module (sets the module count of a layer)
MODULE_OVERLAP = 0.4   # cm of r-phi by which a module overlaps the next one


def with_modules(wl: Workload, ev: Event, pools: HitPools, width: float = MODULE_WIDTH,
                 overlap: float = MODULE_OVERLAP) -> HitPools:
    """The pools split into detector modules, with overlap hits.  Barrel layer
    l of radius R holds n = max(12, ceil(2 pi R / width)) modules; module k
    spans phi in [k d - pi, (k + 1) d - pi) plus `overlap` cm of r-phi beyond
    its upper edge (d = 2 pi / n), so that it overlaps the first `overlap` cm
    of module k + 1.  Modules are numbered layer by layer.  A pool hit belongs
    to the module its phi falls in; a true hit whose crossing lies in an
    overlap region is also measured by the overlapping module: a second hit,
    at the true crossing point smeared anew along r-phi and z, with the next
    free hit id, appended to the layer's hits.  The overlapping modules are
    taken to lie on the layer's surface (no radial offset), so that both hits
    are measurements of the same crossing."""
    g = wl.geometry
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(wl.seed + 104729)))
    trk_of_hit = np.repeat(np.arange(ev.n_tracks, dtype=np.int32), ev.lengths())
    off = np.asarray(pools.layer_offsets, np.int64)
    pos_l, cov_l, id_l, trk_l, mod_l, new_off = [], [], [], [], [], [0]
    next_id = int(pools.hit_id.max()) + 1 if pools.hit_id.size else 0
    base = 0
    for lay in range(g.n_layers):
        a, b = int(off[lay]), int(off[lay + 1])
        pos, cov = pools.pos[:, a:b], pools.cov[:, a:b]
        ids, trk = pools.hit_id[a:b], pools.track[a:b]
        if g.kind[lay] != BARREL or b == a:
            mods = np.full(b - a, -1, np.int64)
            pos_l.append(pos), cov_l.append(cov), id_l.append(ids), trk_l.append(trk), mod_l.append(mods)
            new_off.append(new_off[-1] + (b - a))
            continue
        R = float(g.pos[lay])
        n_mod = max(12, int(np.ceil(2 * np.pi * R / width)))
        d = 2 * np.pi / n_mod
        k = np.minimum(((np.arctan2(pos[1], pos[0]) + np.pi) / d).astype(np.int64), n_mod - 1)
        mods = base + k
        # true crossings of this layer inside an overlap region
        sel = np.nonzero((ev.hit_layer == lay) & (ev.hit_valid == 1))[0]
        tx, ty, tz = ev.truth[sel, 0], ev.truth[sel, 1], ev.truth[sel, 2]
        tphi = np.arctan2(ty, tx)
        kt = np.minimum(((tphi + np.pi) / d).astype(np.int64), n_mod - 1)
        into = (tphi + np.pi - kt * d) * R          # r-phi distance into module kt
        dup = np.nonzero(into < overlap)[0]
        g_r = rng.normal(0.0, 1.0, dup.size)
        g_z = rng.normal(0.0, 1.0, dup.size)
        ph2 = tphi[dup] + wl.sigma_rphi * g_r / R
        npos = np.stack([R * np.cos(ph2), R * np.sin(ph2), tz[dup] + wl.sigma_z * g_z])
        ncov = _hit_cov_barrel(ph2, wl.sigma_rphi, wl.sigma_z, wl.sigma_n)
        nmod = base + (kt[dup] - 1) % n_mod          # the overlapping module below
        nid = np.arange(next_id, next_id + dup.size, dtype=np.int32)
        next_id += dup.size
        pos_l.append(np.concatenate([pos, npos], axis=1))
        cov_l.append(np.concatenate([cov, ncov], axis=1))
        id_l.append(np.concatenate([ids, nid]))
        trk_l.append(np.concatenate([trk, trk_of_hit[sel[dup]]]))
        mod_l.append(np.concatenate([mods, nmod]))
        new_off.append(new_off[-1] + (b - a) + dup.size)
        base += n_mod
    cat = lambda xs, ax=0: np.concatenate(xs, axis=ax)
    return HitPools(layer_offsets=np.asarray(new_off, np.int32), pos=cat(pos_l, 1), cov=cat(cov_l, 1),
                    hit_id=cat(id_l).astype(np.int32), track=cat(trk_l).astype(np.int32),
                    module=cat(mod_l).astype(np.int32))
