"""Toy barrel of tilted planar modules (the Phase-2 geometry style of the
paper's Sec. 3.1: each module described by a position, a normal and a
phi-direction vector) and tracks through it.

Each barrel layer of radius R is tiled by modules: n_phi(R) columns in phi
and n_z rows in z (segments of `seg` cm).  Module (k, j) of a layer has its
centre at radius R, phi_k = 2 pi (k + 1/2) / n_phi, z_j the segment's centre;
its normal is the radial direction turned by `tilt_phi` about the beam axis
and, for rows away from z = 0, turned towards the beam axis' direction by
tilt_z(z_j) (the rows face the interaction region, as the tilted Phase-2
rings do); its phi-direction u = z_hat x n / |z_hat x n| lies in the plane;
v = n x u.  A module is an unbounded plane here: the track crosses the
module whose (k, j) cell its crossing of the radius-R cylinder falls in.

The helix and the plane crossing are this module's own (rotation form,
Newton on the plane equation); the filter implementations share nothing
with it.  Hits are local coordinates (m_u, m_v) on the crossed module,
smeared by sigma_u and sigma_v, then a multiple-scattering kick of x/X0 /
|cos| at the crossing.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .detector import BARREL10_RADII
from .generate import C_LIGHT, GRAZING_COS, _advance, _barrel_candidates, _highland, _wrap

MODULE_WIDTH = 4.0      # cm, target module width in r-phi (sets n_phi)
SEG = 30.0              # cm, module length in z
HALF_LENGTH = 150.0
TILT_PHI = np.deg2rad(12.0)
TILT_Z_MAX = np.deg2rad(25.0)


@dataclass(frozen=True)
class ModuleGeometry:
    modules: np.ndarray    # float64 [10, M]: cx cy cz nx ny nz ux uy uz x_over_x0
    layer_of: np.ndarray   # int16 [M]
    radii: np.ndarray      # float64 [L]
    n_phi: np.ndarray      # int64 [L]
    n_z: int
    base: np.ndarray       # int64 [L]: id of module (0, 0) of each layer
    bz: float = 3.8
    mass: float = 0.13957

    @property
    def n_layers(self) -> int:
        return int(self.radii.shape[0])

    @property
    def n_modules(self) -> int:
        return int(self.modules.shape[1])


def tilted_barrel(radii=BARREL10_RADII, tilt_phi=TILT_PHI, tilt_z_max=TILT_Z_MAX, width=MODULE_WIDTH, seg=SEG,
                  half_length=HALF_LENGTH, x_over_x0=0.02, bz=3.8) -> ModuleGeometry:
    radii = np.asarray(radii, np.float64)
    n_z = int(round(2 * half_length / seg))
    cols, lay, nphi = [], [], []
    for l, R in enumerate(radii):
        n_phi = max(12, int(np.ceil(2 * np.pi * R / width)))
        nphi.append(n_phi)
        for j in range(n_z):
            zc = -half_length + (j + 0.5) * seg
            # rows face the interaction region: tilt towards +z for z > 0
            gam = tilt_z_max * np.clip(zc / half_length, -1.0, 1.0) if abs(zc) > seg else 0.0
            for k in range(n_phi):
                ph = 2 * np.pi * (k + 0.5) / n_phi
                n1 = np.array([np.cos(ph + tilt_phi), np.sin(ph + tilt_phi), 0.0])
                u = np.array([-np.sin(ph + tilt_phi), np.cos(ph + tilt_phi), 0.0])
                n = np.cos(gam) * n1 + np.sin(gam) * np.array([0.0, 0.0, 1.0])
                c = np.array([R * np.cos(ph), R * np.sin(ph), zc])
                cols.append(np.concatenate([c, n, u, [x_over_x0]]))
                lay.append(l)
    mods = np.stack(cols, axis=1)
    base = np.concatenate([[0], np.cumsum(np.asarray(nphi) * n_z)[:-1]]).astype(np.int64)
    return ModuleGeometry(modules=mods, layer_of=np.asarray(lay, np.int16), radii=radii,
                          n_phi=np.asarray(nphi, np.int64), n_z=n_z, base=base, bz=bz)


@dataclass(frozen=True)
class PlaneWorkload:
    name: str
    geometry: ModuleGeometry
    n_tracks: int
    seed: int
    eta_max: float = 1.0
    pt_min: float = 0.5
    pt_max: float = 10.0
    sigma_u: float = 0.003
    sigma_v: float = 0.01


@dataclass
class PlaneEvent:
    geometry: ModuleGeometry
    charge: np.ndarray        # int8 [n]
    vertex: np.ndarray        # float64 [n, 6]
    hit_offsets: np.ndarray   # int32 [n+1]
    hit_module: np.ndarray    # int32 [nh]
    hit_layer: np.ndarray     # int16 [nh]
    hit_valid: np.ndarray     # uint8 [nh]
    hit_uv: np.ndarray        # float64 [2, nh] local coordinates
    hit_cov_uv: np.ndarray    # float64 [3, nh] packed (uu, vu, vv)
    hit_pos: np.ndarray       # float64 [3, nh] global position of the measured point
    truth: np.ndarray         # float64 [nh, 6] true state at the crossing, before the kick
    truth_after: np.ndarray   # float64 [nh, 6] just after the kick

    @property
    def n_tracks(self) -> int:
        return int(self.charge.shape[0])

    @property
    def n_hits(self) -> int:
        return int(self.hit_module.shape[0])

    def lengths(self) -> np.ndarray:
        return np.diff(self.hit_offsets)


def plane_workloads() -> dict[str, PlaneWorkload]:
    return {"tilted10": PlaneWorkload("tilted10", tilted_barrel(), 100_000, 1006)}


def _plane_path(xa, ya, za, pha, cot, om, s0, c, n, steps=8):
    """Newton on n.(x(s) - c) = 0 from s0 (the cylinder crossing)."""
    s = s0.copy()
    for _ in range(steps):
        x, y, z, ph = _advance(xa, ya, za, pha, cot, om, s)
        h = (x - c[0]) * n[0] + (y - c[1]) * n[1] + (z - c[2]) * n[2]
        dh = np.cos(ph) * n[0] + np.sin(ph) * n[1] + cot * n[2]
        with np.errstate(divide="ignore", invalid="ignore"):
            s = s - h / dh
    x, y, z, ph = _advance(xa, ya, za, pha, cot, om, s)
    h = (x - c[0]) * n[0] + (y - c[1]) * n[1] + (z - c[2]) * n[2]
    return s, np.abs(h) < 1e-9


def generate_planes(wl: PlaneWorkload, n_tracks: int | None = None, *, smear: bool = True,
                    scatter: bool = True, min_hits: int = 3) -> PlaneEvent:
    """Tracks from the beam spot outwards through the tilted barrel, one module
    crossing per layer (a track ends at a grazing crossing, when it turns back
    before the next layer or leaves the barrel's length)."""
    g = wl.geometry
    n = wl.n_tracks if n_tracks is None else int(n_tracks)
    ss = np.random.SeedSequence(wl.seed)
    rng_trk, rng_smear, rng_kick = [np.random.Generator(np.random.PCG64(c_)) for c_ in ss.spawn(3)]
    L = g.n_layers
    out = []
    have = 0
    while have < n:
        m = max(64, int((n - have) * 1.05) + 16)
        vx = rng_trk.normal(0.0, 0.01, m)
        vy = rng_trk.normal(0.0, 0.01, m)
        vz = rng_trk.normal(0.0, 5.0, m)
        pt = np.exp(rng_trk.uniform(np.log(wl.pt_min), np.log(wl.pt_max), m))
        eta = rng_trk.uniform(-wl.eta_max, wl.eta_max, m)
        phi = rng_trk.uniform(0.0, 2 * np.pi, m)
        q = np.where(rng_trk.uniform(0.0, 1.0, m) < 0.5, 1, -1).astype(np.int8)
        theta = 2.0 * np.arctan(np.exp(-eta))
        phi0, theta0 = phi.copy(), theta.copy()
        x, y, z = vx.copy(), vy.copy(), vz.copy()
        ptot = pt / np.sin(theta)
        recs = []           # per layer: arrays of the tracks that made a hit there
        alive = np.ones(m, bool)
        for l in range(L):
            act = np.nonzero(alive)[0]
            if act.size == 0:
                break
            tha = theta[act]
            cot = np.cos(tha) / np.sin(tha)
            pta = ptot[act] * np.sin(tha)
            om = -q[act].astype(np.float64) * C_LIGHT * g.bz / pta
            R = np.full(act.size, g.radii[l])
            s1, s2 = _barrel_candidates(x[act], y[act], phi[act], om, R)
            sc = np.fmin(s1, s2)
            ok = np.isfinite(sc)
            scv = np.where(ok, sc, 0.0)
            cx_, cy_, cz_, _ = _advance(x[act], y[act], z[act], phi[act], cot, om, scv)
            ok &= np.abs(cz_) < HALF_LENGTH
            # the module cell of the cylinder crossing
            pc = np.mod(np.arctan2(cy_, cx_), 2 * np.pi)
            k = np.minimum((pc / (2 * np.pi) * g.n_phi[l]).astype(np.int64), g.n_phi[l] - 1)
            j = np.clip(((cz_ + HALF_LENGTH) / SEG).astype(np.int64), 0, g.n_z - 1)
            mid = g.base[l] + j * g.n_phi[l] + k
            mods = g.modules[:, mid]
            c_, n_, u_ = mods[0:3], mods[3:6], mods[6:9]
            sp, conv = _plane_path(x[act], y[act], z[act], phi[act], cot, om, scv, c_, n_)
            ok &= conv & (sp > 1e-6)
            spv = np.where(ok, sp, 0.0)
            nx, ny, nz, nphi = _advance(x[act], y[act], z[act], phi[act], cot, om, spv)
            dvec = np.stack([np.sin(tha) * np.cos(nphi), np.sin(tha) * np.sin(nphi), np.cos(tha)])
            cos_a = np.abs((dvec * n_).sum(0))
            ok &= cos_a >= GRAZING_COS
            alive[act[~ok]] = False
            sel = np.nonzero(ok)[0]
            if sel.size == 0:
                continue
            v_ = np.cross(n_.T, u_.T).T
            rel = np.stack([nx, ny, nz]) - c_
            mu = (rel * u_).sum(0)
            mv = (rel * v_).sum(0)
            gu = rng_smear.normal(0.0, 1.0, act.size) if smear else np.zeros(act.size)
            gv = rng_smear.normal(0.0, 1.0, act.size) if smear else np.zeros(act.size)
            hu, hv = mu + wl.sigma_u * gu, mv + wl.sigma_v * gv
            p_ = ptot[act]
            beta = p_ / np.sqrt(p_ * p_ + g.mass ** 2)
            th0 = _highland(p_, beta, g.modules[9, mid] / np.maximum(cos_a, GRAZING_COS))
            if scatter:
                d_th = rng_kick.normal(0.0, 1.0, act.size) * th0
                d_ps = rng_kick.normal(0.0, 1.0, act.size) * th0
            else:
                d_th = np.zeros(act.size)
                d_ps = np.zeros(act.size)
            new_th = np.clip(tha + d_th, 1e-3, np.pi - 1e-3)
            new_phi = nphi + d_ps / np.sin(tha)
            truth = np.stack([nx, ny, nz, 1.0 / pta, _wrap(nphi), tha], axis=1)[sel]
            after = np.stack([nx, ny, nz, 1.0 / (p_ * np.sin(new_th)), _wrap(new_phi), new_th], axis=1)[sel]
            gpos = (c_ + hu * u_ + hv * v_)[:, sel]
            recs.append(dict(t=act[sel], mid=mid[sel], layer=np.full(sel.size, l), hu=hu[sel], hv=hv[sel],
                             gpos=gpos, truth=truth, after=after))
            t_ok = act[sel]
            x[t_ok], y[t_ok], z[t_ok] = nx[sel], ny[sel], nz[sel]
            phi[t_ok] = new_phi[sel]
            theta[t_ok] = new_th[sel]
        # every track's records in layer order; tracks with enough hits are
        # taken in generation order until n are had
        if recs:
            cat = {key: np.concatenate([r[key] for r in recs], axis=-1 if key == "gpos" else 0) for key in recs[0]}
            order = np.argsort(cat["t"], kind="stable")
            cnt = np.bincount(cat["t"], minlength=m)
        else:
            cat, order, cnt = None, np.zeros(0, np.int64), np.zeros(m, np.int64)
        take = np.nonzero(cnt >= min_hits)[0][: n - have]
        if take.size:
            first = np.concatenate([[0], np.cumsum(cnt)[:-1]])
            idx = np.concatenate([order[first[t]:first[t] + cnt[t]] for t in take])
            out.append(dict(q=q[take], vertex=np.stack([vx, vy, vz, 1.0 / pt, _wrap(phi0), theta0], axis=1)[take],
                            cnt=cnt[take], mid=cat["mid"][idx], layer=cat["layer"][idx], hu=cat["hu"][idx],
                            hv=cat["hv"][idx], gpos=cat["gpos"][:, idx], truth=cat["truth"][idx],
                            after=cat["after"][idx]))
            have += take.size
    cat = lambda key, axis=0: np.concatenate([o[key] for o in out], axis=axis)
    cnt = cat("cnt")
    off = np.zeros(n + 1, np.int32)
    off[1:] = np.cumsum(cnt)
    nh = int(off[-1])
    cov1 = np.array([wl.sigma_u ** 2, 0.0, wl.sigma_v ** 2])
    return PlaneEvent(geometry=g, charge=cat("q").astype(np.int8), vertex=cat("vertex").astype(np.float64),
                      hit_offsets=off, hit_module=cat("mid").astype(np.int32),
                      hit_layer=cat("layer").astype(np.int16), hit_valid=np.ones(nh, np.uint8),
                      hit_uv=np.stack([cat("hu"), cat("hv")]).astype(np.float64),
                      hit_cov_uv=np.repeat(cov1[:, None], nh, axis=1),
                      hit_pos=np.ascontiguousarray(cat("gpos", 1), np.float64),
                      truth=cat("truth").astype(np.float64), truth_after=cat("after").astype(np.float64))
