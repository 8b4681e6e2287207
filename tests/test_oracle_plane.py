"""Pins for the oracle of tilted planar modules (oracle/kf_plane.py): the
crossing against the generator's own plane crossings (its helix is separate
code, and the oracle's helix is pinned against a Runge-Kutta integration of
the Lorentz force elsewhere), the surface-to-surface Jacobian against central
differences, the plane normal as a null vector, the 2-D local update against
the 3-D update with a thickness term along the normal (pinned elsewhere
against batch conditioning), the incidence of the scattering, and the fit's
statistics and exactness on the tilted toy."""
import math

import numpy as np
import pytest
import torch

from oracle import kf_oracle as O
from oracle import kf_plane as P
from toygen import generate_planes, plane_workloads, subset

DT = torch.float64


def _event(n=400, **kw):
    wl = plane_workloads()["tilted10"]
    return wl, generate_planes(wl, n, **kw)


def _pairs(ev):
    """(state at entry e, module of entry e + 1) for every entry with a successor."""
    off = ev.hit_offsets
    e = np.concatenate([np.arange(off[t], off[t + 1] - 1) for t in range(ev.n_tracks)])
    return e, e + 1


def test_crossing_lands_on_the_generators_crossing():
    """Noise-free tracks without scattering: from the true state at one
    module, the oracle's crossing of the next module's plane is the
    generator's crossing (truth), to 1e-9 cm, with the same direction."""
    wl, ev = _event(300, smear=False, scatter=False)
    g = wl.geometry
    c, n, u, v, x0 = P.frames(g.modules)
    e0, e1 = _pairs(ev)
    p = torch.tensor(ev.truth[e0])
    q = torch.tensor(ev.charge[np.searchsorted(ev.hit_offsets, e0, side="right") - 1], dtype=DT)
    m = torch.as_tensor(ev.hit_module[e1].astype(np.int64))
    s, ok = P.crossing_plane(p, q, c[m], n[m], g.bz)
    assert bool(ok.all())
    x = O.helix_at(p, q, s, g.bz)
    tr = torch.tensor(ev.truth[e1])
    assert float((x[:, :3] - tr[:, :3]).abs().max()) < 1e-9
    d = x[:, 4] - tr[:, 4]
    assert float(O.wrap_phi(d).abs().max()) < 1e-12
    # on the plane, and the local coordinates are the noise-free measurements
    h = ((x[:, :3] - c[m]) * n[m]).sum(1)
    assert float(h.abs().max()) < 1e-9
    mu = ((x[:, :3] - c[m]) * u[m]).sum(1)
    assert float((mu - torch.tensor(ev.hit_uv[0, e1])).abs().max()) < 1e-9


def _first_root_by_scan(p, q, c, n, bz, lo=-O.S_BACK, step=0.05):
    """The smallest root s > lo of n.(x(s) - c) within one turn, by brute
    force: the first sign change on a grid of `step` cm, then bisection.
    (nan, False) when h keeps its sign over the turn."""
    w = float(O.omega(torch.tensor(q), torch.tensor(p[3]), bz))
    s_max = lo + 2 * math.pi / abs(w)
    grid = torch.arange(lo, s_max + step, step, dtype=DT)
    grid = grid[grid <= s_max]
    P_ = torch.tensor(p).expand(grid.numel(), 6)
    Q_ = torch.full((grid.numel(),), float(q), dtype=DT)
    h = ((O.helix_at(P_, Q_, grid, bz)[:, :3] - c) * n).sum(1)
    ch = torch.nonzero(torch.sign(h[1:]) != torch.sign(h[:-1]))[:, 0]
    if ch.numel() == 0:
        return math.nan, False
    a, b = float(grid[ch[0]]), float(grid[ch[0] + 1])
    ha = float(h[ch[0]])
    one = lambda s_: float(((O.helix_at(torch.tensor(p)[None], torch.tensor([float(q)], dtype=DT),
                                        torch.tensor([s_], dtype=DT), bz)[0, :3] - c) * n).sum())
    for _ in range(80):
        m = 0.5 * (a + b)
        hm = one(m)
        if (hm < 0) == (ha < 0):
            a, ha = m, hm
        else:
            b = m
    return 0.5 * (a + b), True


def test_crossing_is_the_first_root_found_by_brute_force():
    """The crossing is the smallest root s > -1 cm within one turn, checked by
    a scan and bisection: on the true states (the next module), with the
    curvature raised so that low-pT tracks turn back before the module, and
    with a module of the next layer a quarter turn away in phi (crossed far
    from it, or not within the turn)."""
    wl, ev = _event(300)
    g = wl.geometry
    c, n, u, v, x0 = P.frames(g.modules)
    e0, e1 = _pairs(ev)
    rng = np.random.default_rng(11)
    pick = rng.choice(e0.size, 40, replace=False)
    cases = []
    for i in pick:
        p = ev.truth_after[e0[i]].copy()
        q = float(ev.charge[np.searchsorted(ev.hit_offsets, e0[i], side="right") - 1])
        m = int(ev.hit_module[e1[i]])
        lay = int(g.layer_of[m])
        cases.append((p, q, m))
        p2 = p.copy()
        p2[3] *= 1.0 + 2.0 * rng.uniform()
        cases.append((p2, q, m))
        k = (m - g.base[lay]) % g.n_phi[lay]
        j = (m - g.base[lay]) // g.n_phi[lay]
        far = int(g.base[lay] + j * g.n_phi[lay] + (k + g.n_phi[lay] // 4) % g.n_phi[lay])
        cases.append((p, q, far))
    P_ = torch.tensor(np.array([x[0] for x in cases]))
    Q_ = torch.tensor([x[1] for x in cases], dtype=DT)
    M_ = torch.tensor([x[2] for x in cases])
    s, ok = P.crossing_plane(P_, Q_, c[M_], n[M_], g.bz)
    found = 0
    for i, (p, q, m) in enumerate(cases):
        sb, okb = _first_root_by_scan(p, q, c[m], n[m], g.bz)
        assert bool(ok[i]) == okb, (i, float(s[i]), sb)
        if okb:
            found += 1
            assert abs(float(s[i]) - sb) < 1e-8 * max(1.0, abs(sb)), (i, float(s[i]), sb)
    assert 40 <= found < len(cases)


def test_plane_jacobian_equals_central_differences():
    wl, ev = _event(60)
    g = wl.geometry
    c, n, u, v, x0 = P.frames(g.modules)
    e0, e1 = _pairs(ev)
    sel = np.arange(0, e0.size, 7)[:60]
    e0, e1 = e0[sel], e1[sel]
    p = torch.tensor(ev.truth_after[e0])
    q = torch.tensor(ev.charge[np.searchsorted(ev.hit_offsets, e0, side="right") - 1], dtype=DT)
    m = torch.as_tensor(ev.hit_module[e1].astype(np.int64))
    s, ok = P.crossing_plane(p, q, c[m], n[m], g.bz)
    assert bool(ok.all())
    F = P.jacobian_plane(p, q, s, n[m], g.bz)
    # steps large enough that the crossing's own rounding (~1e-13 cm) stays
    # far below the differences, small enough for the O(h^2) term
    h = torch.tensor([1e-4, 1e-4, 1e-4, 1e-5, 1e-5, 1e-5], dtype=DT)

    def f(pp):
        ss, _ = P.crossing_plane(pp, q, c[m], n[m], g.bz)
        out = O.helix_at(pp, q, ss, g.bz)
        return out

    worst = 0.0
    for k in range(6):
        dp = torch.zeros(6, dtype=DT)
        dp[k] = h[k]
        fp, fm = f(p + dp), f(p - dp)
        col = (fp - fm) / (2 * h[k])
        col[:, 4] = O.wrap_phi(fp[:, 4] - fm[:, 4]) / (2 * h[k])
        err = (F[:, :, k] - col).abs() / (col.abs() + 1e-3)
        worst = max(worst, float(err.max()))
    assert worst < 1e-5, worst


def test_plane_normal_is_a_null_vector_after_propagation():
    wl, ev = _event(100)
    g = wl.geometry
    c, n, u, v, x0 = P.frames(g.modules)
    e0, e1 = _pairs(ev)
    p = torch.tensor(ev.truth_after[e0])
    q = torch.tensor(ev.charge[np.searchsorted(ev.hit_offsets, e0, side="right") - 1], dtype=DT)
    A = torch.randn(p.shape[0], 6, 6, dtype=DT, generator=torch.Generator().manual_seed(2)) * 0.01
    C = A @ A.transpose(1, 2) + 1e-6 * torch.eye(6, dtype=DT)
    m = torch.as_tensor(ev.hit_module[e1].astype(np.int64))
    p2, C2, s, st = P.propagate_plane(p, C, q, c[m], n[m], x0[m], g)
    assert int((st & O.NO_CROSSING).sum()) == 0
    nv = torch.cat([n[m], torch.zeros(p.shape[0], 3, dtype=DT)], 1)
    nn = torch.einsum("ni,nij,nj->n", nv, C2, nv)
    tr = C2[:, 0, 0] + C2[:, 1, 1] + C2[:, 2, 2]
    assert float((nn.abs() / tr).max()) < 1e-9
    # and the rest of the covariance is positive definite on the plane
    B = torch.zeros(p.shape[0], 6, 5, dtype=DT)
    B[:, :3, 0], B[:, :3, 1] = u[m], v[m]
    B[:, 3, 2] = B[:, 4, 3] = B[:, 5, 4] = 1.0
    _, info = torch.linalg.cholesky_ex(B.transpose(1, 2) @ C2 @ B)
    assert int((info != 0).sum()) == 0


def test_local_update_equals_the_3d_update_with_a_thickness_term():
    """The 2-D update on (u, v) and the 3-D update of kf_oracle.update with the
    hit at c + m_u u + m_v v and V3 = [u v n] diag(V_uv, sigma_n^2) [u v n]^T:
    the prior has the normal as a null vector, so the normal coordinate of the
    residual is zero and the two coincide for any sigma_n."""
    wl, ev = _event(100)
    g = wl.geometry
    c, n, u, v, x0 = P.frames(g.modules)
    e0, e1 = _pairs(ev)
    p = torch.tensor(ev.truth_after[e0])
    q = torch.tensor(ev.charge[np.searchsorted(ev.hit_offsets, e0, side="right") - 1], dtype=DT)
    A = torch.randn(p.shape[0], 6, 6, dtype=DT, generator=torch.Generator().manual_seed(3)) * 0.01
    C = A @ A.transpose(1, 2) + 1e-6 * torch.eye(6, dtype=DT)
    m = torch.as_tensor(ev.hit_module[e1].astype(np.int64))
    p2, C2, _, _ = P.propagate_plane(p, C, q, c[m], n[m], x0[m], g)
    muv = torch.tensor(ev.hit_uv[:, e1].T)
    Vuv = P.unpack2(ev.hit_cov_uv[:, e1])
    a = P.update_local(p2, C2, q, muv, Vuv, c[m], u[m], v[m])
    for sn in (1e-3, 0.0087, 0.1):
        Bm = torch.stack([u[m], v[m], n[m]], dim=2)           # columns u, v, n
        D = torch.zeros(p.shape[0], 3, 3, dtype=DT)
        D[:, :2, :2] = Vuv
        D[:, 2, 2] = sn ** 2
        V3 = Bm @ D @ Bm.transpose(1, 2)
        m3 = P.local_to_global(muv, c[m], u[m], v[m])
        b = O.update(p2, C2, q, m3, V3)
        d = a[0] - b[0]
        d[:, 4] = O.wrap_phi(d[:, 4])
        assert float(d.abs().max()) < 1e-9
        assert float(((a[3] - b[3]).abs() / torch.clamp(b[3], min=1.0)).max()) < 1e-9
        sd = torch.sqrt(torch.diagonal(b[1], dim1=1, dim2=2).abs()) + 1e-300
        assert float(((a[1] - b[1]) / (sd[:, :, None] * sd[:, None, :])).abs().max()) < 1e-7


def test_tilted_incidence_thickens_the_scatterer():
    """A module facing the track (normal along the direction) scatters as
    x/X0; tilted by a, as x/X0/|cos a| -- the same angle as a face-on module
    of that thickness."""
    wl, ev = _event(50)
    g = wl.geometry
    p = torch.tensor(ev.truth[:20])
    ph, th = p[:, 4], p[:, 5]
    d = torch.stack([torch.sin(th) * torch.cos(ph), torch.sin(th) * torch.sin(ph), torch.cos(th)], 1)
    face, _ = O.highland_theta0_at(p, P.cos_incidence_plane(p, d), torch.full((20,), 0.02, dtype=DT), g.mass)
    # tilt the normal by 40 degrees about an axis orthogonal to d
    ax = torch.linalg.cross(d, torch.tensor([0.0, 0.0, 1.0], dtype=DT).expand(20, 3))
    ax = ax / ax.norm(dim=1, keepdim=True)
    a = math.radians(40)
    nt = d * math.cos(a) + torch.linalg.cross(ax, d) * math.sin(a)
    tilt, _ = O.highland_theta0_at(p, P.cos_incidence_plane(p, nt), torch.full((20,), 0.02, dtype=DT), g.mass)
    thick, _ = O.highland_theta0_at(p, P.cos_incidence_plane(p, d), torch.full((20,), 0.02 / math.cos(a), dtype=DT),
                                    g.mass)
    assert torch.allclose(tilt, thick, rtol=1e-12) and bool((tilt > face).all())


def _fit(ev, wl, state_round=None):
    g = wl.geometry
    sp, sC, sq, ok = P.make_seeds_planes(ev.hit_offsets, ev.hit_module, ev.hit_valid, ev.hit_uv, g.modules, g.bz)
    return P.fit_plane_tracks(sp, sC, sq, ev.hit_offsets, ev.hit_module, ev.hit_valid, ev.hit_uv, ev.hit_cov_uv,
                              g.modules, g, state_round=state_round)


def test_noise_free_fit_returns_the_truth():
    wl, ev = _event(200, smear=False, scatter=False)
    out = _fit(ev, wl)
    last = ev.hit_offsets[1:] - 1
    assert int((out["status"] & (O.NO_CROSSING | O.NONFINITE)).sum()) == 0
    d = out["p"] - torch.tensor(ev.truth[last])
    d[:, 4] = O.wrap_phi(d[:, 4])
    assert float(d[:, :3].abs().max()) < 1e-7
    assert float((d[:, 3].abs() / out["p"][:, 3]).max()) < 1e-7
    assert float(d[:, 4:].abs().max()) < 1e-9
    assert float(out["chi2"].max()) < 1e-10


def test_fit_statistics_on_the_tilted_barrel():
    """Smeared hits and scattering: chi2/ndf ~ 1 and the pulls of the local
    coordinates, 1/pT, phi and theta at the last module against the truth
    just after its kick are N(0, 1)."""
    wl, ev = _event(3000)
    out = _fit(ev, wl)
    ok = (out["status"].numpy() & (O.NO_CROSSING | O.NONFINITE)) == 0
    ratio = out["chi2"].numpy()[ok].sum() / out["ndf"].numpy()[ok].sum()
    ndf = out["ndf"].numpy()[ok].sum()
    assert abs(ratio - 1.0) < 4.0 * math.sqrt(2.0 / ndf), ratio
    g = wl.geometry
    c, n, u, v, _ = P.frames(g.modules)
    last = ev.hit_offsets[1:] - 1
    m = torch.as_tensor(ev.hit_module[last].astype(np.int64))
    tr = torch.tensor(ev.truth_after[last])
    d = out["p"] - tr
    d[:, 4] = O.wrap_phi(d[:, 4])
    C = out["C"]
    pulls = {}
    for name, vec in (("u", u[m]), ("v", v[m])):
        dv = (d[:, :3] * vec).sum(1)
        sv = torch.sqrt(torch.einsum("ni,nij,nj->n", vec, C[:, :3, :3], vec))
        pulls[name] = (dv / sv).numpy()
    sd = torch.sqrt(torch.diagonal(C, dim1=1, dim2=2))
    for k, name in ((3, "ipt"), (4, "phi"), (5, "theta")):
        pulls[name] = (d[:, k] / sd[:, k]).numpy()
    for name, x in pulls.items():
        x = x[ok]
        assert abs(x.mean()) < 5.0 / math.sqrt(x.size), (name, x.mean())
        assert abs(x.std() - 1.0) < 0.06, (name, x.std())
