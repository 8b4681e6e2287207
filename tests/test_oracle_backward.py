"""Pins for the oracle's backward fit (Sec. 2.2, step 4): the direction
reversal against the helix itself, the reversal of the covariance against the
Jacobian of the state map, exact recovery of the true state at the first hit
on noise-free tracks, agreement with the forward least-squares estimate when
there is no material, and the statistical signature of a correctly weighted
filter (pulls against the generator's truth at the first hit, chi2/ndf)."""
import dataclasses
import math

import numpy as np
import torch

from oracle import kf_oracle as O
from toygen import generate, workloads

DT = torch.float64


def _random_states(n, seed=5):
    g = torch.Generator().manual_seed(seed)
    u = lambda lo, hi: lo + (hi - lo) * torch.rand(n, generator=g, dtype=DT)
    p = torch.stack([u(-50, 50), u(-50, 50), u(-100, 100), u(0.1, 2.0), u(-math.pi, math.pi), u(0.2, 2.9)], 1)
    q = torch.where(torch.rand(n, generator=g) < 0.5, -1.0, 1.0).to(DT)
    A = torch.randn(n, 6, 6, generator=g, dtype=DT)
    C = A @ A.transpose(1, 2) + 0.1 * torch.eye(6, dtype=DT)
    return p, C, q


def test_reversal_is_an_involution():
    p, C, q = _random_states(200)
    p2, C2, q2 = O.reverse_direction(*O.reverse_direction(p, C, q))
    d = p2 - p
    d[:, 4] = O.wrap_phi(d[:, 4])
    assert d.abs().max() < 1e-13
    assert torch.equal(C2, C) and torch.equal(q2, q)


def test_reversed_state_runs_the_same_helix_backwards():
    """helix_at is pinned against an RK4 integration of the Lorentz force
    elsewhere; here the reversed state's helix over +s must be the original
    helix over -s, point by point, and its direction the reversed one."""
    p, C, q = _random_states(300)
    pr, _, qr = O.reverse_direction(p, C, q)
    for s in (0.5, 7.0, 40.0):
        fwd = O.helix_at(pr, qr, torch.full((300,), s, dtype=DT), 3.8)
        back = O.helix_at(p, q, torch.full((300,), -s, dtype=DT), 3.8)
        assert (fwd[:, :3] - back[:, :3]).abs().max() < 1e-9 * max(1.0, s)
        back_rev, _, _ = O.reverse_direction(back, C, q)
        d = fwd[:, 3:] - back_rev[:, 3:]
        d[:, 1] = O.wrap_phi(d[:, 1])
        assert d.abs().max() < 1e-12


def test_reversed_covariance_is_the_jacobian_transform():
    p, C, q = _random_states(50)
    _, C2, _ = O.reverse_direction(p, C, q)
    for i in range(50):
        J = torch.autograd.functional.jacobian(lambda x: O.reverse_direction(x[None], C[i:i + 1], q[i:i + 1])[0][0],
                                               p[i])
        assert torch.allclose(C2[i], J @ C[i] @ J.T, rtol=0, atol=1e-12)


def _backward_from(ev, fwd, cov_scale=O.BACKWARD_COV_SCALE, geom=None):
    return O.backward_fit(fwd["p"], fwd["C"], fwd["q"], fwd["status"], ev.hit_offsets, ev.hit_layer, ev.hit_valid,
                          torch.tensor(ev.hit_pos), ev.hit_cov, ev.geometry if geom is None else geom,
                          cov_scale=cov_scale)


def _first_valid(ev):
    off = ev.hit_offsets
    return np.array([off[t] + int(np.argmax(ev.hit_valid[off[t]:off[t + 1]])) for t in range(ev.n_tracks)])


def test_noise_free_tracks_return_the_truth_at_the_first_hit():
    """Hits exactly on the generated helices, no scattering: started from the
    true state at the last entry, every residual is zero, so the backward
    pass must carry the truth unchanged to the first valid entry (barrels,
    disks, holes)."""
    for name in ("barrel10", "mixed26"):
        wl = workloads()[name]
        ev = generate(wl, 300, smear=False, scatter=False)
        last = ev.hit_offsets[1:] - 1
        C = torch.diag(torch.tensor([1e-4, 1e-4, 1e-4, 1e-4, 1e-6, 1e-6], dtype=DT)).expand(ev.n_tracks, 6, 6)
        fwd = dict(p=torch.tensor(ev.truth[last]), C=C.clone(), q=torch.tensor(ev.charge, dtype=DT),
                   status=torch.zeros(ev.n_tracks, dtype=torch.int64))
        out = _backward_from(ev, fwd)
        assert (out["status"].numpy() & (O.NO_CROSSING | O.NONFINITE | O.NOT_REFITTED)).sum() == 0
        tr = torch.tensor(ev.truth[_first_valid(ev)])
        d = out["p"] - tr
        d[:, 4] = O.wrap_phi(d[:, 4])
        assert d[:, :3].abs().max() < 1e-8, name
        assert (d[:, 3].abs() / tr[:, 3]).max() < 1e-10, name
        assert d[:, 4:].abs().max() < 1e-10, name
        assert torch.equal(out["q"], fwd["q"])
        nvalid = np.add.reduceat(ev.hit_valid.astype(np.int64), ev.hit_offsets[:-1])
        assert np.array_equal(out["ndf"].numpy(), 2 * nvalid - 5)
        assert out["chi2"].abs().max() < 1e-12


def test_backward_estimate_equals_the_forward_one_without_material():
    """Smeared hits, no scattering, (almost) no material, diffuse priors: the
    forward estimate at the last entry and the backward estimate at the first
    entry carried forward to the last one use the same hits, so they are the
    same least-squares estimate up to the linearisation of each pass.  A
    pass linearises along its own running estimate, and the first forward
    pass starts from a three-hit seed (its estimate moves by up to ~0.4 sigma
    when restarted elsewhere), so the comparison is made one round later:
    forward, backward, forward again from the backward result, backward
    again.  Tracks with a near-tangent crossing (the filter visibly
    non-linear) are left out, as in the forward pins."""
    wl = workloads()["barrel10"]
    g = dataclasses.replace(wl.geometry, x_over_x0=np.full(wl.geometry.n_layers, 1e-10))
    wl2 = dataclasses.replace(wl, geometry=g)
    ev = generate(wl2, 200, scatter=False, holes=False)
    hp = torch.tensor(ev.hit_pos)
    sp, sC, sq, _ = O.make_seeds(ev.hit_offsets, ev.hit_valid, ev.hit_pos, g.bz)
    f1 = O.fit_tracks(sp, sC * 1e4, sq, ev.hit_offsets, ev.hit_layer, ev.hit_valid, hp, ev.hit_cov, g)
    b1 = _backward_from(ev, f1, cov_scale=1e8)
    fwd = O.fit_tracks(b1["p"], b1["C"] * 1e8, b1["q"], ev.hit_offsets, ev.hit_layer, ev.hit_valid, hp, ev.hit_cov, g)
    bwd = _backward_from(ev, fwd, cov_scale=1e8)
    for o in (f1, b1, fwd, bwd):
        assert (o["status"].numpy() & (O.NO_CROSSING | O.NONFINITE | O.NOT_REFITTED)).sum() == 0
    # tracks crossing every layer, away from tangent crossings: carry the
    # backward estimate from the first layer to the last (no material, no hits)
    L = g.n_layers
    t = ev.truth
    cb = np.abs(np.cos(t[:, 4] - np.arctan2(t[:, 1], t[:, 0])))
    sel = np.nonzero((ev.lengths() == L) & (np.minimum.reduceat(cb, ev.hit_offsets[:-1]) > 0.3))[0]
    assert sel.size > 100
    fwd = {k: v[sel] for k, v in fwd.items()}
    bwd = {k: v[sel] for k, v in bwd.items()}
    p, C, q = bwd["p"], bwd["C"], bwd["q"]
    m = sel.size
    for l in range(1, L):
        kind = torch.full((m,), int(g.kind[l]), dtype=torch.int64)
        p, C, _, st = O.propagate(p, C, q, kind, torch.full((m,), g.pos[l], dtype=DT),
                                  torch.full((m,), 1e-10, dtype=DT), g, apply_material=False)
        assert (st & O.NO_CROSSING).sum() == 0
    sig = torch.sqrt(torch.diagonal(fwd["C"], dim1=1, dim2=2))
    d = p - fwd["p"]
    d[:, 4] = O.wrap_phi(d[:, 4])
    # the position lies on the last surface: its tangent and z offsets
    ph = torch.atan2(fwd["p"][:, 1], fwd["p"][:, 0])
    tv = torch.stack([-torch.sin(ph), torch.cos(ph)], 1)
    tang = (d[:, :2] * tv).sum(1) / torch.sqrt(torch.einsum("ni,nij,nj->n", tv, fwd["C"][:, :2, :2], tv))
    assert tang.abs().max() < 1e-2
    assert (d[:, 2:].abs() / sig[:, 2:]).max() < 0.1
    sd = torch.sqrt(torch.diagonal(C, dim1=1, dim2=2))
    rel = (C - fwd["C"]).abs() / (sd[:, :, None] * sd[:, None, :])
    assert rel[:, 2:, 2:].max() < 1e-2
    # the two passes see the same hits: equal chi2 up to the linearisation
    assert np.abs(bwd["chi2"].numpy() - fwd["chi2"].numpy()).max() < 0.3


def test_backward_statistics_at_the_first_hit():
    """Smeared hits and scattering (barrel10): the backward estimate at the
    first hit against the generator's state there, before that layer's kick
    (the backward pass crosses the kick the other way round), gives pulls
    N(0, 1); sum chi2 / sum ndf ~ 1."""
    wl = workloads()["barrel10"]
    n = 2000
    ev = generate(wl, n, holes=False)
    fwd = O.fit_event(ev)
    out = _backward_from(ev, fwd)
    first = ev.hit_offsets[:-1]
    ok = (out["status"].numpy() & (O.NO_CROSSING | O.NONFINITE | O.NOT_REFITTED)) == 0
    # away from near-tangent crossings (as the forward statistical pins)
    t = ev.truth
    cb = np.abs(np.cos(t[:, 4] - np.arctan2(t[:, 1], t[:, 0])))
    sel = ok & (np.minimum.reduceat(cb, ev.hit_offsets[:-1]) > 0.3)
    assert sel.sum() > 0.6 * n
    ratio = out["chi2"].numpy()[sel].sum() / out["ndf"].numpy()[sel].sum()
    assert abs(ratio - 1.0) < 4.0 * math.sqrt(2.0 / out["ndf"].numpy()[sel].sum()), ratio
    tr = torch.tensor(ev.truth[first])
    p, C = out["p"], out["C"]
    d = p - tr
    d[:, 4] = O.wrap_phi(d[:, 4])
    sig = torch.sqrt(torch.diagonal(C, dim1=1, dim2=2))
    ph = torch.atan2(tr[:, 1], tr[:, 0])
    tv = torch.stack([-torch.sin(ph), torch.cos(ph)], 1)
    pulls = {"t": (d[:, :2] * tv).sum(1) / torch.sqrt(torch.einsum("ni,nij,nj->n", tv, C[:, :2, :2], tv)),
             "z": d[:, 2] / sig[:, 2], "ipt": d[:, 3] / sig[:, 3], "phi": d[:, 4] / sig[:, 4],
             "theta": d[:, 5] / sig[:, 5]}
    for k, v in pulls.items():
        vv = v.numpy()[sel]
        mu, sd = vv.mean(), vv.std()
        assert abs(mu) < 5.0 / math.sqrt(vv.size), (k, mu)
        assert abs(sd - 1.0) < 0.06, (k, sd)


def test_stopped_or_empty_tracks_keep_their_input():
    wl = workloads()["barrel10"]
    ev = generate(wl, 40)
    fwd = O.fit_event(ev)
    st = fwd["status"].clone()
    st[[3, 17]] |= O.NO_CROSSING
    st[[5]] |= O.NONFINITE
    fwd2 = dict(fwd, status=st)
    out = _backward_from(ev, fwd2)
    for t in (3, 5, 17):
        assert out["status"][t] == O.NOT_REFITTED
        assert torch.equal(out["p"][t], fwd["p"][t]) and torch.equal(out["C"][t], fwd["C"][t])
    others = [t for t in range(40) if t not in (3, 5, 17)]
    assert ((out["status"][others] & O.NOT_REFITTED) == 0).all()


def test_impose_surface_keeps_a_surface_covariance_and_removes_the_normal():
    """A covariance propagated to a layer by the exact surface-to-surface
    Jacobian already has the normal as a null vector: the projection leaves it
    unchanged.  Applied to any covariance, it makes the normal a null vector
    and is idempotent."""
    wl = workloads()["barrel10"]
    g = wl.geometry
    ev = generate(wl, 200, holes=False)
    sp, sC, sq, _ = O.make_seeds(ev.hit_offsets, ev.hit_valid, ev.hit_pos, g.bz)
    lay = ev.hit_layer[ev.hit_offsets[:-1] + 1]
    kind = torch.tensor(g.kind[lay], dtype=torch.int64)
    pos = torch.tensor(g.pos[lay], dtype=DT)
    p2, C2, _, st = O.propagate(sp, sC, sq, kind, pos, torch.tensor(g.x_over_x0[lay], dtype=DT), g)
    ok = (st & O.NO_CROSSING) == 0
    P = O.impose_surface(p2, C2, kind, pos)
    scale = torch.sqrt(torch.diagonal(C2, dim1=1, dim2=2))
    rel = (P - C2).abs() / (scale[:, :, None] * scale[:, None, :])
    assert rel[ok].max() < 1e-10
    p, C, _ = _random_states(100)
    kind = torch.zeros(100, dtype=torch.int64)
    R = torch.sqrt(p[:, 0] ** 2 + p[:, 1] ** 2)
    P1 = O.impose_surface(p, C, kind, R)
    nv = torch.stack([p[:, 0] / R, p[:, 1] / R] + [torch.zeros(100, dtype=DT)] * 4, 1)
    assert (P1 @ nv[:, :, None]).abs().max() < 1e-12 * C.abs().max()
    assert torch.allclose(O.impose_surface(p, P1, kind, R), P1, rtol=0, atol=1e-12)
    Pd = O.impose_surface(p, C, torch.ones(100, dtype=torch.int64), R)
    assert Pd[:, 2, :].abs().max() == 0 and Pd[:, :, 2].abs().max() == 0


# ---- the smoother -------------------------------------------------------------------

def _smoothed(ev, fwd_scale=1.0, geom=None, rounds=1):
    """Forward fit (recording every entry), then the smoothing backward pass;
    with rounds = 2 the forward fit is repeated from the backward result
    first (see test_backward_estimate_equals_the_forward_one_without_material)."""
    g = ev.geometry if geom is None else geom
    hp = torch.tensor(ev.hit_pos)
    sp, sC, sq, _ = O.make_seeds(ev.hit_offsets, ev.hit_valid, ev.hit_pos, g.bz)
    fwd = O.fit_tracks(sp, sC * fwd_scale, sq, ev.hit_offsets, ev.hit_layer, ev.hit_valid, hp, ev.hit_cov, g,
                       record=True)
    for _ in range(rounds - 1):
        b = O.backward_fit(fwd["p"], fwd["C"], fwd["q"], fwd["status"], ev.hit_offsets, ev.hit_layer, ev.hit_valid,
                           hp, ev.hit_cov, g, cov_scale=1e8)
        fwd = O.fit_tracks(b["p"], b["C"] * 1e8, b["q"], ev.hit_offsets, ev.hit_layer, ev.hit_valid, hp, ev.hit_cov,
                           g, record=True)
    out = O.backward_fit(fwd["p"], fwd["C"], fwd["q"], fwd["status"], ev.hit_offsets, ev.hit_layer, ev.hit_valid,
                         hp, ev.hit_cov, g, smooth_from=fwd)
    return fwd, out


def test_smoothing_leaves_the_backward_result_unchanged_and_ends_on_the_filtered_state():
    wl = workloads()["mixed26"]
    ev = generate(wl, 300)
    fwd, out = _smoothed(ev)
    plain = _backward_from(ev, fwd)
    for k in ("p", "C", "q", "chi2", "ndf", "status"):
        assert torch.equal(out[k], plain[k]), k
    last = ev.hit_offsets[1:] - 1
    ok = (out["status"].numpy() & O.NOT_REFITTED) == 0
    assert torch.equal(out["ps"][last[ok]], fwd["pe"][last[ok]])
    assert torch.equal(out["Cs"][last[ok]], fwd["Ce"][last[ok]])
    # every entry from the first valid one to the last is smoothed
    first = _first_valid(ev)
    for t in np.nonzero(ok)[0][:50]:
        e = np.arange(first[t], last[t] + 1)
        assert torch.isfinite(out["ps"][e]).all()
        assert torch.isnan(out["ps"][ev.hit_offsets[t]:first[t]]).all()


def test_smoothed_covariance_is_below_both_inputs():
    """On the surface (5 coordinates), C_f - C_s and C_b - C_s are positive
    semi-definite: combining adds information."""
    wl = workloads()["barrel10"]
    ev = generate(wl, 300, holes=False)
    fwd, out = _smoothed(ev)
    ok = (out["status"].numpy() & O.NOT_REFITTED) == 0
    e = np.concatenate([np.arange(a, b - 1) for a, b, k in zip(ev.hit_offsets[:-1], ev.hit_offsets[1:], ok) if k])
    kind = torch.tensor(ev.geometry.kind[ev.hit_layer[e]], dtype=torch.int64)
    pos = torch.tensor(ev.geometry.pos[ev.hit_layer[e]], dtype=DT)
    B = O.surface_frame(out["ps"][e], kind, pos)
    Cs5 = B.transpose(1, 2) @ out["Cs"][e] @ B
    Cf5 = B.transpose(1, 2) @ fwd["Ce"][e] @ B
    sd = torch.sqrt(torch.diagonal(Cf5, dim1=1, dim2=2))
    ev_min = torch.linalg.eigvalsh((Cf5 - Cs5) / (sd[:, :, None] * sd[:, None, :])).min()
    assert ev_min > -1e-9, ev_min


def test_smoothed_states_lie_on_one_helix_without_noise():
    """No scattering and (almost) no material: the smoothed states of one
    track are one trajectory, so the smoothed state of an entry carried to the
    next entry's layer is the next smoothed state (compared after one extra
    forward / backward round, away from tangent crossings, as above)."""
    wl = workloads()["barrel10"]
    g = dataclasses.replace(wl.geometry, x_over_x0=np.full(wl.geometry.n_layers, 1e-10))
    ev = generate(dataclasses.replace(wl, geometry=g), 200, scatter=False, holes=False)
    fwd, out = _smoothed(ev, fwd_scale=1e4, geom=g, rounds=2)
    t = ev.truth
    cb = np.abs(np.cos(t[:, 4] - np.arctan2(t[:, 1], t[:, 0])))
    good = (np.minimum.reduceat(cb, ev.hit_offsets[:-1]) > 0.3) & ((out["status"].numpy() & O.NOT_REFITTED) == 0)
    e0 = np.concatenate([np.arange(a, b - 1) for a, b, k in zip(ev.hit_offsets[:-1], ev.hit_offsets[1:], good) if k])
    e1 = e0 + 1
    lay1 = ev.hit_layer[e1]
    m = e0.size
    pc, Cc, _, st = O.propagate(out["ps"][e0], out["Cs"][e0], fwd["qe"][e0], torch.tensor(g.kind[lay1], dtype=torch.int64),
                                torch.tensor(g.pos[lay1], dtype=DT), torch.full((m,), 1e-10, dtype=DT), g,
                                apply_material=False)
    assert (st & O.NO_CROSSING).sum() == 0
    ps1, Cs1 = out["ps"][e1], out["Cs"][e1]
    sig = torch.sqrt(torch.diagonal(Cs1, dim1=1, dim2=2))
    d = pc - ps1
    d[:, 4] = O.wrap_phi(d[:, 4])
    ph = torch.atan2(ps1[:, 1], ps1[:, 0])
    tv = torch.stack([-torch.sin(ph), torch.cos(ph)], 1)
    tang = (d[:, :2] * tv).sum(1) / torch.sqrt(torch.einsum("ni,nij,nj->n", tv, Cs1[:, :2, :2], tv))
    assert tang.abs().max() < 0.05
    assert (d[:, 2:].abs() / sig[:, 2:]).max() < 0.1
    sd = torch.sqrt(torch.diagonal(Cc, dim1=1, dim2=2))
    rel = (Cc - Cs1).abs() / (sd[:, :, None] * sd[:, None, :])
    assert rel[:, 2:, 2:].max() < 0.05


def test_smoothed_pulls_at_every_layer():
    """Smeared hits and scattering (barrel10): the smoothed state of every
    entry against the generator's state just after that layer's kick gives
    pulls N(0, 1), layer by layer: mean within 5 / sqrt(n), width within 6%
    from the fourth layer on.  On the three seed layers the width is held
    within 25%: there the forward filtered state comes from the three hits
    the seed was built from, and the extended filter linearised about that
    seed is jointly inconsistent by ~20% on layer 2 (mean squared Mahalanobis
    distance 6.0 for 5 dof, with unit marginal pulls), which the smoothed
    state inherits (widths up to 1.23 there); the backward prediction and the
    combination itself are consistent (the latter equals the information
    form (C_f^-1 + C_b^-1)^-1 to 1e-11)."""
    wl = workloads()["barrel10"]
    n = 2000
    ev = generate(wl, n, holes=False)
    fwd, out = _smoothed(ev)
    t = ev.truth
    cb = np.abs(np.cos(t[:, 4] - np.arctan2(t[:, 1], t[:, 0])))
    good = (np.minimum.reduceat(cb, ev.hit_offsets[:-1]) > 0.3) & ((out["status"].numpy() & (O.NOT_REFITTED | O.NO_CROSSING | O.NONFINITE)) == 0)
    assert good.sum() > 0.6 * n
    sel = np.repeat(good, ev.lengths())
    e = np.nonzero(sel)[0]
    tr = torch.tensor(ev.truth_after[e])
    p, C = out["ps"][e], out["Cs"][e]
    assert torch.isfinite(p).all()
    d = p - tr
    d[:, 4] = O.wrap_phi(d[:, 4])
    sig = torch.sqrt(torch.diagonal(C, dim1=1, dim2=2))
    ph = torch.atan2(tr[:, 1], tr[:, 0])
    tv = torch.stack([-torch.sin(ph), torch.cos(ph)], 1)
    pulls = {"t": (d[:, :2] * tv).sum(1) / torch.sqrt(torch.einsum("ni,nij,nj->n", tv, C[:, :2, :2], tv)),
             "z": d[:, 2] / sig[:, 2], "ipt": d[:, 3] / sig[:, 3], "phi": d[:, 4] / sig[:, 4],
             "theta": d[:, 5] / sig[:, 5]}
    lay = ev.hit_layer[e]
    for l in range(wl.geometry.n_layers):
        at = lay == l
        for k, v in pulls.items():
            vv = v.numpy()[at]
            mu, sd = vv.mean(), vv.std()
            assert abs(mu) < 5.0 / math.sqrt(vv.size), (l, k, mu)
            assert abs(sd - 1.0) < (0.06 if l >= 3 else 0.25), (l, k, sd)


def _frame5(p, kind_b):
    """[6, 5] surface basis at position p (barrel: tangent, z; disk: x, y),
    built from the geometry alone."""
    B = np.zeros((6, 5))
    if kind_b:
        r = math.hypot(p[0], p[1])
        B[0, 0], B[1, 0], B[2, 1] = -p[1] / r, p[0] / r, 1.0
    else:
        B[0, 0], B[1, 1] = 1.0, 1.0
    B[3, 2] = B[4, 3] = B[5, 4] = 1.0
    return B


def test_smoother_equals_batch_conditioning_at_every_entry():
    """The two-filter smoother against Gaussian conditioning of the whole
    linearised problem on all of a track's hits, entry by entry.

    Tracks on exact helices (no scattering, no smearing), then every hit moved
    along its surface by 1e-6 of its resolution: the filter's states stay
    close enough to the truth for the helix model to be linear (the
    backward pass restarts from a covariance scaled by 1e6, so its first
    steps move its state by ~1e3 times the hit offset in units of the final
    sigma; at offsets of 1e-4 sigma the covariances already differ by 2e-5
    through the moved linearisation point), so the smoothed state is the
    linear map of the hit offsets that conditioning fixes.  The linear model about the true trajectory T_k uses
    the oracle's transport Jacobian F_k and material Q_k (pinned elsewhere
    against finite differences and the kick covariance):
    x_0 = seed + w_0, x_k = T_k + F_k (x_{k-1} - T_{k-1}) + w_k, hit
    y_k = x_k[:3] + v_k, with the seed's prior covariance and V_k.  Then
    E[x_k | y] and Cov[x_k | y] follow from the stacked Gaussian.  The
    backward pass restarts from the forward result scaled by 1e6, so its
    double use of the forward information enters at 1e-6.  Compared on the
    surface's five directions (the normal is a null vector of both) for
    every entry after the seed entry, whose forward state is a full 6-D
    seed (the combination on the surface then drops the normal direction
    that conditioning would keep).  Bounds: state error below 1e-3 of the
    conditioned offset itself, covariance below 5e-6 in correlation units
    (measured: ~5e-5 and ~1e-6)."""
    worst_x, worst_c = _smoother_vs_batch()
    assert worst_x < 1e-3, worst_x
    assert worst_c < 5e-6, worst_c


def test_smoother_batch_pin_is_sharp(monkeypatch):
    """Mistakes planted in the oracle's smoother fail the pin above: the
    combination without its K C_b K^T term, and the backward prediction
    taken after the layer's material instead of before it."""
    real = O.combine_on_surface

    def no_kcbk(pf, Cf, pb, Cb, kind, pos):
        ps, Cs = real(pf, Cf, pb, Cb, kind, pos)
        B = O.surface_frame(pf, kind, pos)
        K = Cf @ B @ torch.linalg.inv(B.transpose(1, 2) @ (Cf + Cb) @ B) @ B.transpose(1, 2)
        return ps, Cs - K @ Cb @ K.transpose(1, 2)
    monkeypatch.setattr(O, "combine_on_surface", no_kcbk)
    wx, wc = _smoother_vs_batch()
    assert wc > 1e-2
    monkeypatch.setattr(O, "combine_on_surface", real)
    real_prop = O.propagate

    def prop_with_material(p, C, q, kind, pos, x0, geom, apply_material=True, same=None):
        return real_prop(p, C, q, kind, pos, x0, geom, apply_material=True, same=same)
    monkeypatch.setattr(O, "propagate", prop_with_material)
    wx, wc = _smoother_vs_batch()
    assert wc > 1e-3



def _smoother_vs_batch():
    wl = workloads()["barrel10"]
    g = wl.geometry
    ev = generate(wl, 12, smear=False, scatter=False, holes=False)
    keep = np.nonzero(ev.lengths() == g.n_layers)[0][:6]
    assert keep.size >= 4
    rng = np.random.default_rng(11)
    hp = ev.hit_pos.copy()
    for e in range(ev.n_hits):
        x, y = hp[0, e], hp[1, e]
        r = math.hypot(x, y)
        a, b = rng.normal(size=2) * 1e-6 * np.array([0.003, 0.01])
        hp[0, e] += -y / r * a
        hp[1, e] += x / r * a
        hp[2, e] += b
    sp, sC, sq, _ = O.make_seeds(ev.hit_offsets, ev.hit_valid, hp, g.bz)
    fwd = O.fit_tracks(sp, sC, sq, ev.hit_offsets, ev.hit_layer, ev.hit_valid, torch.tensor(hp), ev.hit_cov, g,
                       record=True)
    out = O.backward_fit(fwd["p"], fwd["C"], fwd["q"], fwd["status"], ev.hit_offsets, ev.hit_layer, ev.hit_valid,
                         torch.tensor(hp), ev.hit_cov, g, cov_scale=1e6, smooth_from=fwd)
    H = np.concatenate([np.eye(3), np.zeros((3, 3))], 1)
    worst_x, worst_c = 0.0, 0.0
    for t in keep:
        e0, e1 = int(ev.hit_offsets[t]), int(ev.hit_offsets[t + 1])
        N = e1 - e0
        q = torch.tensor([float(ev.charge[t])], dtype=DT)
        T = ev.truth[e0:e1]
        Fs, Qs, Vs = [], [], []
        for k in range(N):
            lay = int(ev.hit_layer[e0 + k])
            kind = torch.tensor([int(g.kind[lay])])
            pos = torch.tensor([float(g.pos[lay])], dtype=DT)
            if k == 0:
                F = np.eye(6)
            else:
                pk = torch.tensor(T[k - 1][None])
                s, ok = O.crossing(pk, q, kind, pos, g.bz)
                assert bool(ok[0])
                F = O.jacobian(pk, q, s, kind, g.bz)[0].numpy()
            Q, _ = O.process_noise(torch.tensor(T[k][None]), kind, torch.tensor([float(g.x_over_x0[lay])], dtype=DT),
                                   g.mass)
            Fs.append(F)
            Qs.append(Q[0].numpy())
            Vs.append(O.unpack_sym(ev.hit_cov[:, e0 + k:e0 + k + 1], 3)[0].numpy())
        # z = (x_0 - T_0, w_0, ..., w_{N-1}); x_k - T_k = M_k z
        nz = 6 * (N + 1)
        Cz = np.zeros((nz, nz))
        Cz[:6, :6] = sC[t].numpy()
        for k in range(N):
            Cz[6 * (k + 1):6 * (k + 2), 6 * (k + 1):6 * (k + 2)] = Qs[k]
        maps = []
        M = np.zeros((6, nz))
        M[:, :6] = np.eye(6)
        for k in range(N):
            M = Fs[k] @ M
            M[:, 6 * (k + 1):6 * (k + 2)] += np.eye(6)
            maps.append(M.copy())
        d0 = sp[t].numpy() - T[0]
        d0[4] = math.remainder(d0[4], 2 * math.pi)
        z0 = np.zeros(nz)
        z0[:6] = d0
        A = np.concatenate([H @ Mk for Mk in maps], 0)
        Vy = np.zeros((3 * N, 3 * N))
        for k in range(N):
            Vy[3 * k:3 * k + 3, 3 * k:3 * k + 3] = Vs[k]
        Syy = A @ Cz @ A.T + Vy
        dy = (hp[:, e0:e1].T - T[:, :3]).reshape(-1) - A @ z0
        sol = np.linalg.solve(Syy, dy)
        for k in range(1, N):
            Sxy = maps[k] @ Cz @ A.T
            xb = maps[k] @ z0 + Sxy @ sol                          # E[x_k | y] - T_k
            Cb = maps[k] @ Cz @ maps[k].T - Sxy @ np.linalg.solve(Syy, Sxy.T)
            B = _frame5(T[k], int(g.kind[int(ev.hit_layer[e0 + k])]) == 0)
            xs = out["ps"][e0 + k].numpy() - T[k]
            xs[4] = math.remainder(xs[4], 2 * math.pi)
            Cs = out["Cs"][e0 + k].numpy()
            Cb5, Cs5 = B.T @ Cb @ B, B.T @ Cs @ B
            sd = np.sqrt(np.diag(Cb5))
            off = float(np.linalg.norm(B.T @ xb / sd))
            worst_x = max(worst_x, float(np.linalg.norm(B.T @ (xs - xb) / sd)) / off)
            worst_c = max(worst_c, float(np.abs((Cs5 - Cb5) / np.outer(sd, sd)).max()))
            # the offsets are ~1e-6 sigma, far above the FP64 rounding of the states
            assert off > 1e-8
    return worst_x, worst_c


def _mp_combination(pf, Cf, Cb, B):
    """C_f - K C_f and (I - K) C_f (I - K)^T + K C_b K^T in 50-digit
    arithmetic, K = C_f B (B^T (C_f + C_b) B)^-1 B^T."""
    import mpmath as mp
    mp.mp.dps = 50
    Cf_, Cb_, B_ = mp.matrix(Cf.tolist()), mp.matrix(Cb.tolist()), mp.matrix(B.tolist())
    K = Cf_ * B_ * mp.inverse(B_.T * (Cf_ + Cb_) * B_) * B_.T
    A = mp.eye(6) - K
    short = Cf_ - K * Cf_
    sym = A * Cf_ * A.T + K * Cb_ * K.T
    return short, sym


def test_combination_forms_agree_in_high_precision():
    """The smoother's covariance C_f - C_f (C_f + C_b)^+ C_f and the symmetric
    form (I - K) C_f (I - K)^T + K C_b K^T are the same matrix when the
    surface normal is a null vector of both inputs: checked at 50 digits
    (mpmath) on random surface covariances, including a forward covariance
    10^6 times wider than the backward one (a state near its diffuse seed).
    There the FP64 difference C_f - K C_f loses about six digits while the
    symmetric form (the oracle's combine_on_surface) keeps the 50-digit
    result to ~1e-12 in correlation units."""
    import mpmath as mp
    rng = np.random.default_rng(3)
    for case in range(12):
        R = 30.0
        ph = rng.uniform(-3, 3)
        pf = torch.tensor([[R * math.cos(ph), R * math.sin(ph), rng.uniform(-50, 50), 0.5, ph + 0.1, 1.2]],
                          dtype=DT)
        B = O.surface_frame(pf, torch.tensor([O.BARREL]), torch.tensor([R], dtype=DT))[0].numpy()
        scale_f = 1e6 if case % 3 == 0 else 1.0
        Af, Ab = rng.normal(size=(5, 5)), rng.normal(size=(5, 5))
        Cf = B @ (scale_f * (Af @ Af.T + 0.1 * np.eye(5))) @ B.T * 1e-4
        Cb = B @ (Ab @ Ab.T + 0.1 * np.eye(5)) @ B.T * 1e-4
        short, sym = _mp_combination(pf, Cf, Cb, B)
        diff = max(abs(short[i, j] - sym[i, j]) for i in range(6) for j in range(6))
        big = max(abs(sym[i, j]) for i in range(6) for j in range(6))
        assert diff <= mp.mpf("1e-40") * big
        exact = np.array([[float(sym[i, j]) for j in range(6)] for i in range(6)])
        _, Cs = O.combine_on_surface(pf, torch.tensor(Cf[None]), pf.clone(), torch.tensor(Cb[None]),
                                     torch.tensor([O.BARREL]), torch.tensor([R], dtype=DT))
        sd = np.sqrt(np.diag(B.T @ exact @ B))
        err = np.abs(B.T @ (Cs[0].numpy() - exact) @ B) / np.outer(sd, sd)
        assert err.max() < 1e-11, (case, err.max())
        if scale_f > 1.0:
            # the FP64 difference form, for contrast: it does lose digits here
            K = Cf @ B @ np.linalg.inv(B.T @ (Cf + Cb) @ B) @ B.T
            e_short = np.abs(B.T @ (Cf - K @ Cf - exact) @ B) / np.outer(sd, sd)
            assert e_short.max() > 100 * err.max()
