"""Pins for the oracle's seeding and full fit: exact seeds on noise-free hits,
and the statistical signature of an unbiased, correctly-weighted filter on toys
(chi2/ndf ~ 1, uniform chi2 p-values, pulls ~ N(0,1) against the generator's
truth), plus status handling."""
import math

import numpy as np
import torch
from scipy import stats

from oracle import kf_oracle as O
from toygen import generate, subset, workloads

DT = torch.float64


def test_seed_exact_on_noise_free_hits():
    for name, mode in (("barrel10", O.SEED_FIRST_THREE), ("mixed26", O.SEED_FIRST_THREE),
                       ("mixed26", O.SEED_SPACED)):
        wl = workloads()[name]
        ev = generate(wl, 300, smear=False, scatter=False, holes=False)
        p, C0, q, ok = O.make_seeds(ev.hit_offsets, ev.hit_valid, ev.hit_pos, wl.geometry.bz, mode=mode)
        first = ev.hit_offsets[:-1]
        tr = torch.tensor(ev.truth[first])
        d = p - tr
        d[:, 4] = O.wrap_phi(d[:, 4])
        assert bool(ok.all())
        assert d[:, :3].abs().max() < 1e-12
        assert (d[:, 3].abs() / tr[:, 3]).max() < 1e-9
        assert d[:, 4:].abs().max() < 1e-10
        assert torch.equal(q, torch.tensor(ev.charge, dtype=DT))


def _min_cos_incidence(ev):
    """Smallest transverse incidence cos(phi - phi_pos) over a track's barrel
    crossings (1 for disks).  Near-tangent crossings make the extended filter
    visibly non-linear (the crossing point moves a lot for a small direction
    error), so the statistical pins select tracks away from them."""
    g = ev.geometry
    t = ev.truth
    kind = g.kind[ev.hit_layer]
    cb = np.abs(np.cos(t[:, 4] - np.arctan2(t[:, 1], t[:, 0])))
    c = np.where(kind == 0, cb, 1.0)
    return np.minimum.reduceat(c, ev.hit_offsets[:-1])


def _pulls(ev, out):
    last = ev.hit_offsets[1:] - 1
    tr = torch.tensor(ev.truth_after[last])
    p, C = out["p"], out["C"]
    d = p - tr
    d[:, 4] = O.wrap_phi(d[:, 4])
    sig = torch.sqrt(torch.diagonal(C, dim1=1, dim2=2))
    kind = torch.tensor(ev.geometry.kind[ev.hit_layer[last]])
    # barrel: tangent direction in xy; disk: the two transverse axes are both measured,
    # use the azimuthal direction there too
    ph = torch.atan2(tr[:, 1], tr[:, 0])
    t = torch.stack([-torch.sin(ph), torch.cos(ph)], 1)
    dt = (d[:, :2] * t).sum(1)
    Ct = torch.einsum("ni,nij,nj->n", t, C[:, :2, :2], t)
    out = {"t": dt / torch.sqrt(Ct), "ipt": d[:, 3] / sig[:, 3], "phi": d[:, 4] / sig[:, 4],
           "theta": d[:, 5] / sig[:, 5]}
    out["z"] = torch.where(kind == 0, d[:, 2] / sig[:, 2], torch.zeros_like(dt))
    return out, kind


def _check_statistics(name, n, cos_cut, seed_mode=O.SEED_FIRST_THREE):
    wl = workloads()[name]
    ev = generate(wl, n)
    out = O.fit_event(ev, seed_mode=seed_mode)
    sel = (_min_cos_incidence(ev) > cos_cut) & (out["status"].numpy() == 0)
    chi2 = out["chi2"].numpy()[sel]
    ndf = out["ndf"].numpy()[sel]
    m = sel.sum()
    assert m > 0.6 * n
    ratio = chi2.sum() / ndf.sum()
    # sum of chi2 ~ chi2(sum ndf): 4 sigma band
    assert abs(ratio - 1.0) < 4.0 * math.sqrt(2.0 / ndf.sum()), ratio
    pv = stats.chi2.sf(chi2, ndf)
    assert stats.kstest(pv, "uniform").pvalue > 1e-3
    pulls, kind = _pulls(ev, out)
    for k, v in pulls.items():
        vv = v.numpy()[sel]
        if k == "z":
            vv = vv[kind.numpy()[sel] == 0]
        mu, sd = vv.mean(), vv.std()
        assert abs(mu) < 5.0 / math.sqrt(vv.size), (k, mu)
        assert abs(sd - 1.0) < 0.06, (k, sd)
    return out


def test_fit_statistics_barrel10():
    _check_statistics("barrel10", 2000, 0.3)


def test_fit_statistics_mixed26():
    out = _check_statistics("mixed26", 2000, 0.3, seed_mode=O.SEED_SPACED)
    assert (out["ndf"].numpy() >= 1).all()


def test_ndf_counts_valid_hits_and_holes_keep_material():
    wl = workloads()["mixed26"]
    ev = generate(wl, 200)
    out = O.fit_event(ev, seed_mode=O.SEED_SPACED)
    nvalid = np.add.reduceat(ev.hit_valid.astype(np.int64), ev.hit_offsets[:-1])
    ok = out["status"].numpy() & (O.NO_CROSSING | O.NONFINITE) == 0
    assert np.array_equal(out["ndf"].numpy()[ok], 2 * nvalid[ok] - 5)


def test_tracks_are_independent():
    wl = workloads()["mixed26"]
    ev = generate(wl, 300)
    full = O.fit_event(ev)
    pick = [5, 77, 150, 299]
    part = O.fit_event(subset(ev, pick))
    assert torch.equal(full["p"][pick], part["p"])
    assert torch.equal(full["chi2"][pick], part["chi2"])


def test_unreachable_layer_freezes_track():
    wl = workloads()["barrel10"]
    ev = generate(wl, 20)
    g = wl.geometry
    # a fake geometry whose last layer is out of reach of a 0.5-10 GeV track from r = 85
    from toygen import barrel_geometry
    g2 = barrel_geometry(list(g.pos[:-1]) + [5000.0])
    sp, sC, sq, _ = O.make_seeds(ev.hit_offsets, ev.hit_valid, ev.hit_pos, g.bz)
    out = O.fit_tracks(sp, sC, sq, ev.hit_offsets, ev.hit_layer, ev.hit_valid, torch.tensor(ev.hit_pos),
                       ev.hit_cov, g2)
    ref = O.fit_tracks(sp, sC, sq, ev.hit_offsets - 0, ev.hit_layer, ev.hit_valid, torch.tensor(ev.hit_pos),
                       ev.hit_cov, g)
    lens = ev.lengths()
    hit_last = lens == 10
    st = out["status"].numpy()
    assert ((st[hit_last] & O.NO_CROSSING) != 0).all()
    assert ((st[~hit_last] & O.NO_CROSSING) == 0).all()
    assert torch.isfinite(out["p"]).all() and torch.isfinite(out["C"]).all()
    # frozen at the state after entry 9, i.e. the fit of the first nine entries
    from toygen import truncate
    ev9 = truncate(ev, np.full(20, 9))
    r9 = O.fit_tracks(sp, sC, sq, ev9.hit_offsets, ev9.hit_layer, ev9.hit_valid, torch.tensor(ev9.hit_pos),
                      ev9.hit_cov, g)
    assert torch.equal(out["p"][hit_last], r9["p"][hit_last])
    assert torch.equal(out["chi2"][hit_last], r9["chi2"][hit_last])


def test_spaced_seed_choice_matches_brute_force():
    wl = workloads()["mixed26"]
    ev = generate(wl, 300)
    idx = O.spaced_three_valid(ev.hit_offsets, ev.hit_valid, ev.hit_pos).numpy()
    for t in range(ev.n_tracks):
        chosen = []
        for e in range(ev.hit_offsets[t], ev.hit_offsets[t + 1]):
            if not ev.hit_valid[e] or len(chosen) == 3:
                continue
            if not chosen or math.hypot(*(ev.hit_pos[:2, e] - ev.hit_pos[:2, chosen[-1]])) >= O.SEED_MIN_SPACING:
                chosen.append(e)
        expect = chosen if len(chosen) == 3 else [-1, -1, -1]
        assert list(idx[t]) == expect
