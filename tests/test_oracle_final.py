"""Pins for the oracle's final fit with outlier rejection: the backward fit
(Sec. 2.2, step 4) in which a hit whose chi2 against the backward prediction
exceeds a cut is not used.  Pinned by: an infinite cut is the backward fit
bit for bit; a hit displaced far beyond the resolution is rejected, and the
result is then exactly the backward fit with that hit marked as a hole; clean
tracks lose (almost) no hits; with a few displaced hits in the sample, the
rejection restores chi2/ndf ~ 1 and N(0, 1) pulls at the first hit."""
import dataclasses
import math

import numpy as np
import torch

from oracle import kf_oracle as O
from toygen import generate, workloads

SHIFT_Z = 1.0   # cm: 100 times the barrel z resolution, beyond the prediction at every pT


def _final(ev, fwd, chi2_cut=O.FINAL_CHI2_CUT, hit_valid=None):
    return O.backward_fit(fwd["p"], fwd["C"], fwd["q"], fwd["status"], ev.hit_offsets, ev.hit_layer,
                          ev.hit_valid if hit_valid is None else hit_valid, torch.tensor(ev.hit_pos), ev.hit_cov,
                          ev.geometry, chi2_cut=chi2_cut)


def _plant(ev, tracks, entry_of_track, shift=SHIFT_Z):
    """A copy of ev with the hit at entry_of_track[t] of every listed track
    moved along z (a barrel hit stays on its cylinder)."""
    hp = ev.hit_pos.copy()
    e = ev.hit_offsets[tracks] + entry_of_track
    sign = np.where(np.arange(len(tracks)) % 2 == 0, 1.0, -1.0)
    hp[2, e] += sign * shift
    return dataclasses.replace(ev, hit_pos=hp), e


def test_infinite_cut_is_the_backward_fit():
    ev = generate(workloads()["barrel10"], 200)
    fwd = O.fit_event(ev)
    a = _final(ev, fwd, chi2_cut=math.inf)
    b = _final(ev, fwd, chi2_cut=None)
    for k in ("p", "C", "q", "chi2", "ndf", "status"):
        assert torch.equal(a[k], b[k]), k
    assert not a["outlier"].any()


def test_displaced_hit_is_rejected_and_equals_the_fit_without_it():
    n = 400
    ev0 = generate(workloads()["barrel10"], n, holes=False)
    tracks = np.arange(n)
    ev, e_bad = _plant(ev0, tracks, 5)
    fwd = O.fit_event(ev)
    out = _final(ev, fwd)
    ok = (out["status"].numpy() & (O.NO_CROSSING | O.NONFINITE | O.NOT_REFITTED)) == 0
    out_mask = out["outlier"].numpy()
    hit = out_mask[e_bad]
    assert hit[ok].mean() >= 0.97, hit[ok].mean()
    assert ((out["status"].numpy()[hit] & O.OUTLIER) != 0).all()
    # the tracks whose only rejected hit is the displaced one: exactly the
    # backward fit with that hit taken as a hole
    n_rej = np.add.reduceat(out_mask.astype(np.int64), ev.hit_offsets[:-1])
    only = ok & hit & (n_rej == 1)
    assert only.mean() >= 0.95, only.mean()
    hv = ev.hit_valid.copy()
    hv[e_bad] = 0
    ref = _final(ev, fwd, chi2_cut=None, hit_valid=hv)
    t = torch.tensor(np.nonzero(only)[0])
    for k in ("p", "C", "q", "chi2", "ndf"):
        assert torch.equal(out[k][t], ref[k][t]), k
    assert torch.equal(out["status"][t] & ~O.OUTLIER, ref["status"][t])


def test_clean_tracks_keep_their_hits():
    ev = generate(workloads()["barrel10"], 1000)
    fwd = O.fit_event(ev)
    out = _final(ev, fwd)
    base = _final(ev, fwd, chi2_cut=None)
    valid = ev.hit_valid == 1
    frac = out["outlier"].numpy()[valid].mean()
    assert frac < 1e-3, frac
    # tracks with no rejection are the backward fit unchanged
    n_rej = np.add.reduceat(out["outlier"].numpy().astype(np.int64), ev.hit_offsets[:-1])
    t = torch.tensor(np.nonzero(n_rej == 0)[0])
    assert torch.equal(out["p"][t], base["p"][t]) and torch.equal(out["chi2"][t], base["chi2"][t])


def _first_hit_stats(ev, out, sel):
    first = ev.hit_offsets[:-1]
    ratio = out["chi2"].numpy()[sel].sum() / out["ndf"].numpy()[sel].sum()
    tr = torch.tensor(ev.truth[first])
    d = out["p"] - tr
    d[:, 4] = O.wrap_phi(d[:, 4])
    sig = torch.sqrt(torch.diagonal(out["C"], dim1=1, dim2=2))
    pz = (d[:, 2] / sig[:, 2]).numpy()[sel]
    pt = (d[:, 5] / sig[:, 5]).numpy()[sel]
    return ratio, pz.std(), pt.std()


def test_rejection_restores_the_statistics():
    """One displaced hit on every tenth track: without rejection those
    tracks' chi2 blows up and the sample's z pulls at the first hit widen;
    with it, chi2 / ndf ~ 1 and the pulls are N(0, 1) again."""
    n = 2000
    ev0 = generate(workloads()["barrel10"], n, holes=False)
    rng = np.random.default_rng(11)
    tracks = np.arange(0, n, 10)
    ev, _ = _plant(ev0, tracks, rng.integers(4, 8, size=tracks.size))
    fwd = O.fit_event(ev)
    out = _final(ev, fwd)
    plain = _final(ev, fwd, chi2_cut=None)
    ok = (out["status"].numpy() & (O.NO_CROSSING | O.NONFINITE | O.NOT_REFITTED)) == 0
    t = ev.truth
    cb = np.abs(np.cos(t[:, 4] - np.arctan2(t[:, 1], t[:, 0])))
    sel = ok & (np.minimum.reduceat(cb, ev.hit_offsets[:-1]) > 0.3)
    assert sel.sum() > 0.6 * n
    r_plain, _, _ = _first_hit_stats(ev, plain, sel)
    r, sz, st = _first_hit_stats(ev, out, sel)
    ndf = out["ndf"].numpy()[sel].sum()
    assert r_plain > 2.0, r_plain
    assert abs(r - 1.0) < 4.0 * math.sqrt(2.0 / ndf), r
    assert abs(sz - 1.0) < 0.06 and abs(st - 1.0) < 0.06, (sz, st)
