"""GPU parity of the final fit with outlier rejection (kf_final_fit, through
the C interface): rounds of seeding, forward fit and smoothing backward fit,
each rejecting the hit whose unbiased chi2 (against the estimate from the
track's other hits) is worst and above the cut.  Both sides start from the
same hits, in events where one hit of every tenth track -- anywhere on it,
first and last entries included -- is moved by 1 cm along its surface.
States, covariances, chi2 and status are held to the backward fit's
tolerances, the outlier masks must agree entry by entry and the per-hit
unbiased chi2 to its own tolerance, on every track the conditioning probes
do not flag (a probe that moves a track's result or a hit's chi2, or flips
one of its rejections, flags it).  A cut no chi2 reaches gives the bits of
kf_seed_fit_tracks followed by kf_smooth_tracks."""
from __future__ import annotations

import dataclasses
import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

from oracle import kf_oracle as O
from toygen import generate, subset, workloads

from parity import BACKWARD_SCALE, chi2_error, compare_fit, outputs_np, param_error, rounded

pytestmark = pytest.mark.gpu

TOL32 = (1e-4, 1e-3)
TOL64 = (1e-8, 1e-8)
# per-hit unbiased chi2: |d| <= tol * max(chi2, 1).  FP32: the smoothed
# position (rounded to FP32, ~1e-5 of a residual at r ~ 100 cm) and the
# difference R = V - H C_s H^T of two comparable FP32 matrices
HIT_TOL32 = 2e-2
HIT_TOL64 = 1e-6
CUT = O.FINAL_CHI2_CUT


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_11728_amd import kf as _kf
    return _kf


@pytest.fixture(scope="module")
def ctx(kf):
    c = kf.Context(0)
    c.set_fit_launch(torch.float32, 256, 0, 1, 2, 3)
    c.set_fit_launch(torch.float64, 256, 0, 1, 1, 3)
    yield c
    c.close()


def planted(ev, every=10, seed=3, shift=1.0):
    """A copy of ev in which one hit (any entry, first and last included) of
    every `every`-th track is moved by `shift` cm along its surface: along z
    on a barrel, along x on a disk."""
    rng = np.random.default_rng(seed)
    hp = ev.hit_pos.copy()
    tracks = np.arange(0, ev.n_tracks, every)
    lens = ev.lengths()[tracks]
    e = ev.hit_offsets[tracks] + rng.integers(0, lens)
    disk = ev.geometry.kind[ev.hit_layer[e]] == O.DISK
    sign = np.where(rng.random(tracks.size) < 0.5, -1.0, 1.0)
    hp[2, e[~disk]] += shift * sign[~disk]
    hp[0, e[disk]] += shift * sign[disk]
    return dataclasses.replace(ev, hit_pos=hp)


def oracle_final(ev, dtype, seed_mode=0, chi2_cut=CUT, hit_pos=None, state_round=None, state_jitter=None, **kw):
    hp = rounded(ev.hit_pos, dtype) if hit_pos is None else np.asarray(hit_pos, np.float64)
    f = O.final_fit(ev.hit_offsets, ev.hit_layer, ev.hit_valid, torch.tensor(hp), rounded(ev.hit_cov, dtype),
                    ev.geometry, seed_mode=seed_mode, chi2_cut=chi2_cut, cov_scale=BACKWARD_SCALE,
                    state_round=state_round, state_jitter=state_jitter, **kw)
    return dict(p=f["p"].numpy(), C=f["C"].numpy(), q=f["q"].numpy(), chi2=f["chi2"].numpy(), ndf=f["ndf"].numpy(),
                status=f["status"].numpy(), outlier=f["outlier"].numpy().astype(np.uint8),
                hit_chi2=f["hit_chi2"].numpy(), rounds=f["rounds"].numpy())


def gpu_final(c, kf, ev, dtype, seed_mode=0, chi2_cut=CUT, prefill=None, **kw):
    dev = c.device
    t = kf.event_tensors(ev, dtype, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    outlier = None if prefill is None else torch.full((ev.n_hits,), prefill, dtype=torch.uint8, device=dev)
    out, mask, hc = c.final_fit(t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom,
                                seed_mode, chi2_cut=chi2_cut, cov_scale=BACKWARD_SCALE, outlier=outlier, **kw)
    torch.cuda.synchronize()
    r = outputs_np(out)
    r["outlier"] = mask.cpu().numpy()
    r["hit_chi2"] = hc.double().cpu().numpy()
    return r


def hit_chi2_error(a, b):
    """|a - b| / max(|b|, 1) per entry; 0 where both are NaN, inf where one is."""
    both = np.isnan(a) & np.isnan(b)
    err = np.abs(a - b) / np.maximum(np.abs(b), 1.0)
    return np.where(both, 0.0, np.nan_to_num(err, nan=np.inf))


def per_track_max(ev, x):
    return np.maximum.reduceat(x, ev.hit_offsets[:-1]) if ev.n_hits else np.zeros(ev.n_tracks)


def final_probes(ev, dtype, seed_mode, ref, tol, hit_tol, seed=99):
    """Tracks whose oracle result moves by more than half the tolerance, whose
    status or closing round changes, one of whose rejections flips or one of
    whose hit chi2 moves by more than half its tolerance under the
    rounding-level probes."""
    rng = np.random.default_rng(seed)
    hp = rounded(ev.hit_pos, dtype)
    if dtype == torch.float32:
        ulp = np.spacing(np.abs(hp).astype(np.float32)).astype(np.float64)
        probes = [dict(hit_pos=hp + ulp * rng.choice([-1.0, 1.0], size=hp.shape)), dict(state_round=torch.float32)]
    else:
        ulp = 1e-13 * np.maximum(np.abs(hp), 1.0)
        probes = [dict(hit_pos=hp + ulp * rng.choice([-1.0, 1.0], size=hp.shape)), dict(state_jitter=4e-16)]
    bad = np.zeros(ev.n_tracks, bool)
    for kw in probes:
        o2 = oracle_final(ev, dtype, seed_mode, **kw)
        flip = per_track_max(ev, (o2["outlier"] != ref["outlier"]).astype(np.int64)) > 0
        hmove = per_track_max(ev, hit_chi2_error(o2["hit_chi2"], ref["hit_chi2"])) > 0.5 * hit_tol
        bad |= (param_error(o2["p"], ref["p"]).max(axis=1) > 0.5 * tol[0]) | \
               (chi2_error(o2["chi2"], ref["chi2"]) > 0.5 * tol[1]) | (o2["status"] != ref["status"]) | \
               (o2["rounds"] != ref["rounds"]) | flip | hmove
    return bad


def _case(c, kf, ev, dtype, seed_mode, max_bad_frac, tail_frac, sample=None):
    """GPU on the whole batch, the oracle on `sample` of its tracks (each
    track's rounds depend on its own hits only) or on all."""
    fp32 = dtype == torch.float32
    tol, hit_tol = (TOL32, HIT_TOL32) if fp32 else (TOL64, HIT_TOL64)
    g = gpu_final(c, kf, ev, dtype, seed_mode)
    if sample is not None:
        pick = np.sort(np.random.default_rng(21).choice(ev.n_tracks, sample, replace=False))
        sub = subset(ev, pick)
        ent = np.concatenate([np.arange(ev.hit_offsets[t], ev.hit_offsets[t + 1]) for t in pick])
        g = {k: (v[ent] if k in ("outlier", "hit_chi2") else v[pick]) for k, v in g.items()}
        ev = sub
    of = oracle_final(ev, dtype, seed_mode)
    bad = final_probes(ev, dtype, seed_mode, of, tol, hit_tol)
    assert bad.mean() <= max(max_bad_frac, 0.005), bad.mean()
    s = compare_fit(g, of, tol[0], tol[1], ~bad, tail_frac=tail_frac, geom=ev.geometry)
    ok_e = np.repeat(~bad, ev.lengths())
    assert np.array_equal(g["outlier"][ok_e], of["outlier"][ok_e])
    assert set(np.unique(g["outlier"])) <= {0, 1}
    he = hit_chi2_error(g["hit_chi2"], of["hit_chi2"])
    nan_diff = np.nonzero(ok_e & (np.isnan(g["hit_chi2"]) != np.isnan(of["hit_chi2"])))[0]
    for e in nan_diff[:5]:
        t = int(np.searchsorted(ev.hit_offsets, e, side="right") - 1)
        e0, e1 = ev.hit_offsets[t], ev.hit_offsets[t + 1]
        say("  nan mismatch: track", t, "entry", int(e - e0), "of", int(e1 - e0), "valid", ev.hit_valid[e0:e1],
            "layers", ev.hit_layer[e0:e1], "gpu", g["hit_chi2"][e0:e1], "oracle", of["hit_chi2"][e0:e1],
            "status gpu/oracle", int(g["status"][t]), int(of["status"][t]), "rounds", int(of["rounds"][t]))
    assert nan_diff.size == 0, nan_diff[:10]
    assert (he[ok_e] <= hit_tol).mean() >= 1.0 - tail_frac and (he[ok_e] <= 10 * hit_tol).all(), he[ok_e].max()
    n_out = int(of["outlier"].sum())
    planted_n = len(range(0, ev.n_tracks, 10)) if sample is None else None
    if planted_n is not None:
        assert n_out >= 0.8 * planted_n   # the displaced hits are found
    assert ((of["status"] & O.OUTLIER) != 0).sum() == np.count_nonzero(per_track_max(ev, of["outlier"].astype(np.int64)))
    s.update(ill_conditioned=int(bad.sum()), rejected=n_out, rejected_gpu=int(g["outlier"].sum()),
             max_hit_chi2_err=float(he[ok_e].max(initial=0.0)), rounds_max=int(of["rounds"].max(initial=0)))
    say(s)


@pytest.mark.parametrize("name,n,mode,dtype", [("barrel10", None, 0, torch.float64), ("barrel10", None, 0, torch.float32),
                                               ("mixed26", 3000, 1, torch.float64),
                                               ("mixed26", 3000, 1, torch.float32)])
def test_final_fit_parity(ctx, kf, name, n, mode, dtype):
    say("final fit", name, n, dtype)
    ev = planted(generate(workloads()[name], n))
    fp32 = dtype == torch.float32
    _case(ctx, kf, ev, dtype, mode, 0.05 if fp32 else 0.0, 0.005 if fp32 else 0.0)


def test_final_fit_barrel20_full_size(ctx, kf):
    """100,000 tracks x 20 layers, one displaced hit on every tenth, FP32 and
    FP64 on the GPU; the oracle on 5,000 sampled tracks."""
    say("final fit barrel20 100k fp32 (oracle on 5k)")
    ev = planted(generate(workloads()["barrel20"]))
    _case(ctx, kf, ev, torch.float32, 0, 0.02, 0.002, sample=5000)
    say("final fit barrel20 100k fp64 (oracle on 5k)")
    _case(ctx, kf, ev, torch.float64, 0, 0.0, 1e-3, sample=5000)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_no_rejection_is_the_smoothed_fit(ctx, kf, dtype):
    """A cut no chi2 reaches: one round, whose result is the bits of
    kf_seed_fit_tracks (with its filtered states) followed by
    kf_smooth_tracks, and every entry of the mask written (0) over a buffer
    filled with 7."""
    say("final fit, no rejection", dtype)
    ev = planted(generate(workloads()["barrel10"], 3000))
    g = gpu_final(ctx, kf, ev, dtype, chi2_cut=1e300, prefill=7)
    dev = ctx.device
    t = kf.event_tensors(ev, dtype, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    n, max_len = ev.n_tracks, 26
    ck = torch.empty(28, n * (max_len - 1), dtype=dtype, device=dev)
    fwd = ctx.seed_fit_tracks(t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom, 0,
                              checkpoints=ck, seg=1, max_len=max_len)
    out, _ = ctx.smooth_tracks(fwd, ck, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"],
                               geom, cov_scale=BACKWARD_SCALE, max_len=max_len)
    torch.cuda.synchronize()
    b = outputs_np(out)
    for k in ("p", "C", "q", "chi2", "ndf", "status"):
        assert np.array_equal(g[k], b[k]), k
    assert (g["outlier"] == 0).all()


def test_final_fit_ragged_sizes_and_repeat(ctx, kf):
    """Batches that end inside a wave and inside a block, then a second call
    on the same context with a smaller batch (the workspace keeps the larger
    call's contents)."""
    ev0 = planted(generate(workloads()["barrel10"], 700))
    for n in (700, 1, 63, 65, 257):
        ev = subset(ev0, np.arange(n))
        of = oracle_final(ev, torch.float64)
        g = gpu_final(ctx, kf, ev, torch.float64, prefill=9)
        assert np.array_equal(g["outlier"], of["outlier"]), n
        ep = param_error(g["p"], of["p"]).max(axis=1)
        assert (ep <= 1e-7).all(), (n, ep.max())
    say("ragged ok")


def test_final_fit_offsets_past_zero(ctx, kf):
    """The tracks' entries need not start at entry 0 of the hit arrays: the
    same tracks behind 7 entries that belong to no track (valid hits, so that
    a kernel reading them would use them) and before 5 more give the same
    results bit for bit, and the entries outside the tracks keep what the
    caller's outlier and hit_chi2 arrays held."""
    say("final fit, offsets past zero")
    ev = planted(generate(workloads()["barrel10"], 300))
    dev = ctx.device
    for dt in (torch.float32, torch.float64):
        t = kf.event_tensors(ev, dt, dev)
        geom = kf.Geometry.from_toy(ev.geometry)
        nh = ev.n_hits
        ref = ctx.final_fit(t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom, 0,
                            chi2_cut=CUT, cov_scale=BACKWARD_SCALE)
        front, back = 7, 5
        src = (torch.arange(front + nh + back, device=dev) - front) % nh   # entry front + e holds hit e; the padding copies real hits
        pad = lambda x: x[..., src].contiguous()
        off = (t["hit_offsets"] + front).contiguous()
        mask = torch.full((front + nh + back,), 9, dtype=torch.uint8, device=dev)
        hc = torch.full((front + nh + back,), -5.0, dtype=dt, device=dev)
        valid = pad(t["hit_valid"])
        valid[:front] = 1
        valid[front + nh:] = 1
        got = ctx.final_fit(off, pad(t["hit_layer"]), valid, pad(t["hit_pos"]), pad(t["hit_cov"]), geom, 0,
                            chi2_cut=CUT, cov_scale=BACKWARD_SCALE, outlier=mask, hit_chi2=hc)
        torch.cuda.synchronize()
        for k in ref[0]:
            assert torch.equal(ref[0][k], got[0][k]), (dt, k)
        assert torch.equal(got[1][front:front + nh], ref[1]), dt
        assert torch.equal(got[2][front:front + nh].nan_to_num(7.0), ref[2].nan_to_num(7.0)), dt
        assert (mask[:front] == 9).all() and (mask[front + nh:] == 9).all(), dt
        assert (hc[:front] == -5.0).all() and (hc[front + nh:] == -5.0).all(), dt
        assert int(ref[1].sum()) > 0
    say("offsets past zero ok")


def test_final_fit_limits_and_degenerate_cut(ctx, kf):
    """max_reject = 0 is the smoothed fit; a tiny cut rejects a hit in every
    round it may (max_reject of them) unless the track would keep fewer than
    min_keep hits; the oracle agrees on both."""
    say("final fit limits")
    ev = generate(workloads()["barrel10"], 500)
    dt = torch.float64
    g0 = gpu_final(ctx, kf, ev, dt, max_reject=0)
    assert (g0["outlier"] == 0).all()
    for max_reject, min_keep in ((3, 4), (5, 8)):
        of = oracle_final(ev, dt, chi2_cut=1e-30, max_reject=max_reject, min_keep=min_keep)
        g = gpu_final(ctx, kf, ev, dt, chi2_cut=1e-30, max_reject=max_reject, min_keep=min_keep)
        assert np.array_equal(g["outlier"], of["outlier"])
        n_rej = per_track_max(ev, np.zeros(ev.n_hits)) * 0 + np.add.reduceat(g["outlier"].astype(np.int64),
                                                                             ev.hit_offsets[:-1])
        nval = np.add.reduceat(ev.hit_valid.astype(np.int64), ev.hit_offsets[:-1])
        refit = (of["status"] & O.NOT_REFITTED) == 0
        assert np.array_equal(n_rej[refit], np.minimum(max_reject, np.maximum(nval - min_keep, 0))[refit])
        assert (param_error(g["p"], of["p"]).max(axis=1) <= 1e-7).all()
