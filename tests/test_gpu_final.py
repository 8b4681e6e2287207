"""GPU parity of the final fit with outlier rejection (kf_final_fit): the
backward fit in which a hit whose chi2 against the backward prediction
exceeds the cut is not used.  Both sides start from the oracle's forward
result (rounded to the working precision) on events in which every tenth
track carries one hit displaced by 1 cm along its surface.  States, chi2 and
status are held to the backward fit's tolerances and the outlier masks must
agree entry by entry, on every track the conditioning probes do not flag (a
probe that moves a track's result or flips one of its rejections flags it).
An infinite cut gives kf_backward_fit's bits."""
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

from parity import (BACKWARD_SCALE, chi2_error, compare_fit, gpu_backward, oracle_fit, outputs_np, pack21,
                    param_error, rounded, rounded_forward)

pytestmark = pytest.mark.gpu

TOL32 = (1e-4, 1e-3)
TOL64 = (1e-8, 1e-8)
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
    yield c
    c.close()


def planted(ev, every=10, seed=3):
    """A copy of ev in which one hit (entries 3..6) of every `every`-th track
    is moved by 1 cm along its surface: along z on a barrel, along x on a
    disk."""
    rng = np.random.default_rng(seed)
    hp = ev.hit_pos.copy()
    tracks = np.arange(0, ev.n_tracks, every)
    lens = ev.lengths()[tracks]
    e = ev.hit_offsets[tracks] + np.minimum(rng.integers(3, 7, size=tracks.size), lens - 1)
    disk = ev.geometry.kind[ev.hit_layer[e]] == O.DISK
    sign = np.where(rng.random(tracks.size) < 0.5, -1.0, 1.0)
    hp[2, e[~disk]] += sign[~disk]
    hp[0, e[disk]] += sign[disk]
    return dataclasses.replace(ev, hit_pos=hp)


def oracle_final(ev, dtype, fwd, chi2_cut=CUT, hit_pos=None, state_round=None, state_jitter=None):
    hp = rounded(ev.hit_pos, dtype) if hit_pos is None else np.asarray(hit_pos, np.float64)
    b = O.backward_fit(torch.tensor(fwd["p"]), torch.tensor(fwd["C"]), torch.tensor(fwd["q"]),
                       torch.tensor(fwd["status"]), ev.hit_offsets, ev.hit_layer, ev.hit_valid, torch.tensor(hp),
                       rounded(ev.hit_cov, dtype), ev.geometry, cov_scale=BACKWARD_SCALE, state_round=state_round,
                       state_jitter=state_jitter, chi2_cut=chi2_cut)
    return dict(p=b["p"].numpy(), C=b["C"].numpy(), q=b["q"].numpy(), chi2=b["chi2"].numpy(), ndf=b["ndf"].numpy(),
                status=b["status"].numpy(), outlier=b["outlier"].numpy().astype(np.uint8))


def gpu_final(c, kf, ev, dtype, fwd, chi2_cut=CUT, prefill=None):
    dev = c.device
    t = kf.event_tensors(ev, dtype, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    f = dict(state=torch.tensor(np.ascontiguousarray(fwd["p"].T), dtype=dtype, device=dev),
             cov=torch.tensor(np.ascontiguousarray(pack21(fwd["C"])), dtype=dtype, device=dev),
             charge=torch.tensor(fwd["q"].astype(np.int8), device=dev),
             status=torch.tensor(fwd["status"].astype(np.int32), device=dev))
    outlier = None
    if prefill is not None:
        outlier = torch.full((ev.n_hits,), prefill, dtype=torch.uint8, device=dev)
    out, mask = c.final_fit(f, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom,
                            chi2_cut=chi2_cut, cov_scale=BACKWARD_SCALE, outlier=outlier)
    torch.cuda.synchronize()
    r = outputs_np(out)
    r["outlier"] = mask.cpu().numpy()
    return r


def final_probes(ev, dtype, fwd, ref, tol, seed=99):
    """Tracks whose oracle result moves by more than half the tolerance, whose
    status changes, or one of whose rejections flips under the rounding-level
    probes."""
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
        o2 = oracle_final(ev, dtype, fwd, **kw)
        flip = np.maximum.reduceat((o2["outlier"] != ref["outlier"]).astype(np.int64), ev.hit_offsets[:-1]) > 0 \
            if ev.n_hits else np.zeros(ev.n_tracks, bool)
        bad |= (param_error(o2["p"], ref["p"]).max(axis=1) > 0.5 * tol[0]) | \
               (chi2_error(o2["chi2"], ref["chi2"]) > 0.5 * tol[1]) | (o2["status"] != ref["status"]) | flip
    return bad


def _case(c, kf, ev, dtype, seed_mode, tol, max_bad_frac, tail_frac):
    fwd = rounded_forward(oracle_fit(ev, dtype, seed_mode), dtype)
    of = oracle_final(ev, dtype, fwd)
    bad = final_probes(ev, dtype, fwd, of, tol)
    assert bad.mean() <= max(max_bad_frac, 0.005), bad.mean()
    g = gpu_final(c, kf, ev, dtype, fwd)
    s = compare_fit(g, of, tol[0], tol[1], ~bad, tail_frac=tail_frac)
    ok_e = np.repeat(~bad, ev.lengths())
    assert np.array_equal(g["outlier"][ok_e], of["outlier"][ok_e])
    assert set(np.unique(g["outlier"])) <= {0, 1}
    n_out = int(of["outlier"].sum())
    assert n_out >= 0.8 * (ev.n_tracks // 10)   # the displaced hits are found
    assert ((of["status"] & O.OUTLIER) != 0).sum() == np.count_nonzero(
        np.add.reduceat(of["outlier"].astype(np.int64), ev.hit_offsets[:-1]))
    s.update(ill_conditioned=int(bad.sum()), rejected=n_out, rejected_gpu=int(g["outlier"].sum()))
    say(s)


@pytest.mark.parametrize("name,n,mode,dtype", [("barrel10", None, 0, torch.float64), ("barrel10", None, 0, torch.float32),
                                               ("mixed26", 3000, 1, torch.float64),
                                               ("mixed26", 3000, 1, torch.float32)])
def test_final_fit_parity(ctx, kf, name, n, mode, dtype):
    say("final fit", name, n, dtype)
    ev = planted(generate(workloads()[name], n))
    fp32 = dtype == torch.float32
    _case(ctx, kf, ev, dtype, mode, TOL32 if fp32 else TOL64, 0.05 if fp32 else 0.0, 0.005 if fp32 else 0.0)


def test_final_fit_barrel20_full_size(ctx, kf):
    """100,000 tracks x 20 layers, one displaced hit on every tenth, in FP32
    and FP64."""
    say("final fit barrel20 100k fp32")
    ev = planted(generate(workloads()["barrel20"]))
    _case(ctx, kf, ev, torch.float32, 0, TOL32, 0.02, 0.002)
    say("final fit barrel20 100k fp64")
    _case(ctx, kf, ev, torch.float64, 0, TOL64, 0.0, 1e-4)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_infinite_cut_is_the_backward_fit(ctx, kf, dtype):
    """No hit rejected: kf_backward_fit's result (the same arithmetic in
    another kernel, so equal up to the compiler's contraction choices), and
    every entry of the mask written (0) over a buffer filled with 7."""
    say("final fit, infinite cut", dtype)
    ev = planted(generate(workloads()["barrel10"], 3000))
    fwd = rounded_forward(oracle_fit(ev, dtype, 0), dtype)
    g = gpu_final(ctx, kf, ev, dtype, fwd, chi2_cut=float("inf"), prefill=7)
    b = gpu_backward(ctx, kf, ev, dtype, fwd)
    for k in ("q", "ndf", "status"):
        assert np.array_equal(g[k], b[k]), k
    tol = 1e-5 if dtype == torch.float32 else 1e-12
    assert (param_error(g["p"], b["p"]) <= tol).all()
    assert (chi2_error(g["chi2"], b["chi2"]) <= tol).all()
    assert (g["outlier"] == 0).all()
    say("identical bits:", bool(np.array_equal(g["p"], b["p"]) and np.array_equal(g["C"], b["C"])))


def test_final_fit_ragged_sizes(ctx, kf):
    """Batches that end inside a wave and inside a block."""
    ev0 = planted(generate(workloads()["barrel10"], 700))
    for n in (1, 63, 65, 257, 700):
        ev = subset(ev0, np.arange(n))
        fwd = rounded_forward(oracle_fit(ev, torch.float64, 0), torch.float64)
        of = oracle_final(ev, torch.float64, fwd)
        g = gpu_final(ctx, kf, ev, torch.float64, fwd, prefill=9)
        assert np.array_equal(g["outlier"], of["outlier"]), n
        ep = param_error(g["p"], of["p"]).max(axis=1)
        assert (ep <= 1e-7).all(), (n, ep.max())
    say("ragged ok")


def test_tiny_cut_rejects_every_hit(ctx, kf):
    """The degenerate cut: every valid hit a refitted track reaches is
    rejected (a positive chi2 is above 1e-30), so the pass only carries the
    restart through the material: ndf = -5, chi2 = 0, the mask equals the
    valid entries, and the oracle agrees."""
    say("final fit, tiny cut")
    ev = generate(workloads()["barrel10"], 500)
    dt = torch.float64
    fwd = rounded_forward(oracle_fit(ev, dt, 0), dt)
    of = oracle_final(ev, dt, fwd, chi2_cut=1e-30)
    g = gpu_final(ctx, kf, ev, dt, fwd, chi2_cut=1e-30, prefill=5)
    refit = (of["status"] & O.NOT_REFITTED) == 0
    assert refit.mean() > 0.99
    assert (g["ndf"][refit] == -5).all() and (g["chi2"][refit] == 0).all()
    assert ((g["status"][refit] & O.OUTLIER) != 0).all()
    assert np.array_equal(g["outlier"], of["outlier"])
    ok_e = np.repeat(refit, ev.lengths())
    assert np.array_equal(g["outlier"][ok_e].astype(bool), (ev.hit_valid == 1)[ok_e])
    assert (param_error(g["p"], of["p"]).max(axis=1) <= 1e-8).all()
