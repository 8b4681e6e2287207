"""GPU parity of the backward fit (kf_backward_fit, through the C interface)
against the FP64 oracle.

1. The backward pass alone: both sides start from the oracle's forward fit
   result, rounded to the path's precision (no input of the oracle comes from
   the GPU).
2. The whole chain: seeding and forward fit in one launch, then the backward
   fit, against the oracle's seeding, forward fit and backward fit; at
   barrel20's full size in the launch shapes the benchmark times, and on a
   mixed26 sample (barrels, disks, holes).

Tolerances, the tail rule and the conditioning probes are those of the forward
fit (see tests/parity.py): a track whose oracle result moves by more than half
the tolerance when the hits are moved by one unit in the last place, or the
running state is rounded to FP32 (FP32 path) or jittered at the FP64 rounding
level (FP64 path), is left out of the comparison; such tracks must stay few.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import kf_oracle as O
from toygen import generate, subset, workloads

from parity import (BACKWARD_SCALE, backward_probes, compare_fit, gpu_backward, gpu_smooth,
                    oracle_backward, oracle_fit, oracle_forward_recorded, oracle_smooth, outputs_np,
                    param_error, per_entry, rounded, rounded_forward, smooth_errors)

pytestmark = pytest.mark.gpu

TOL32 = (1e-4, 1e-3)
TOL64 = (1e-8, 1e-8)


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


def _backward_only(c, kf, ev, dtype, seed_mode, tol, max_bad_frac, tail_frac):
    fwd = rounded_forward(oracle_fit(ev, dtype, seed_mode), dtype)
    ob = oracle_backward(ev, dtype, fwd)
    bad = backward_probes(ev, dtype, lambda **kw: oracle_backward(ev, dtype, fwd, **kw), ob, tol)
    assert bad.mean() <= max(max_bad_frac, 0.005), bad.mean()
    gb = gpu_backward(c, kf, ev, dtype, fwd)
    s = compare_fit(gb, ob, tol[0], tol[1], ~bad, tail_frac=tail_frac, geom=ev.geometry)
    s["ill_conditioned"] = int(bad.sum())
    say(s)
    return gb, ob


@pytest.mark.parametrize("name,n,mode,dtype", [("barrel10", None, 0, torch.float64), ("barrel10", None, 0, torch.float32),
                                               ("barrel20", 5000, 0, torch.float32),
                                               ("mixed26", 5000, 1, torch.float64),
                                               ("mixed26", 5000, 1, torch.float32)])
def test_backward_pass_parity(ctx, kf, name, n, mode, dtype):
    say("backward only", name, n, dtype)
    ev = generate(workloads()[name], n)
    fp32 = dtype == torch.float32
    gb, ob = _backward_only(ctx, kf, ev, dtype, mode, TOL32 if fp32 else TOL64, 0.04 if fp32 else 0.0,
                            0.005 if fp32 else 0.0)
    refit = (ob["status"] & O.NOT_REFITTED) == 0
    assert refit.mean() > 0.99
    assert np.isfinite(gb["p"]).all() and np.isfinite(gb["C"]).all()


def _chain(c, kf, ev, dtype, seed_mode):
    """GPU: seeding and forward fit in one launch, then the backward fit."""
    dev = c.device
    t = kf.event_tensors(ev, dtype, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    fwd = c.seed_fit_tracks(t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom,
                            seed_mode)
    out = c.backward_fit(fwd, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom,
                         cov_scale=BACKWARD_SCALE)
    torch.cuda.synchronize()
    return outputs_np(out)


def _oracle_chain(ev, dtype, seed_mode, hit_pos=None, state_round=None, state_jitter=None):
    o = oracle_fit(ev, dtype, seed_mode, hit_pos=hit_pos, state_round=state_round, state_jitter=state_jitter)
    return oracle_backward(ev, dtype, dict(p=o["p"], C=o["C"], q=o["q"], status=o["status"]), hit_pos=hit_pos,
                           state_round=state_round, state_jitter=state_jitter)


def _chain_case(c, kf, ev, dtype, seed_mode, tol, max_bad_frac, tail_frac):
    ob = _oracle_chain(ev, dtype, seed_mode)
    bad = backward_probes(ev, dtype, lambda **kw: _oracle_chain(ev, dtype, seed_mode, **kw), ob, tol)
    assert bad.mean() <= max(max_bad_frac, 0.005), bad.mean()
    gb = _chain(c, kf, ev, dtype, seed_mode)
    s = compare_fit(gb, ob, tol[0], tol[1], ~bad, tail_frac=tail_frac, geom=ev.geometry)
    s["ill_conditioned"] = int(bad.sum())
    s["launch"] = c.get_fit_launch(dtype)
    say(s)


def test_chain_barrel20_full_size(ctx, kf):
    """100,000 tracks x 20 layers: the benchmark's forward launch shapes, then
    the backward fit, in FP32 and FP64."""
    say("chain barrel20 100k")
    ev = generate(workloads()["barrel20"])
    _chain_case(ctx, kf, ev, torch.float32, 0, TOL32, 0.02, 0.002)
    _chain_case(ctx, kf, ev, torch.float64, 0, TOL64, 0.0, 1e-4)


def test_chain_mixed26_sample(ctx, kf):
    say("chain mixed26 20k")
    ev = generate(workloads()["mixed26"], 20_000)
    _chain_case(ctx, kf, ev, torch.float32, 1, TOL32, 0.05, 0.005)
    _chain_case(ctx, kf, ev, torch.float64, 1, TOL64, 0.0, 0.0)


def test_not_refitted_tracks_keep_their_input(ctx, kf):
    """Tracks the forward fit stopped (any of its stop bits) come back
    unchanged with KF_TRK_BAD_INPUT, chi2 0 and ndf -5; the others are
    unaffected by them.  Without a status every track is refitted."""
    say("backward stopped tracks")
    ev = generate(workloads()["mixed26"], 300)
    for dt in (torch.float32, torch.float64):
        fwd = rounded_forward(oracle_fit(ev, dt, 1), dt)
        base = gpu_backward(ctx, kf, ev, dt, fwd)
        st = fwd["status"].copy()
        stop = {3: O.NO_CROSSING, 40: O.NONFINITE, 41: O.NOT_REFITTED, 299: O.NO_CROSSING | O.GRAZING}
        for t, b in stop.items():
            st[t] |= b
        g = gpu_backward(ctx, kf, ev, dt, dict(fwd, status=st))
        for t in stop:
            assert g["status"][t] == O.NOT_REFITTED
            assert np.array_equal(g["p"][t], fwd["p"][t].astype(np.float32 if dt == torch.float32 else np.float64))
            assert g["chi2"][t] == 0 and g["ndf"][t] == -5
        others = np.setdiff1d(np.arange(ev.n_tracks), list(stop))
        for k in ("p", "C", "chi2", "ndf", "status", "q"):
            assert np.array_equal(g[k][others], base[k][others]), k
        o = oracle_backward(ev, dt, dict(fwd, status=st))
        assert np.array_equal(g["status"][list(stop)], o["status"][list(stop)])
        nost = gpu_backward(ctx, kf, ev, dt, dict(fwd, status=st), use_status=False)
        assert np.array_equal(nost["p"][others], base["p"][others])
        assert (nost["status"][list(stop)] & O.NOT_REFITTED).sum() == 0


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1000 + 13])
def test_backward_ragged_sizes(ctx, kf, n):
    say("backward n =", n)
    ev = generate(workloads()["mixed26"], max(n, 1))
    if n == 0:
        ev = subset(ev, [])
    dt = torch.float32
    fwd = rounded_forward(oracle_fit(ev, dt, 1), dt) if n else dict(p=np.zeros((0, 6)), C=np.zeros((0, 6, 6)),
                                                                 q=np.zeros(0), status=np.zeros(0, np.int64))
    g = gpu_backward(ctx, kf, ev, dt, fwd)
    assert g["chi2"].shape == (n,)
    if n:
        o = oracle_backward(ev, dt, fwd)
        bad = backward_probes(ev, dt, lambda **kw: oracle_backward(ev, dt, fwd, **kw), o, TOL32)
        compare_fit(g, o, TOL32[0], TOL32[1], ~bad, tail_frac=0.01, geom=ev.geometry)


def test_backward_is_deterministic(ctx, kf):
    ev = generate(workloads()["barrel20"], 3000)
    for dt in (torch.float32, torch.float64):
        fwd = rounded_forward(oracle_fit(ev, dt, 0), dt)
        a = gpu_backward(ctx, kf, ev, dt, fwd)
        b = gpu_backward(ctx, kf, ev, dt, fwd)
        for k in a:
            assert np.array_equal(a[k], b[k]), k


# ---- smoothing -----------------------------------------------------------------------

def _smooth_case(c, kf, ev, dtype, seed_mode, tol, max_bad_frac, tail_frac):
    rec = oracle_forward_recorded(ev, dtype, seed_mode)
    o = oracle_smooth(ev, dtype, rec)
    ops = o["ps"].numpy()
    # conditioning probes on the smoothed states
    rng = np.random.default_rng(7)
    hp = rounded(ev.hit_pos, dtype)
    if dtype == torch.float32:
        ulp = np.spacing(np.abs(hp).astype(np.float32)).astype(np.float64)
        probes = [dict(hit_pos=hp + ulp * rng.choice([-1.0, 1.0], size=hp.shape)), dict(state_round=torch.float32)]
    else:
        probes = [dict(hit_pos=hp + 1e-13 * np.maximum(np.abs(hp), 1.0) * rng.choice([-1.0, 1.0], size=hp.shape)),
                  dict(state_jitter=4e-16)]
    bad = np.zeros(ev.n_tracks, bool)
    for kw in probes:
        rec2 = oracle_forward_recorded(ev, dtype, seed_mode, **kw)
        o2 = oracle_smooth(ev, dtype, rec2, **kw)
        bad |= smooth_errors(ev, o2["ps"].numpy(), ops) > 0.5 * tol[0]
        bad |= param_error(o2["p"].numpy(), o["p"].numpy()).max(axis=1) > 0.5 * tol[0]
        bad |= o2["status"].numpy() != o["status"].numpy()
    assert bad.mean() <= max(max_bad_frac, 0.005), bad.mean()
    g, gstate, gcov = gpu_smooth(c, kf, ev, dtype, rec)
    ob = dict(p=o["p"].numpy(), C=o["C"].numpy(), q=o["q"].numpy(), chi2=o["chi2"].numpy(), ndf=o["ndf"].numpy(),
              status=o["status"].numpy())
    s = compare_fit(g, ob, tol[0], tol[1], ~bad, tail_frac=tail_frac, geom=ev.geometry)
    gps = per_entry(ev, gstate)
    ok_e = np.repeat(~bad, ev.lengths())
    # the same entries are smoothed
    assert np.array_equal(np.isnan(gps[ok_e]).any(axis=1), np.isnan(ops[ok_e]).any(axis=1))
    have = ok_e & ~np.isnan(ops).any(axis=1)
    ep = param_error(gps[have], ops[have]).max(axis=1)
    over = ep > tol[0]
    assert over.mean() <= max(tail_frac, 0.0) + 1e-12 and (ep <= 10 * tol[0]).all(), (ep.max(), over.sum())
    # covariance on the surface (5 coordinates), in correlation units
    e = np.nonzero(have)[0]
    gC = np.stack([sym_unpack_from_packed(per_entry(ev, gcov)[e])])[0]
    kind = torch.tensor(ev.geometry.kind[ev.hit_layer[e]], dtype=torch.int64)
    pos = torch.tensor(ev.geometry.pos[ev.hit_layer[e]], dtype=torch.float64)
    B = O.surface_frame(torch.tensor(ops[e]), kind, pos).numpy()
    Bt = B.transpose(0, 2, 1)
    g5, o5 = Bt @ gC @ B, Bt @ o["Cs"].numpy()[e] @ B
    d = np.sqrt(np.abs(np.einsum("naa->na", o5)))
    rel = (np.abs(g5 - o5) / (d[:, :, None] * d[:, None, :])).max(axis=(1, 2))
    if dtype == torch.float64:
        assert (rel <= 10 * tol[0]).all() and (rel > tol[0]).mean() <= max(tail_frac, 0.0) + 1e-12, rel.max()
    else:
        # FP32 covariances carry fewer digits than FP32 states: the backward
        # pass restarts from a covariance scaled by 100, and its first updates
        # shrink it back by that factor, in FP32; the smoothed covariance one
        # layer before the last takes most of its theta block from there
        # (measured: median 4e-6, 99% 8e-4, worst entries a few % in
        # correlation units, the smoothed states unaffected)
        assert (rel <= 0.5).all() and (rel > 1e-2).mean() <= 2e-3, (rel.max(), (rel > 1e-2).mean())
    s.update(smoothed_entries=int(have.sum()), max_smoothed_err=float(ep.max(initial=0)),
             max_smoothed_cov_err=float(rel.max(initial=0)), ill_conditioned=int(bad.sum()))
    say(s)


def sym_unpack_from_packed(P):
    """[N, 21] packed -> [N, 6, 6]."""
    M = np.zeros((P.shape[0], 6, 6))
    k = 0
    for i in range(6):
        for j in range(i + 1):
            M[:, i, j] = M[:, j, i] = P[:, k]
            k += 1
    return M


@pytest.mark.parametrize("name,n,mode,dtype", [("barrel10", None, 0, torch.float64), ("barrel10", None, 0, torch.float32),
                                               ("mixed26", 3000, 1, torch.float64),
                                               ("mixed26", 3000, 1, torch.float32)])
def test_smoothing_parity(ctx, kf, name, n, mode, dtype):
    say("smoothing", name, n, dtype)
    ev = generate(workloads()[name], n)
    fp32 = dtype == torch.float32
    _smooth_case(ctx, kf, ev, dtype, mode, TOL32 if fp32 else TOL64, 0.05 if fp32 else 0.0, 0.005 if fp32 else 0.0)


def test_smoothing_barrel20_full_size(ctx, kf):
    """100,000 FP32 tracks x 20 layers, the benchmark's workload."""
    say("smoothing barrel20 100k fp32")
    ev = generate(workloads()["barrel20"])
    _smooth_case(ctx, kf, ev, torch.float32, 0, TOL32, 0.02, 0.002)
