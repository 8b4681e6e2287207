"""GPU parity of seeding, single-step propagate/update and the fused fit
(through the C interface) against the FP64 oracle on the same seeded inputs."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import kf_oracle as O
from toygen import generate, subset, truncate, workloads

from parity import (chi2_error, compare_fit, cov_rel_error, gpu_fit, ill_conditioned, oracle_fit, param_error,
                    rounded, sym_unpack, tangent_frame_cov)

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
    """Context with the workspace, set to the sorted and packed layout."""
    c = kf.Context(0)
    c.reserve(600_000, 26)
    for dt in (torch.float32, torch.float64):
        c.set_fit_launch(dt, 256, 0, 1, 1, 2)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_staged(kf):
    """Context set to CSR in track order staged through LDS by each wave, in
    the launch shapes the benchmark's tuner picks for barrel20."""
    c = kf.Context(0)
    c.set_fit_launch(torch.float32, 256, 0, 1, 2, 3)
    c.set_fit_launch(torch.float64, 256, 0, 1, 1, 3)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_staged_sorted(kf):
    """Context with the workspace, set to length-sorted CSR staged through LDS."""
    c = kf.Context(0)
    c.reserve(600_000, 26)
    c.set_fit_launch(torch.float32, 128, 1, 4, 2, 4)
    c.set_fit_launch(torch.float64, 256, 0, 1, 1, 4)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ctx_csr(kf):
    """Context without a workspace: the fit reads the CSR arrays directly."""
    c = kf.Context(0)
    yield c
    c.close()


# ---- seeding -------------------------------------------------------------------

@pytest.mark.parametrize("name,mode,dtype", [("barrel10", 0, torch.float64), ("barrel20", 0, torch.float32),
                                             ("mixed26", 1, torch.float32), ("mixed26", 1, torch.float64)])
def test_seeds_parity(ctx, kf, name, mode, dtype):
    say("seeds", name, mode, dtype)
    ev = generate(workloads()[name], 3000)
    t = kf.event_tensors(ev, dtype, ctx.device)
    st, cov, q, status = ctx.make_seeds(t["hit_offsets"], t["hit_valid"], t["hit_pos"], ev.geometry.bz, mode)
    hp = rounded(ev.hit_pos, dtype)
    sp, sC, sq, ok = O.make_seeds(ev.hit_offsets, ev.hit_valid, hp, ev.geometry.bz, mode=mode)
    g = st.double().cpu().numpy().T
    err = param_error(g, sp.numpy()).max(axis=1)
    tol = 1e-4 if dtype == torch.float32 else 1e-10
    # ill-conditioned three-point circles (nearly collinear hits) are excluded by the
    # oracle's own sensitivity to an FP32-ulp change of the hits
    rel = 2.0 ** -23 if dtype == torch.float32 else 1e-13
    sp2, _, _, _ = O.make_seeds(ev.hit_offsets, ev.hit_valid, hp * (1 + rel), ev.geometry.bz, mode=mode)
    cond = param_error(sp2.numpy(), sp.numpy()).max(axis=1) < 0.5 * tol
    assert cond.mean() > 0.99
    assert err[cond].max() < tol, err[cond].max()
    assert np.array_equal(q.cpu().numpy()[cond].astype(float), sq.numpy()[cond])
    assert (status.cpu().numpy()[ok.numpy()] == 0).all()
    C = cov.double().cpu().numpy().T
    assert np.allclose(sym_unpack(C), sC.numpy())


# ---- single steps ----------------------------------------------------------------

def _step_inputs(name, n_tracks, seed):
    """Generator truth at entry k (random k per track), a random SPD covariance
    and the layer of entry k+1 as target."""
    wl = workloads()[name]
    ev = generate(wl, n_tracks)
    rng = np.random.default_rng(seed)
    L = ev.lengths()
    k = rng.integers(0, L - 1)
    e = ev.hit_offsets[:-1] + k
    p = ev.truth_after[e].copy()
    A = rng.normal(size=(n_tracks, 6, 6)) * np.array([0.01, 0.01, 0.01, 0.01, 0.001, 0.001])[None, :, None]
    C = A @ A.transpose(0, 2, 1) + np.diag([1e-4, 1e-4, 1e-4, 1e-4, 1e-6, 1e-6])[None]
    return ev, p, C, ev.charge.astype(np.float64), ev.hit_layer[e + 1], ev.hit_layer[e], e + 1


def _pack(C):
    out = []
    for i in range(6):
        for j in range(i + 1):
            out.append(C[:, i, j])
    return np.stack(out)


@pytest.mark.parametrize("name,dtype", [("barrel20", torch.float32), ("mixed26", torch.float32),
                                        ("mixed26", torch.float64)])
def test_propagate_parity(ctx, kf, name, dtype):
    say("propagate", name, dtype)
    ev, p, C, q, target, frm, _ = _step_inputs(name, 5000, 5)
    p = rounded(p, dtype)
    C = rounded(C, dtype)
    dev = ctx.device
    geom = kf.Geometry.from_toy(ev.geometry)
    st = torch.tensor(p.T.copy(), dtype=dtype, device=dev)
    cv = torch.tensor(_pack(C), dtype=dtype, device=dev)
    ch = torch.tensor(q, dtype=torch.int8, device=dev)
    tg = torch.tensor(target, dtype=torch.int16, device=dev)
    fr = torch.tensor(frm, dtype=torch.int16, device=dev)
    so, co, path, status = ctx.propagate(st, cv, ch, tg, geom, from_layer=fr)
    torch.cuda.synchronize()
    g = ev.geometry
    kind = torch.tensor(g.kind[target].astype(np.int64))
    op, oC, os_, ostat = O.propagate(torch.tensor(p), torch.tensor(C), torch.tensor(q), kind,
                                     torch.tensor(g.pos[target]), torch.tensor(g.x_over_x0[target]), g,
                                     same=torch.tensor(target == frm))
    gp = so.double().cpu().numpy().T
    ok = ostat.numpy() & O.NO_CROSSING == 0
    tol = 1e-4 if dtype == torch.float32 else 1e-10
    err = param_error(gp, op.numpy()).max(axis=1)
    assert err[ok].max() < tol, err[ok].max()
    assert np.array_equal(status.cpu().numpy(), ostat.numpy())
    kind_t = g.kind[target]
    Cg = tangent_frame_cov(sym_unpack(co.double().cpu().numpy().T), op.numpy(), kind_t)
    Co = tangent_frame_cov(oC.numpy(), op.numpy(), kind_t)
    rel = cov_rel_error(Cg, Co)
    assert rel[ok].max() < (1e-3 if dtype == torch.float32 else 1e-9), rel[ok].max()
    pe = np.abs(path.double().cpu().numpy() - os_.numpy()) / np.maximum(np.abs(os_.numpy()), 1.0)
    assert pe[ok].max() < (1e-4 if dtype == torch.float32 else 1e-10)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_update_parity(ctx, kf, dtype):
    say("update", dtype)
    ev, p, C, q, target, frm, e = _step_inputs("barrel20", 5000, 7)
    # predicted state: truth plus a small offset, hit of that crossing
    rng = np.random.default_rng(8)
    p = p.copy()
    p[:, :2] += rng.normal(0, 0.01, (p.shape[0], 2))
    e = e - 1
    m = np.ascontiguousarray(ev.hit_pos[:, e])
    V = np.ascontiguousarray(ev.hit_cov[:, e])
    p, C, m, V = (np.ascontiguousarray(rounded(x, dtype)) for x in (p, C, m, V))
    dev = ctx.device
    st = torch.tensor(p.T.copy(), dtype=dtype, device=dev)
    cv = torch.tensor(_pack(C), dtype=dtype, device=dev)
    ch = torch.tensor(q, dtype=torch.int8, device=dev)
    hp = torch.tensor(m, dtype=dtype, device=dev)
    hc = torch.tensor(V, dtype=dtype, device=dev)
    chi2, status = ctx.update(st, cv, ch, hp, hc)
    torch.cuda.synchronize()
    op, oC, oq, oc2, ostat = O.update(torch.tensor(p), torch.tensor(C), torch.tensor(q), torch.tensor(m.T),
                                      O.unpack_sym(V, 3))
    tol = 1e-4 if dtype == torch.float32 else 1e-10
    assert param_error(st.double().cpu().numpy().T, op.numpy()).max() < tol
    assert chi2_error(chi2.double().cpu().numpy(), oc2.numpy()).max() < (1e-3 if dtype == torch.float32 else 1e-9)
    assert np.array_equal(ch.cpu().numpy().astype(float), oq.numpy())
    assert np.array_equal(status.cpu().numpy() & ~O.FP64_FALLBACK, ostat.numpy())
    # the updated covariance (a full-rank prior here), in correlation units:
    # the FP32 form is the expanded Joseph form C - K B^T - E K^T
    rel = cov_rel_error(sym_unpack(cv.double().cpu().numpy().T), oC.numpy())
    say("update cov err max", float(rel.max()), "p99.9", float(np.quantile(rel.reshape(len(rel), -1).max(1), 0.999)))
    assert rel.max() < (1e-3 if dtype == torch.float32 else 1e-9), rel.max()


def test_update_fp64_fallback(ctx, kf):
    """Updates whose prior position variance exceeds the hit variance by more
    than 1e4 (a diffuse prior) or whose residual covariance is nearly singular
    take the FP64 path in the FP32 kernel and still match the oracle."""
    say("fp64 fallback")
    n = 512
    rng = np.random.default_rng(3)
    ph = rng.uniform(-math.pi, math.pi, n)
    R = 30.0
    p = np.stack([R * np.cos(ph), R * np.sin(ph), rng.uniform(-10, 10, n), np.full(n, 0.5), ph, np.full(n, 1.2)], 1)
    t = np.stack([-np.sin(ph), np.cos(ph), np.zeros(n)], 1)
    z = np.tile([0.0, 0.0, 1.0], (n, 1))
    nh = np.stack([np.cos(ph), np.sin(ph), np.zeros(n)], 1)
    # half the lanes: diffuse prior (ratio ~1e5); half: a tight prior with a
    # nearly singular S (normal variance 4e-8 against 5e-2 in z: kappa > 1e6)
    diffuse = np.arange(n) < n // 2
    C = np.zeros((n, 6, 6))
    Cp_d = 1.0 * t[:, :, None] * t[:, None, :] + 1.0 * z[:, :, None] * z[:, None, :]
    Cp_t = 1e-2 * t[:, :, None] * t[:, None, :] + 5e-2 * z[:, :, None] * z[:, None, :]
    C[:, :3, :3] = np.where(diffuse[:, None, None], Cp_d, Cp_t)
    C[:, 3:, 3:] = np.diag([1e-3, 1e-4, 1e-4])
    C[:, 0:3, 4] = C[:, 4, 0:3] = 1e-4 * t     # position-angle correlation
    sn = np.where(diffuse, 0.03 / math.sqrt(12), 2e-4)
    V = (0.003 ** 2) * t[:, :, None] * t[:, None, :] + 0.01 ** 2 * z[:, :, None] * z[:, None, :] + \
        (sn ** 2)[:, None, None] * nh[:, :, None] * nh[:, None, :]
    m = p[:, :3] + 0.004 * t + 0.02 * z
    p, C, m, V = (np.ascontiguousarray(rounded(x, torch.float32)) for x in (p, C, m, V))
    Vp = np.ascontiguousarray(np.stack([V[:, 0, 0], V[:, 1, 0], V[:, 1, 1], V[:, 2, 0], V[:, 2, 1], V[:, 2, 2]]))
    dev = ctx.device
    st = torch.tensor(np.ascontiguousarray(p.T), dtype=torch.float32, device=dev)
    cv = torch.tensor(_pack(C), dtype=torch.float32, device=dev)
    ch = torch.ones(n, dtype=torch.int8, device=dev)
    chi2, status = ctx.update(st, cv, ch, torch.tensor(np.ascontiguousarray(m.T), dtype=torch.float32, device=dev),
                              torch.tensor(Vp, dtype=torch.float32, device=dev))
    torch.cuda.synchronize()
    stt = status.cpu().numpy()
    assert (stt & O.FP64_FALLBACK).all()
    op, oC, oq, oc2, ostat = O.update(torch.tensor(p), torch.tensor(C), torch.ones(n, dtype=torch.float64),
                                      torch.tensor(m), torch.tensor(V))
    assert param_error(st.double().cpu().numpy().T, op.numpy()).max() < 1e-4
    assert chi2_error(chi2.double().cpu().numpy(), oc2.numpy()).max() < 1e-3
    # covariance on the surface's five directions (the priors have the normal as a null vector)
    kind0 = np.zeros(n, int)
    rel = cov_rel_error(tangent_frame_cov(sym_unpack(cv.double().cpu().numpy().T), p, kind0),
                        tangent_frame_cov(oC.numpy(), p, kind0))
    # the diffuse-prior half runs the whole update in FP64; the nearly
    # singular half inverts S in FP64 but forms the gain and the covariance
    # in FP32, where a condition number ~1e6 costs ~kappa * eps32 ~ 0.1
    diffuse_half = np.arange(n) < n // 2
    say("fp64 lane cov err max", float(rel[diffuse_half].max()), "inverse-only lanes", float(rel[~diffuse_half].max()))
    assert rel[diffuse_half].max() < 1e-3, rel[diffuse_half].max()


# ---- the fused fit -------------------------------------------------------------------

def _fit_case(ctxs, kf, ev, dtype, seed_mode, tol, max_bad_frac=0.0, tail_frac=0.0):
    """Parity of the fit against the oracle for one context or several (the
    oracle runs once)."""
    ctxs = ctxs if isinstance(ctxs, (list, tuple)) else [ctxs]
    o = oracle_fit(ev, dtype, seed_mode)
    bad = ill_conditioned(ev, dtype, o, seed_mode, *tol)
    mask = ~bad
    assert bad.sum() <= max(max_bad_frac, 0.005) * ev.n_tracks, bad.mean()
    for c in ctxs:
        g = gpu_fit(c, kf, ev, dtype, seed_mode)
        s = compare_fit(g, o, tol[0], tol[1], mask, tail_frac=tail_frac, geom=ev.geometry)
        s["ill_conditioned"] = int((~mask).sum())
        s["launch"] = c.get_fit_launch(dtype)
        say(s)
    return g, o, s


def test_fit_barrel10_fp64_all_tracks(ctx, ctx_staged, kf):
    say("fit barrel10 fp64")
    ev = generate(workloads()["barrel10"])
    _fit_case([ctx, ctx_staged], kf, ev, torch.float64, 0, TOL64)


def test_fit_barrel10_fp32(ctx, ctx_staged, kf):
    say("fit barrel10 fp32")
    ev = generate(workloads()["barrel10"])
    _fit_case([ctx, ctx_staged], kf, ev, torch.float32, 0, TOL32, max_bad_frac=0.03, tail_frac=0.003)


def test_fit_barrel20_full_size_fp32_and_fp64(ctx, ctx_staged, kf):
    """100,000 tracks x 20 layers, in the packed layout and in the staged
    layout and launch shape the benchmark times."""
    say("fit barrel20 100k fp32 + fp64")
    ev = generate(workloads()["barrel20"])
    _fit_case([ctx, ctx_staged], kf, ev, torch.float32, 0, TOL32, max_bad_frac=0.01, tail_frac=0.001)
    # at 100k tracks the FP64 jitter probe misses the odd track whose chi2
    # differs by slightly more than 1e-8 (the rounding order of the two
    # implementations differs)
    _fit_case([ctx, ctx_staged], kf, ev, torch.float64, 0, TOL64, tail_frac=1e-4)


def test_fit_mixed26_sample(ctx, ctx_staged_sorted, kf):
    say("fit mixed26 20k fp32 + fp64")
    ev = generate(workloads()["mixed26"], 20_000)
    _fit_case([ctx, ctx_staged_sorted], kf, ev, torch.float32, 1, TOL32, max_bad_frac=0.04, tail_frac=0.005)
    _fit_case([ctx, ctx_staged_sorted], kf, ev, torch.float64, 1, TOL64)


def _sampled_full_size(c, kf, ev, dtype, seed_mode, tol, sample, max_bad_frac, tail_frac, launch):
    """The whole batch through the GPU in the given launch shape (seeding and
    fit in one launch, as the benchmark times it); the oracle on a sample of
    its tracks (each track's result depends on its own hits only)."""
    dev = c.device
    old = c.get_fit_launch(dtype)
    c.set_fit_launch(dtype, *launch)
    try:
        t = kf.event_tensors(ev, dtype, dev)
        geom = kf.Geometry.from_toy(ev.geometry)
        out = c.seed_fit_tracks(t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom,
                                seed_mode)
        torch.cuda.synchronize()
    finally:
        c.set_fit_launch(dtype, *old)
    pick = np.sort(np.random.default_rng(5).choice(ev.n_tracks, sample, replace=False))
    sub = subset(ev, pick)
    tp = torch.as_tensor(pick, device=dev)
    g = dict(p=out["state"][:, tp].double().cpu().numpy().T, C=out["cov"][:, tp].double().cpu().numpy().T,
             q=out["charge"][tp].cpu().numpy().astype(np.float64), chi2=out["chi2"][tp].double().cpu().numpy(),
             ndf=out["ndf"][tp].cpu().numpy(), status=out["status"][tp].cpu().numpy().astype(np.int64))
    o = oracle_fit(sub, dtype, seed_mode)
    bad = ill_conditioned(sub, dtype, o, seed_mode, *tol)
    assert bad.mean() <= max_bad_frac, bad.mean()
    # tracks without three usable hits: flagged on the GPU, not compared.
    # A spaced choice whose distances lie within FP32 rounding of the 2.5 cm
    # spacing can go either way in FP32 (both choices are valid): such
    # tracks are left out like the ill-conditioned ones
    hp_r = rounded(sub.hit_pos, dtype)
    _, _, _, seeded = O.make_seeds(sub.hit_offsets, sub.hit_valid, hp_r, ev.geometry.bz, mode=seed_mode)
    seeded = seeded.numpy().astype(bool)
    either = np.zeros(sub.n_tracks, bool)
    if seed_mode == 1:
        _, margin = O.spaced_three_valid(sub.hit_offsets, sub.hit_valid, hp_r, return_margin=True)
        either = margin.numpy() < (1e-5 if dtype == torch.float32 else 1e-12)
    gbad = (g["status"] & kf.TRK_BAD_INPUT) != 0
    assert np.array_equal(gbad[~either], ~seeded[~either]), np.nonzero((gbad != ~seeded) & ~either)[0][:10]
    s = compare_fit(g, o, tol[0], tol[1], ~bad & seeded & ~either, tail_frac=tail_frac, geom=ev.geometry)
    s["ill_conditioned"] = int(bad.sum())
    s["not_seeded"] = int((~seeded).sum())
    s["seed_spacing_either_way"] = int(either.sum())
    say(s)
    return out


def test_fit_mixed26_full_size(ctx_staged_sorted, kf):
    """The uneven-length workload at its full size (500,000 tracks, 10 barrel
    layers and 2 x 8 disks, 5% holes), in the launch shape the benchmark's
    tuner picks for it (length-sorted CSR staged through LDS), FP32 and FP64,
    the oracle on 5,000 sampled tracks; then the same batch with every track
    cut to a random length in 3..26, so that the short tracks run at full size
    too."""
    say("fit mixed26 full size (500k), oracle on 5k sampled tracks")
    ev = generate(workloads()["mixed26"])
    assert ev.n_tracks == 500_000
    _sampled_full_size(ctx_staged_sorted, kf, ev, torch.float32, 1, TOL32, 5000, 0.04, 0.005, (256, 0, 1, 2, 4))
    _sampled_full_size(ctx_staged_sorted, kf, ev, torch.float64, 1, TOL64, 5000, 0.005, 1e-3, (256, 0, 1, 1, 4))
    lens = np.random.default_rng(9).integers(3, 27, ev.n_tracks)
    ev3 = truncate(ev, np.minimum(lens, ev.lengths()))
    nval = np.add.reduceat(ev3.hit_valid.astype(np.int64), ev3.hit_offsets[:-1])
    say("truncated: lengths", int(ev3.lengths().min()), "..", int(ev3.lengths().max()),
        "tracks with < 3 valid hits", int((nval < 3).sum()))
    out = _sampled_full_size(ctx_staged_sorted, kf, ev3, torch.float32, 1, TOL32, 5000, 0.06, 0.01,
                             (256, 0, 1, 2, 4))
    st = out["status"].cpu().numpy()
    assert ((st & kf.TRK_BAD_INPUT) != 0)[nval < 3].all()


def test_fit_every_length_3_to_26(ctx, kf):
    say("fit lengths 3..26")
    ev = generate(workloads()["mixed26"], 4000)
    long = np.nonzero(ev.lengths() >= 26)[0]
    assert long.size >= 24
    lengths = np.arange(3, 27)
    pick = np.repeat(long[:24], 1)
    ev2 = truncate(subset(ev, pick), lengths)
    keep = np.add.reduceat(ev2.hit_valid.astype(int), ev2.hit_offsets[:-1]) >= 3
    ev2 = subset(ev2, np.nonzero(keep)[0])
    _fit_case(ctx, kf, ev2, torch.float64, 1, TOL64)
    _fit_case(ctx, kf, ev2, torch.float32, 1, TOL32, max_bad_frac=0.1, tail_frac=0.05)


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, 1000 + 13])
def test_fit_ragged_sizes(ctx, ctx_csr, ctx_staged, ctx_staged_sorted, kf, n):
    say("fit ragged", n)
    ev = generate(workloads()["mixed26"], max(n, 1))
    if n == 0:
        ev = subset(ev, [])
    for c in (ctx, ctx_csr, ctx_staged, ctx_staged_sorted):
        _fit_case(c, kf, ev, torch.float64, 1, TOL64)


def test_fit_max_len_truncates_and_flags(ctx, ctx_csr, ctx_staged, ctx_staged_sorted, kf):
    """Entries beyond max_len are ignored (every layout) and the track is flagged."""
    say("fit max_len")
    ev = generate(workloads()["mixed26"], 500)
    for c in (ctx, ctx_csr, ctx_staged, ctx_staged_sorted):
        g = gpu_fit(c, kf, ev, torch.float64, 1, max_len=12)
        o = oracle_fit(truncate(ev, np.full(ev.n_tracks, 12)), torch.float64, 1)
        long_ = ev.lengths() > 12
        assert ((g["status"][long_] & kf.TRK_BAD_INPUT) != 0).all()
        assert ((g["status"][~long_] & kf.TRK_BAD_INPUT) == 0).all()
        g["status"] = g["status"] & ~kf.TRK_BAD_INPUT
        # seeds: the oracle seeds from the truncated track, the GPU from the full one
        ok = np.ones(ev.n_tracks, bool)
        sp_full = g["seed"]
        ok &= param_error(sp_full, o["seed"]).max(axis=1) < 1e-12
        compare_fit(g, o, TOL64[0], TOL64[1], ok, geom=ev.geometry)


@pytest.mark.parametrize("which", ["ctx", "ctx_staged", "ctx_staged_sorted"])
def test_fit_edge_cases(which, request, kf):
    """Holes in front of the first valid hit, a track with no valid hit, an
    unreachable layer and a non-finite hit, all in one batch."""
    say("fit edge cases", which)
    ctx = request.getfixturevalue(which)
    wl = workloads()["barrel10"]
    ev = generate(wl, 200)
    valid = ev.hit_valid.copy()
    off = ev.hit_offsets
    valid[off[0]] = 0              # track 0: leading hole
    valid[off[1]:off[1] + 2] = 0   # track 1: two leading holes
    valid[off[2]:off[3]] = 0       # track 2: no valid hit at all
    pos = ev.hit_pos.copy()
    pos[:, off[4] + 5] = np.nan    # track 4: non-finite hit at entry 5
    ev.hit_valid = valid
    ev.hit_pos = pos
    from toygen import barrel_geometry
    g2 = barrel_geometry(list(wl.geometry.pos[:-1]) + [5000.0])   # last layer unreachable
    ev.geometry = g2
    dt = torch.float64
    gres = gpu_fit(ctx, kf, ev, dt, 0)
    assert gres["status"][2] & kf.TRK_BAD_INPUT
    assert np.isfinite(gres["p"]).all() and np.isfinite(gres["chi2"]).all()
    assert gres["status"][4] & O.NONFINITE
    # compare every track the oracle can seed (track 2 cannot be seeded)
    o = oracle_fit(ev, dt, 0)
    mask = np.ones(ev.n_tracks, bool)
    mask[2] = False
    compare_fit(gres, o, TOL64[0], TOL64[1], mask, geom=ev.geometry)
    full = ev.lengths() == 10
    full[[2, 4]] = False          # no seed / frozen before the last layer
    assert ((gres["status"][full] & O.NO_CROSSING) != 0).all()


def test_fit_deterministic_and_launch_shape_independent(ctx, ctx_csr, kf):
    """Bit-identical on a repeat and across launch shapes within each family
    of hit layouts: direct reads (0 to 2) and staging through LDS (3, 4).  The
    two families inline the same arithmetic into different loops, so the
    compiler fuses different multiply-adds: across them results agree to
    rounding, and each family meets the oracle tolerances on its own (the
    parity tests run both)."""
    say("fit determinism")
    ev = generate(workloads()["mixed26"], 20_000)
    a = gpu_fit(ctx, kf, ev, torch.float32, 1)
    b = gpu_fit(ctx, kf, ev, torch.float32, 1)
    e = gpu_fit(ctx_csr, kf, ev, torch.float32, 1)     # CSR layout, same arithmetic
    assert np.array_equal(a["p"], e["p"]) and np.array_equal(a["chi2"], e["chi2"])
    old = ctx.get_fit_launch(torch.float32)
    try:
        ctx.set_fit_launch(torch.float32, 64, 1, 8, 2, 2)
        c = gpu_fit(ctx, kf, ev, torch.float32, 1)
        ctx.set_fit_launch(torch.float32, 128, 0, 1, 1, 1)
        d = gpu_fit(ctx, kf, ev, torch.float32, 1)
        ctx.set_fit_launch(torch.float32, 256, 1, 4, 1, 0)
        f = gpu_fit(ctx, kf, ev, torch.float32, 1)
        ctx.set_fit_launch(torch.float32, 256, 0, 1, 2, 3)
        h = gpu_fit(ctx, kf, ev, torch.float32, 1)
        ctx.set_fit_launch(torch.float32, 64, 1, 8, 1, 4)
        i = gpu_fit(ctx, kf, ev, torch.float32, 1)
        ctx.set_fit_launch(torch.float32, 192, 0, 1, 1, 4)
        j = gpu_fit(ctx, kf, ev, torch.float32, 1)
    finally:
        ctx.set_fit_launch(torch.float32, *old)
    for x in (b, c, d, f):
        assert np.array_equal(a["p"], x["p"]) and np.array_equal(a["C"], x["C"])
        assert np.array_equal(a["chi2"], x["chi2"]) and np.array_equal(a["status"], x["status"])
    for x in (i, j):
        assert np.array_equal(h["p"], x["p"]) and np.array_equal(h["C"], x["C"])
        assert np.array_equal(h["chi2"], x["chi2"]) and np.array_equal(h["status"], x["status"])


def test_fit_alignment_parity(ctx, kf):
    say("fit with alignment")
    wl = workloads()["align20"]
    ev = generate(wl, 3000)
    al = ev.align_true
    for dt, tol in ((torch.float64, TOL64), (torch.float32, TOL32)):
        g = gpu_fit(ctx, kf, ev, dt, 0, align=al)
        o = oracle_fit(ev, dt, 0, align=al)
        mask = ~ill_conditioned(ev, dt, o, 0, *tol, align=al)
        say(compare_fit(g, o, tol[0], tol[1], mask, tail_frac=0.002 if dt == torch.float32 else 0.0, geom=ev.geometry))


def test_fit_kernel_timing_counts_launches_and_keeps_results(kf):
    """kf_set_kernel_timing records one event pair per fit call (graph replay
    is bypassed while it is on), drops the calls past the last pair, and
    changes no result."""
    say("fit kernel timing")
    ev = generate(workloads()["barrel20"], 20_000)
    dev = torch.device("cuda", 0)
    t = kf.event_tensors(ev, torch.float32, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    c = kf.Context(0)
    try:
        c.reserve(ev.n_tracks, 20)
        c.set_fit_launch(torch.float32, 256, 0, 1, 1, 2)
        st, cov, q, _ = c.make_seeds(t["hit_offsets"], t["hit_valid"], t["hit_pos"], ev.geometry.bz, 0)
        args = (st, cov, q, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom)
        ref = {k: v.clone() for k, v in c.fit_tracks(*args).items()}
        c.set_fit_graph(True)
        c.set_kernel_timing(3)
        out = kf.fit_outputs(ev.n_tracks, torch.float32, dev)
        for _ in range(5):
            c.fit_tracks(*args, out=out)
        ms, n, dropped = c.fit_kernel_time()
        assert (n, dropped) == (3, 2)
        assert 0.0 < ms < 1000.0
        for k in ref:
            assert torch.equal(ref[k], out[k]), k
        c.fit_tracks(*args, out=out)
        assert c.fit_kernel_time()[1:] == (1, 0)   # the count starts again
        c.set_kernel_timing(0)
        c.fit_tracks(*args, out=out)               # graph replay again
        assert c.fit_kernel_time() == (0.0, 0, 0)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(ref[k], out[k]), k
    finally:
        c.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_fit_layouts_agree_on_irregular_entries(kf, dtype):
    """Inputs that exercise the staging: runs of leading holes longer than a
    staged chunk, tracks with no valid entry, a non-finite hit, an
    out-of-range layer mid-track, max_len truncation, a batch that ends inside
    a wave.  Within each layout family every launch shape gives the same bits;
    across the families, in FP64, the decisions (status, ndf, charge) are the
    same and the values agree to rounding.  Seeds come from the unmodified tracks so
    that the fits run."""
    say("fit layouts agree", dtype)
    ev = generate(workloads()["mixed26"], 3000 + 37)
    dev = torch.device("cuda", 0)
    t0 = kf.event_tensors(ev, dtype, dev)
    c = kf.Context(0)
    try:
        c.reserve(ev.n_tracks, 26)
        st, cov, q, _ = c.make_seeds(t0["hit_offsets"], t0["hit_valid"], t0["hit_pos"], ev.geometry.bz, 1)
        valid = ev.hit_valid.copy()
        layer = ev.hit_layer.copy()
        pos = ev.hit_pos.copy()
        off = ev.hit_offsets
        lens = ev.lengths()
        rng = np.random.default_rng(11)
        long_ = np.nonzero(lens >= 20)[0]
        for tr in rng.choice(long_, 40, replace=False):
            valid[off[tr]:off[tr] + int(rng.integers(1, 15))] = 0   # up to 14 leading holes
        for tr in rng.choice(ev.n_tracks, 10, replace=False):
            valid[off[tr]:off[tr + 1]] = 0                          # no valid entry
        for tr in rng.choice(ev.n_tracks, 10, replace=False):
            pos[:, off[tr] + int(rng.integers(0, lens[tr]))] = np.nan
        for tr in rng.choice(ev.n_tracks, 10, replace=False):
            layer[off[tr] + int(rng.integers(0, lens[tr]))] = 99   # no such layer
        ev.hit_valid, ev.hit_layer, ev.hit_pos = valid, layer, pos
        t = kf.event_tensors(ev, dtype, dev)
        geom = kf.Geometry.from_toy(ev.geometry)
        families = [[(256, 0, 1, 1, 0), (128, 1, 4, 2, 1), (256, 0, 1, 1, 2)],
                    [(256, 0, 1, 2, 3), (64, 1, 8, 1, 3), (192, 0, 1, 1, 4), (128, 1, 4, 2, 4)]]
        for max_len in (26, 17):
            refs = []
            for fam in families:
                res = {}
                for shape in fam:
                    c.set_fit_launch(dtype, *shape)
                    out = c.fit_tracks(st, cov, q, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"],
                                       t["hit_cov"], geom, max_len=max_len)
                    torch.cuda.synchronize()
                    res[shape] = {k: v.cpu().numpy() for k, v in out.items()}
                ref = res[fam[0]]
                st_ = ref["status"]
                assert (st_ & kf.TRK_BAD_INPUT).sum() >= 20 and (st_ & O.NONFINITE).any()
                for shape, r in res.items():
                    for k in ref:
                        a_, b_ = ref[k], r[k]
                        assert np.array_equal(a_, b_, equal_nan=a_.dtype.kind == "f"), (max_len, shape, k)
                refs.append(ref)
            # across the two families (FP64): the same decisions, values
            # equal to rounding.  In FP32 a rounding difference can move a
            # marginal decision (the FP64 lane switch, a PSD flag), so there
            # each family is held to the oracle by the parity tests instead.
            if dtype == torch.float64:
                x, y = refs
                for k in ("status", "ndf", "charge"):
                    assert np.array_equal(x[k], y[k]), (max_len, k)
                for k in ("state", "cov", "chi2"):
                    assert np.allclose(x[k], y[k], rtol=1e-9, atol=1e-12, equal_nan=True), (max_len, k)
    finally:
        c.close()


@pytest.mark.parametrize("name,mode,dtype", [("barrel20", 0, torch.float32), ("mixed26", 1, torch.float32),
                                             ("mixed26", 1, torch.float64)])
def test_seed_fit_matches_seeding_then_fit(kf, name, mode, dtype):
    """kf_seed_fit_tracks gives the bits of kf_make_seeds followed by
    kf_fit_tracks, in both layout families, with and without checkpoints and
    under graph replay: the same fit outputs, the same seeds written out, and
    the status of the two calls or-ed.  Some tracks keep a single valid hit
    (no seed: KF_TRK_BAD_INPUT from the seeding)."""
    say("seed + fit", name, mode, dtype)
    ev = generate(workloads()[name], 4000 + 17)
    valid = ev.hit_valid.copy()
    off = ev.hit_offsets
    for tr in range(0, 80, 8):
        valid[off[tr] + 1:off[tr + 1]] = 0
    ev.hit_valid = valid
    dev = torch.device("cuda", 0)
    t = kf.event_tensors(ev, dtype, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    hits = (t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"])
    n = ev.n_tracks
    c = kf.Context(0)
    try:
        c.reserve(n, 26)
        for shape in [(256, 0, 1, 1, 0), (256, 1, 4, 2, 2), (256, 0, 1, 2, 3), (128, 1, 4, 1, 4)]:
            c.set_fit_launch(dtype, *shape)
            for graph in (False, True):
                c.set_fit_graph(graph)
                for seg in (None, 3):
                    ck = None if seg is None else torch.full((28, n * kf.n_checkpoint_segments(26, seg)), 7.0,
                                                             dtype=dtype, device=dev)
                    ck2 = None if ck is None else ck.clone()
                    st, cov, q, sst = c.make_seeds(t["hit_offsets"], t["hit_valid"], t["hit_pos"],
                                                   ev.geometry.bz, mode)
                    ref = c.fit_tracks(st, cov, q, *hits, geom, checkpoints=ck, seg=seg or 1)
                    seeds = (torch.full_like(st, 5.0), torch.full_like(cov, 5.0), torch.full_like(q, 5))
                    fused = c.seed_fit_tracks(*hits, geom, mode, seeds=seeds, checkpoints=ck2, seg=seg or 1)
                    torch.cuda.synchronize()
                    for k in ("state", "cov", "charge", "chi2", "ndf"):
                        a_, b_ = ref[k].cpu().numpy(), fused[k].cpu().numpy()
                        assert np.array_equal(a_, b_, equal_nan=a_.dtype.kind == "f"), (shape, graph, seg, k)
                    assert torch.equal(fused["status"], ref["status"] | sst), (shape, graph, seg)
                    assert torch.equal(seeds[0], st) and torch.equal(seeds[1], cov) and torch.equal(seeds[2], q)
                    if ck is not None:
                        assert torch.equal(ck.isnan(), ck2.isnan())
                        assert torch.equal(ck.nan_to_num(0.0), ck2.nan_to_num(0.0)), (shape, graph)
            c.set_fit_graph(False)
        bad = ((sst.cpu().numpy() & kf.TRK_BAD_INPUT) != 0)
        assert bad[:80:8].all()
        # without seed outputs
        plain = c.seed_fit_tracks(*hits, geom, mode)
        torch.cuda.synchronize()
        assert torch.equal(plain["chi2"].nan_to_num(0.0), fused["chi2"].nan_to_num(0.0))
    finally:
        c.close()


@pytest.mark.parametrize("layout,persistent", [(2, 1), (0, 1), (1, 0), (3, 1), (4, 0)])
def test_fit_graph_replay_matches_direct_launches(kf, layout, persistent):
    """Graph replays (several, with the program's own eager work and
    synchronisations between them) give the direct launches' results bit for
    bit; changing an argument captures a new graph."""
    say("fit graph replay", layout, persistent)
    ev = generate(workloads()["mixed26"], 30_000)
    dev = torch.device("cuda", 0)
    t = kf.event_tensors(ev, torch.float32, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    c = kf.Context(0)
    try:
        c.reserve(ev.n_tracks, 26)
        c.set_fit_launch(torch.float32, 128, persistent, 4, 1, layout)
        st, cov, q, _ = c.make_seeds(t["hit_offsets"], t["hit_valid"], t["hit_pos"], ev.geometry.bz, 1)
        args = (st, cov, q, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom)
        ref = c.fit_tracks(*args)
        ref = {k: v.clone() for k, v in ref.items()}
        c.set_fit_graph(True)
        out = kf.fit_outputs(ev.n_tracks, torch.float32, dev)
        for rep in range(4):
            for v in out.values():
                v.fill_(-7)
            c.fit_tracks(*args, out=out)
            junk = torch.randn(1 << 20, device=dev).sum()   # eager work between replays
            torch.cuda.synchronize()
            for k in ref:
                assert torch.equal(ref[k], out[k]), (rep, k)
        # a different output buffer: captured again, same results
        out2 = c.fit_tracks(*args)
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(ref[k], out2[k]), k
        # a smaller batch through the same graph cache
        n2 = 1000
        sub = c.fit_tracks(st[:, :n2].contiguous(), cov[:, :n2].contiguous(), q[:n2].contiguous(),
                           t["hit_offsets"][:n2 + 1].contiguous(), t["hit_layer"], t["hit_valid"], t["hit_pos"],
                           t["hit_cov"], geom)
        torch.cuda.synchronize()
        assert torch.equal(sub["chi2"], ref["chi2"][:n2])
        c.set_fit_graph(False)
        again = c.fit_tracks(*args)
        torch.cuda.synchronize()
        assert torch.equal(again["state"], ref["state"])
    finally:
        c.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_seed_fit_offsets_past_zero(kf, dtype):
    """The tracks' entries need not start at entry 0 of the hit arrays: in
    every layout, the same tracks behind 7 entries that belong to no track
    (valid hits, so that a kernel reading them would use them) and before 5
    more give the same results, bit for bit."""
    say("seed + fit, offsets past zero", dtype)
    ev = generate(workloads()["barrel10"], 300)
    dev = torch.device("cuda", 0)
    geom = kf.Geometry.from_toy(ev.geometry)
    t = kf.event_tensors(ev, dtype, dev)
    nh, front, back = ev.n_hits, 7, 5
    src = (torch.arange(front + nh + back, device=dev) - front) % nh   # entry front + e holds hit e
    pad = lambda x: x[..., src].contiguous()
    valid = pad(t["hit_valid"])
    valid[:front] = 1
    valid[front + nh:] = 1
    padded = ((t["hit_offsets"] + front).contiguous(), pad(t["hit_layer"]), valid, pad(t["hit_pos"]),
              pad(t["hit_cov"]))
    plain = (t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"])
    for layout in range(5):
        c = kf.Context(0)
        try:
            c.reserve(ev.n_tracks, 26)
            c.set_fit_launch(dtype, 256, 0, 1, 2 if dtype == torch.float32 else 1, layout)
            a = c.seed_fit_tracks(*plain, geom, 0)
            b = c.seed_fit_tracks(*padded, geom, 0)
            torch.cuda.synchronize()
            for k in a:
                assert torch.equal(a[k].nan_to_num(7.0), b[k].nan_to_num(7.0)), (layout, k)
        finally:
            c.close()
