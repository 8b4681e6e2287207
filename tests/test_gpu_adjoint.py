"""GPU parity of the hand-written reverse pass (kf_fit_adjoint, through the C
interface): against the FP64 oracle's gradient (autograd through the oracle
fit, a mechanism that shares nothing with the reverse pass), against central
finite differences of the GPU fit (step 1e-4 cm on hit positions and
alignment offsets), and through the torch.autograd.Function.

Tolerances.  FP64: the per-track relative L2 error of the track's hit-position
gradients is held to 1e-6 and the alignment gradient (a sum over tracks) to
1e-8.  The seed-state gradient is held to 1e-5: chi2 depends only weakly on a
seed with a wide covariance, so that gradient is a small difference of much
larger terms of the reverse sweep (median error ~4e-10, tail ~1e-6).
FP32 (forward states in FP32, reverse arithmetic in FP64): the gradient
inherits the forward path's FP32 error.  Its scale is measured, per batch, by
two conditioning probes of the FP64 oracle: the hit positions moved by one
unit in the last place of FP32, and the running state rounded to FP32 after
every propagation and update.  How far the oracle's own gradient moves under
them is what any FP32 computation must be allowed; the FP32 errors are held,
quantile by quantile (50%, 90%, 99%), within 3x of that movement and the
single worst track within 10x of the worst movement, with
absolute caps of 5e-2 (hit gradients, per-track relative L2), 1e-1 (seed
gradient, which amplifies state errors by the seed's weak influence) and
2e-3 (the alignment gradient, a sum over all tracks).  Measured: medians
~1e-4 to 3e-4, maxima ~1e-2.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import kf_oracle as O
from toygen import generate, truncate, workloads

from parity import rounded

pytestmark = pytest.mark.gpu


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


IL = [(i, j) for i in range(6) for j in range(i + 1)]


def unpack(packed):
    """[21, n] packed lower triangle -> [n, 6, 6]."""
    n = packed.shape[1]
    M = np.zeros((n, 6, 6))
    for k, (i, j) in enumerate(IL):
        M[:, i, j] = M[:, j, i] = packed[k]
    return M


def gpu_run(ctx, kf, ev, dtype, align=None, w=None, seg=4, max_len=26, mode=0, hit_pos=None, layer=None):
    """Seeds, fit with checkpoints and adjoint on the GPU.  Returns numpy
    arrays (float64) of the seeds, the fit and the gradients."""
    dev = ctx.device
    t = kf.event_tensors(ev, dtype, dev)
    if hit_pos is not None:
        t["hit_pos"] = torch.as_tensor(np.asarray(hit_pos), device=dev).to(dtype).contiguous()
    if layer is not None:
        t["hit_layer"] = torch.as_tensor(np.asarray(layer, np.int16), device=dev).contiguous()
    geom = kf.Geometry.from_toy(ev.geometry)
    st, cov, q, _ = ctx.make_seeds(t["hit_offsets"], t["hit_valid"], t["hit_pos"], ev.geometry.bz, mode)
    al = None if align is None else torch.as_tensor(np.asarray(align), device=dev).to(dtype).contiguous()
    wt = None if w is None else torch.as_tensor(np.asarray(w), device=dev).to(dtype).contiguous()
    n = ev.n_tracks
    ck = torch.empty(28, n * kf.n_checkpoint_segments(max_len, seg), dtype=dtype, device=dev)
    out = ctx.fit_tracks(st, cov, q, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"],
                         geom, align=al, checkpoints=ck, seg=seg, max_len=max_len)
    gs, gh, ga = ctx.fit_adjoint(st, cov, q, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"],
                                 t["hit_cov"], geom, ck, seg, max_len, out["status"], align=al, dL_dchi2=wt)
    torch.cuda.synchronize()
    f = lambda x: x.double().cpu().numpy()
    return dict(seed=f(st).T, seed_cov=unpack(f(cov)), seed_q=q.cpu().numpy().astype(np.float64),
                chi2=f(out["chi2"]), status=out["status"].cpu().numpy(), gs=f(gs).T, gh=f(gh), ga=f(ga))


def oracle_grad(ev, g, dtype, align=None, w=None, hit_pos=None, state_round=None):
    """FP64 oracle gradient at the inputs the GPU path of precision dtype saw
    (hits and alignment rounded to dtype, the GPU's own seeds)."""
    hp = rounded(ev.hit_pos, dtype) if hit_pos is None else np.asarray(hit_pos, np.float64)
    al = None if align is None else torch.tensor(rounded(align, dtype))
    wt = None if w is None else torch.tensor(rounded(w, dtype))
    loss, gs, gh, ga, out = O.fit_gradients(torch.tensor(g["seed"]), torch.tensor(g["seed_cov"]),
                                            torch.tensor(g["seed_q"]), ev.hit_offsets, ev.hit_layer, ev.hit_valid,
                                            torch.tensor(hp), rounded(ev.hit_cov, dtype), ev.geometry, align=al,
                                            weights=wt, state_round=state_round)
    return dict(chi2=out["chi2"].numpy(), gs=gs.numpy(), gh=gh.numpy(), ga=ga.numpy())


def fp32_probes(ev, g, o, align, w):
    """Per-track movement (seed block, hit block) of the FP64 oracle's
    gradient under the two FP32 conditioning probes: hit positions moved by
    one unit in the last place of FP32 (random sign), and the running state
    rounded to FP32 after every propagation and update."""
    rng = np.random.default_rng(77)
    hp = rounded(ev.hit_pos, torch.float32)
    ulp = np.spacing(np.abs(hp).astype(np.float32)).astype(np.float64)
    o_u = oracle_grad(ev, g, torch.float32, align, w, hit_pos=hp + ulp * rng.choice([-1.0, 1.0], size=hp.shape))
    o_r = oracle_grad(ev, g, torch.float32, align, w, state_round=torch.float32)
    s_u, h_u = per_track_rel(ev, o_u, o)
    s_r, h_r = per_track_rel(ev, o_r, o)
    return np.maximum(s_u, s_r), np.maximum(h_u, h_r)


def per_track_rel(ev, g, o):
    """Per-track relative L2 errors of the seed gradient and of the track's
    hit-position gradients."""
    es = np.linalg.norm(g["gs"] - o["gs"], axis=1) / np.maximum(np.linalg.norm(o["gs"], axis=1), 1e-300)
    off = ev.hit_offsets
    eh = np.zeros(ev.n_tracks)
    for t in range(ev.n_tracks):
        a, b = off[t], off[t + 1]
        eh[t] = np.linalg.norm(g["gh"][:, a:b] - o["gh"][:, a:b]) / max(np.linalg.norm(o["gh"][:, a:b]), 1e-300)
    return es, eh


def check_fp32(es, eh, probes=None, factor=3.0):
    """FP32 gradient bounds (see the module docstring)."""
    assert eh.max() <= 5e-2, (eh.max(), int(eh.argmax()))
    assert es.max() <= 1e-1, (es.max(), int(es.argmax()))
    assert np.median(es) <= 1e-3 and np.median(eh) <= 1e-3, (np.median(es), np.median(eh))
    if probes is not None:
        ps, ph = probes
        for q, f in ((0.5, factor), (0.9, factor), (0.99, factor), (1.0, 10 * factor / 3)):
            assert np.quantile(es, q) <= f * np.quantile(ps, q), ("seed", q, np.quantile(es, q), np.quantile(ps, q))
            assert np.quantile(eh, q) <= f * np.quantile(ph, q), ("hits", q, np.quantile(eh, q), np.quantile(ph, q))


@pytest.mark.parametrize("name,mode,n,dtype", [("align20", 0, 300, torch.float64), ("mixed26", 1, 300, torch.float64),
                                               ("align20", 0, 2000, torch.float32),
                                               ("mixed26", 1, 2000, torch.float32)])
def test_adjoint_matches_oracle_gradient(ctx, kf, name, mode, n, dtype):
    say("adjoint vs oracle", name, n, dtype)
    ev = generate(workloads()[name], n)
    align = ev.align_true * 0.5
    w = np.linspace(0.5, 2.0, n)
    g = gpu_run(ctx, kf, ev, dtype, align=align, w=w, seg=4, mode=mode)
    o = oracle_grad(ev, g, dtype, align=align, w=w)
    es, eh = per_track_rel(ev, g, o)
    ea = np.linalg.norm(g["ga"] - o["ga"]) / np.linalg.norm(o["ga"])
    say("  seed grad rel L2 max %.2e median %.2e; hit grad max %.2e median %.2e; align %.2e"
        % (es.max(), np.median(es), eh.max(), np.median(eh), ea))
    assert np.isfinite(g["gh"]).all() and np.isfinite(g["gs"]).all()
    if dtype == torch.float64:
        assert es.max() <= 1e-5 and eh.max() <= 1e-6, (int(es.argmax()), int(eh.argmax()))
        assert ea <= 1e-8
    else:
        ps, ph = fp32_probes(ev, g, o, align, w)
        say("  probe quantiles (50/90/99/100%%): seed %s hits %s" % (np.quantile(ps, [.5, .9, .99, 1]),
                                                                    np.quantile(ph, [.5, .9, .99, 1])))
        check_fp32(es, eh, (ps, ph))
        assert ea <= 2e-3


def _fd_loss(ctx, kf, ev, hp, align, geom, t64, seeds):
    """Per-track chi2 of the FP64 GPU fit at hit positions hp, alignment align."""
    dev = ctx.device
    st, cov, q = seeds
    al = torch.as_tensor(align, device=dev).double().contiguous()
    h = torch.as_tensor(hp, device=dev).double().contiguous()
    out = ctx.fit_tracks(st, cov, q, t64["hit_offsets"], t64["hit_layer"], t64["hit_valid"], h, t64["hit_cov"], geom,
                         align=al)
    return out["chi2"].cpu().numpy()


def _central(f, x, dx):
    """Central difference at step dx and its Richardson extrapolation from
    steps dx and dx/2 (error O(dx^4))."""
    d1 = (f(x + dx) - f(x - dx)) / (2 * dx)
    d2 = (f(x + dx / 2) - f(x - dx / 2)) / dx
    return d1, (4 * d2 - d1) / 3


def _rel_rows(a, b):
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_adjoint_matches_finite_differences(ctx, kf, dtype):
    """Central differences of the FP64 GPU fit, step 1e-4 cm, on 64 tracks:
    hit positions (three entries of every track, all three coordinates, all
    tracks perturbed at once since their chi2 are independent), the alignment
    offsets of every layer, and the seed states.  The plain difference at
    1e-4 cm carries a truncation error of up to ~1e-4 relative (the early hits
    move the curvature, on which the scattering noise and the Jacobian
    depend); its Richardson extrapolation (steps 1e-4 and 5e-5) does not, and
    holds the FP64 adjoint to 1e-6."""
    say("adjoint vs finite differences", dtype)
    ev = generate(workloads()["align20"], 64)
    n = ev.n_tracks
    hp = rounded(ev.hit_pos, torch.float32)   # the same inputs for both precisions
    align = rounded(ev.align_true * 0.5, torch.float32)
    g = gpu_run(ctx, kf, ev, dtype, align=align, hit_pos=hp, seg=5)
    dev = ctx.device
    t64 = kf.event_tensors(ev, torch.float64, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    seeds = (torch.as_tensor(g["seed"].T.copy(), device=dev).contiguous(),
             torch.as_tensor(np.stack([g["seed_cov"][:, i, j] for i, j in IL]), device=dev).contiguous(),
             torch.as_tensor(g["seed_q"].astype(np.int8), device=dev))
    h = 1e-4
    off = ev.hit_offsets
    entries = [(k, c) for k in (2, 9, 17) for c in range(3)]
    fd1, fdr, ad = np.zeros((n, 9)), np.zeros((n, 9)), np.zeros((n, 9))
    for col, (k, c) in enumerate(entries):
        e = off[:-1] + k
        assert (ev.hit_valid[e] != 0).all()

        def f(x, e=e, c=c):
            hpx = hp.copy()
            hpx[c, e] = x
            return _fd_loss(ctx, kf, ev, hpx, align, geom, t64, seeds)

        fd1[:, col], fdr[:, col] = _central(f, hp[c, e], h)
        ad[:, col] = g["gh"][c, e]
    L = ev.geometry.n_layers
    ga1, gar = np.zeros((2, L)), np.zeros((2, L))
    for c in range(2):
        for lay in range(L):
            def fa(x, c=c, lay=lay):
                ax = align.copy()
                ax[c, lay] = x
                return _fd_loss(ctx, kf, ev, hp, ax, geom, t64, seeds).sum()

            ga1[c, lay], gar[c, lay] = _central(fa, align[c, lay], h)
    steps = [1e-4] * 6
    gs1, gsr = np.zeros((n, 6)), np.zeros((n, 6))
    for j in range(6):
        def fs(x, j=j):
            st = seeds[0].clone()
            st[j] = torch.as_tensor(x, device=dev)
            return _fd_loss(ctx, kf, ev, hp, align, geom, t64, (st, seeds[1], seeds[2]))

        gs1[:, j], gsr[:, j] = _central(fs, g["seed"][:, j], steps[j])
    eh1, ehr = _rel_rows(ad, fd1), _rel_rows(ad, fdr)
    es1, esr = _rel_rows(g["gs"], gs1), _rel_rows(g["gs"], gsr)
    ea1 = np.linalg.norm(g["ga"] - ga1) / np.linalg.norm(ga1)
    ear = np.linalg.norm(g["ga"] - gar) / np.linalg.norm(gar)
    say("  hits: plain %.2e richardson %.2e | seeds: plain %.2e richardson %.2e | align: plain %.2e richardson %.2e"
        % (eh1.max(), ehr.max(), es1.max(), esr.max(), ea1, ear))
    if dtype == torch.float64:
        assert eh1.max() <= 2e-4 and es1.max() <= 2e-4 and ea1 <= 2e-4
        assert ehr.max() <= 1e-6, (ehr.max(), int(ehr.argmax()))
        assert esr.max() <= 1e-6, (esr.max(), int(esr.argmax()))
        assert ear <= 1e-6
    else:
        check_fp32(esr, ehr)
        assert ear <= 2e-3


def test_autograd_function_matches_the_direct_call(ctx, kf):
    say("autograd function")
    ev = generate(workloads()["align20"], 1000)
    dev = ctx.device
    dt = torch.float32
    t = kf.event_tensors(ev, dt, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    st, cov, q, _ = ctx.make_seeds(t["hit_offsets"], t["hit_valid"], t["hit_pos"], ev.geometry.bz, 0)
    align = torch.as_tensor(ev.align_true * 0.5, device=dev).to(dt).contiguous()
    w = torch.linspace(0.5, 2.0, 1000, device=dev, dtype=dt)
    s1, h1, a1 = st.clone().requires_grad_(True), t["hit_pos"].clone().requires_grad_(True), align.clone().requires_grad_(True)
    chi2, out = kf.fit_chi2(ctx, s1, h1, a1, cov, q, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_cov"],
                            geom, seg=5, max_len=26)
    (w * chi2).sum().backward()
    ck = torch.empty(28, 1000 * kf.n_checkpoint_segments(26, 5), dtype=dt, device=dev)
    o2 = ctx.fit_tracks(st, cov, q, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom,
                        align=align, checkpoints=ck, seg=5, max_len=26)
    gs, gh, ga = ctx.fit_adjoint(st, cov, q, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"],
                                 t["hit_cov"], geom, ck, 5, 26, o2["status"], align=align, dL_dchi2=w)
    assert torch.equal(chi2.detach(), o2["chi2"])
    assert torch.equal(s1.grad, gs) and torch.equal(h1.grad, gh) and torch.equal(a1.grad, ga)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_adjoint_is_deterministic_and_segment_independent(ctx, kf, dtype):
    """Bit-identical on a repeat.  Across checkpoint spacings the recomputed
    states differ from the stored ones by rounding only (the fit kernel and
    the adjoint kernel are compiled separately, and an FP32 update near the
    FP32/FP64 switch may take the other branch): in FP64 the gradients agree
    to 1e-6, in FP32 every spacing meets the bounds against the oracle."""
    say("determinism / segments", dtype)
    ev = generate(workloads()["align20"], 5000)
    align = ev.align_true * 0.5
    ref = gpu_run(ctx, kf, ev, dtype, align=align, seg=4)
    again = gpu_run(ctx, kf, ev, dtype, align=align, seg=4)
    for k in ("gs", "gh", "ga"):
        assert np.array_equal(ref[k], again[k]), k
    if dtype == torch.float32:
        o = oracle_grad(ev, ref, dtype, align=align)
        probes = fp32_probes(ev, ref, o, align, None)
    for seg in (1, 7, 25):
        g = gpu_run(ctx, kf, ev, dtype, align=align, seg=seg)
        es, eh = per_track_rel(ev, g, ref)
        ea = np.linalg.norm(g["ga"] - ref["ga"]) / np.linalg.norm(ref["ga"])
        say("  seg %d vs seg 4: seed %.2e hits %.2e align %.2e" % (seg, es.max(), eh.max(), ea))
        if dtype == torch.float64:
            assert es.max() <= 1e-6 and eh.max() <= 1e-6 and ea <= 1e-9, (seg, es.max(), eh.max(), ea)
        else:
            check_fp32(*per_track_rel(ev, g, o), probes)
            assert ea <= 1e-4, (seg, ea)


def test_adjoint_truncation_and_stops(ctx, kf):
    """max_len below the track length: the gradient is that of the fit of the
    first max_len entries, and the rest get 0.  A bad layer id at entry 10
    stops the forward fit there: the gradient is that of the first 10
    entries."""
    say("adjoint truncation / stops")
    ev = generate(workloads()["align20"], 200)
    align = ev.align_true * 0.5
    dt = torch.float64
    g = gpu_run(ctx, kf, ev, dt, align=align, seg=3, max_len=12)
    tr = truncate(ev, np.full(ev.n_tracks, 12))
    o = oracle_grad(tr, g, dt, align=align)
    off, toff = ev.hit_offsets, tr.hit_offsets
    for t in range(ev.n_tracks):
        a = off[t]
        np.testing.assert_allclose(g["gh"][:, a:a + 12], o["gh"][:, toff[t]:toff[t + 1]], rtol=1e-6,
                                   atol=1e-9 * np.abs(o["gh"]).max())
        assert not g["gh"][:, a + 12:off[t + 1]].any()
    np.testing.assert_allclose(g["gs"], o["gs"], rtol=1e-6, atol=1e-9 * np.abs(o["gs"]).max())
    np.testing.assert_allclose(g["ga"], o["ga"], rtol=1e-6, atol=1e-9 * np.abs(o["ga"]).max())
    layer = ev.hit_layer.copy()
    layer[off[:-1] + 10] = 99
    g2 = gpu_run(ctx, kf, ev, dt, align=align, seg=3, layer=layer)
    assert (g2["status"] & kf.KF_TRK_BAD_INPUT).all()
    tr = truncate(ev, np.full(ev.n_tracks, 10))
    o = oracle_grad(tr, g2, dt, align=align)
    for t in range(ev.n_tracks):
        a = off[t]
        np.testing.assert_allclose(g2["gh"][:, a:a + 10], o["gh"][:, tr.hit_offsets[t]:tr.hit_offsets[t + 1]],
                                   rtol=1e-6, atol=1e-9 * np.abs(o["gh"]).max())
        assert not g2["gh"][:, a + 10:off[t + 1]].any()
    np.testing.assert_allclose(g2["gs"], o["gs"], rtol=1e-6, atol=1e-9 * np.abs(o["gs"]).max())


def test_adjoint_empty_batch(ctx, kf):
    dev = ctx.device
    geom = kf.Geometry.from_toy(workloads()["align20"].geometry)
    z = lambda *s, dt=torch.float32: torch.zeros(*s, dtype=dt, device=dev)
    gs, gh, ga = ctx.fit_adjoint(z(6, 0), z(21, 0), z(0, dt=torch.int8), z(1, dt=torch.int32), z(0, dt=torch.int16),
                                 z(0, dt=torch.uint8), z(3, 0), z(6, 0), geom, z(28, 0), 4, 26, z(0, dt=torch.int32))
    torch.cuda.synchronize()
    assert gs.shape == (6, 0) and gh.shape == (3, 0)
    assert not ga.any()


def test_adjoint_full_size_sampled(kf):
    """align20 at its full size (100,000 FP32 tracks x 20 barrel layers) in the
    benchmark's configuration: the forward fit in the staged launch shape with
    the state checkpointed before every entry (seg 1), zero alignment
    offsets, the adjoint and the alignment reduction.  Tracks are independent,
    so 40 sampled tracks are held to the FP64 oracle's gradient computed on
    those tracks alone, within the FP32 bounds above.  The alignment gradient
    sums over all 2,000,000 entries; it is held to the same sum formed in FP64
    from the returned hit-position gradients (d(hit)/d(offset) at zero
    offsets: (-y, x, 0) / R for the r-phi offset, (0, 0, 1) for z), to 2e-5 of
    the sum of the terms' magnitudes (FP32 sums of 100,000 terms per layer)."""
    from toygen import subset
    say("adjoint full size align20")
    wl = workloads()["align20"]
    ev = generate(wl)
    n, nh = ev.n_tracks, ev.n_hits
    dev = torch.device("cuda", 0)
    dt = torch.float32
    c = kf.Context(0)
    try:
        c.set_fit_launch(dt, 256, 0, 1, 2, 3)
        t = kf.event_tensors(ev, dt, dev)
        geom = kf.Geometry.from_toy(wl.geometry)
        max_len = int(ev.lengths().max())
        st, cov, q, _ = c.make_seeds(t["hit_offsets"], t["hit_valid"], t["hit_pos"], wl.geometry.bz, 0)
        al = torch.zeros(2, wl.geometry.n_layers, dtype=dt, device=dev)
        ck = torch.empty(28, n * kf.n_checkpoint_segments(max_len, 1), dtype=dt, device=dev)
        out = c.fit_tracks(st, cov, q, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"],
                           geom, align=al, checkpoints=ck, seg=1, max_len=max_len)
        gs, gh, ga = c.fit_adjoint(st, cov, q, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"],
                                   t["hit_cov"], geom, ck, 1, max_len, out["status"], align=al)
        torch.cuda.synchronize()
        f = lambda x: x.double().cpu().numpy()
        gs, gh, ga, hp = f(gs).T, f(gh), f(ga), f(t["hit_pos"])
        seed, seed_cov, seed_q = f(st).T, unpack(f(cov)), q.cpu().numpy().astype(np.float64)
    finally:
        c.close()
    assert np.isfinite(gs).all() and np.isfinite(gh).all() and np.isfinite(ga).all()
    # alignment gradient: the full-size sum against the FP64 sum of its terms
    R = wl.geometry.pos[ev.hit_layer].astype(np.float64)
    v = ev.hit_valid.astype(bool)
    terms_rphi = np.where(v, (hp[0] * gh[1] - hp[1] * gh[0]) / R, 0.0)
    terms_z = np.where(v, gh[2], 0.0)
    L = wl.geometry.n_layers
    for row, terms in ((0, terms_rphi), (1, terms_z)):
        ref = np.bincount(ev.hit_layer, weights=terms, minlength=L)
        mag = np.bincount(ev.hit_layer, weights=np.abs(terms), minlength=L)
        err = np.abs(ga[row] - ref)
        say("  alignment row %d: max |err| / sum|terms| = %.2e" % (row, (err / np.maximum(mag, 1e-300)).max()))
        assert (err <= 2e-5 * mag + 1e-30).all(), (row, int(np.argmax(err / np.maximum(mag, 1e-300))))
    # sampled tracks against the oracle on those tracks alone
    idx = np.sort(np.random.default_rng(2025).choice(n, 40, replace=False))
    sub = subset(ev, idx)
    g = dict(seed=seed[idx], seed_cov=seed_cov[idx], seed_q=seed_q[idx], gs=gs[idx],
             gh=np.concatenate([gh[:, ev.hit_offsets[i]:ev.hit_offsets[i + 1]] for i in idx], axis=1))
    o = oracle_grad(sub, g, dt)
    es, eh = per_track_rel(sub, g, o)
    ps, ph = fp32_probes(sub, g, o, None, None)
    say("  sampled tracks: seed grad rel L2 max %.2e median %.2e; hit grad max %.2e median %.2e"
        % (es.max(), np.median(es), eh.max(), np.median(eh)))
    check_fp32(es, eh, (ps, ph))
