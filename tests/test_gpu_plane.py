"""GPU parity of the tilted-module entry points (through the C interface)
against the FP64 plane oracle on the same seeded inputs: propagation to a
module's plane, the local 2-D update, the forward fit over modules (with
holes), and the local-to-global map."""
import sys

import numpy as np
import pytest
import torch

from oracle import kf_oracle as O
from oracle import kf_plane as P
from toygen import generate_planes, plane_workloads

from parity import chi2_error, cov_rel_error, param_error, rounded, sym_unpack

pytestmark = pytest.mark.gpu

TOL32 = (1e-4, 1e-3)
TOL64 = (1e-8, 1e-8)
COV32, COV64 = 1e-3, 1e-7
DT = torch.float64


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


def _event(n, holes=0.0, seed=5, **kw):
    wl = plane_workloads()["tilted10"]
    ev = generate_planes(wl, n, **kw)
    if holes > 0:
        # holes anywhere but in the first three entries (which seed the track)
        rng = np.random.default_rng(seed)
        off = ev.hit_offsets
        pos = np.arange(ev.n_hits) - np.repeat(off[:-1], np.diff(off))
        ev.hit_valid[(pos >= 3) & (rng.uniform(size=ev.n_hits) < holes)] = 0
    return wl, ev


def plane_frame_cov(C, u, v):
    """[N,6,6] covariances in the plane's five coordinates (u, v, ipt, phi,
    theta), which removes the normal null vector."""
    N = C.shape[0]
    B = np.zeros((N, 6, 5))
    B[:, :3, 0], B[:, :3, 1] = u, v
    B[:, 3, 2] = B[:, 4, 3] = B[:, 5, 4] = 1.0
    return np.einsum("nia,nij,njb->nab", B, C, B)


def _frames(tab, mod):
    """(c, n, u, v, x0) of the modules ``mod`` of the table ``tab``."""
    c, n, u, v, x0 = P.frames(tab)
    m = torch.as_tensor(np.asarray(mod, np.int64))
    return c[m], n[m], u[m], v[m], x0[m]


def _spd(k, seed, scale=0.01):
    A = torch.randn(k, 6, 6, dtype=DT, generator=torch.Generator().manual_seed(seed)) * scale
    return A @ A.transpose(1, 2) + 1e-6 * torch.eye(6, dtype=DT)


def _pack(C):
    i, j = np.tril_indices(6)
    return np.ascontiguousarray(np.asarray(C)[:, i, j].T)


def _dev(x, dtype):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).cuda().contiguous()


def _pairs(ev):
    off = ev.hit_offsets
    e0 = np.concatenate([np.arange(off[t], off[t + 1] - 1) for t in range(ev.n_tracks)])
    return e0, e0 + 1


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_propagate_plane_parity(ctx, kf, dtype):
    """From the true state at one module (with a random covariance) to the next
    module's plane, with material: state, path, status and covariance (in the
    target plane's frame)."""
    wl, ev = _event(1500)
    g = wl.geometry
    e0, e1 = _pairs(ev)
    say("propagate_plane", dtype, e0.size)
    p = rounded(ev.truth_after[e0], dtype)
    q = ev.charge[np.searchsorted(ev.hit_offsets, e0, side="right") - 1]
    C = rounded(_spd(e0.size, 7).numpy(), dtype)
    mod = ev.hit_module[e1]
    tab = rounded(g.modules, dtype)
    c, n, u, v, x0 = _frames(tab, mod)
    op, oC, os_, ost = P.propagate_plane(torch.tensor(p), torch.tensor(C), torch.tensor(q, dtype=DT), c, n, x0,
                                         g)
    pg = kf.PlaneGeometry(tab, g.bz, g.mass, dtype=dtype)
    st, cv, path, status = ctx.propagate_plane(_dev(p.T, dtype), _dev(_pack(C), dtype),
                                               torch.as_tensor(q, dtype=torch.int8).cuda(),
                                               torch.as_tensor(mod, dtype=torch.int32).cuda(), pg)
    torch.cuda.synchronize()
    gp = st.double().cpu().numpy().T
    gC = sym_unpack(cv.double().cpu().numpy().T)
    # FP32: a few units in the last place of positions ~100 cm from the origin
    tol = TOL32[0] if dtype == torch.float32 else 1e-10
    ep = param_error(gp, op.numpy()).max(axis=1)
    assert np.array_equal(status.cpu().numpy().astype(np.int64), ost.numpy())
    assert float(ep.max()) < tol, float(ep.max())
    ds = np.abs(path.double().cpu().numpy() - os_.numpy()) / np.maximum(np.abs(os_.numpy()), 1.0)
    assert float(ds.max()) < tol
    uu, vv = u.numpy(), v.numpy()
    rel = cov_rel_error(plane_frame_cov(gC, uu, vv), plane_frame_cov(oC.numpy(), uu, vv))
    ctol = COV32 if dtype == torch.float32 else COV64
    assert float(rel.max()) < ctol, float(rel.max())
    # the GPU covariance also has the normal as a null vector
    nn = np.einsum("ni,nij,nj->n", n.numpy(), gC[:, :3, :3], n.numpy())
    tr = np.trace(gC[:, :3, :3], axis1=1, axis2=2)
    assert float((np.abs(nn) / tr).max()) < (1e-5 if dtype == torch.float32 else 1e-12)
    say("  max param err", float(ep.max()), "max cov err", float(rel.max()))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_update_plane_parity(ctx, kf, dtype):
    """The local update on predicted states (propagated by the oracle, so
    that they lie on the plane), with the generator's smeared hits."""
    wl, ev = _event(1500)
    g = wl.geometry
    e0, e1 = _pairs(ev)
    say("update_plane", dtype, e0.size)
    q = ev.charge[np.searchsorted(ev.hit_offsets, e0, side="right") - 1]
    mod = ev.hit_module[e1]
    tab = rounded(g.modules, dtype)
    c, n, u, v, x0 = _frames(tab, mod)
    # a prior typical of a fit in progress: a few hits' worth of information
    C0 = _spd(e0.size, 8, scale=0.003)
    pp, Cp, _, pst = P.propagate_plane(torch.tensor(ev.truth_after[e0]), C0, torch.tensor(q, dtype=DT), c, n, x0,
                                       g)
    assert int((pst & O.NO_CROSSING).sum()) == 0
    p = rounded(pp.numpy(), dtype)
    C = rounded(Cp.numpy(), dtype)
    m = rounded(ev.hit_uv[:, e1], dtype)
    V = rounded(ev.hit_cov_uv[:, e1], dtype)
    o = P.update_local(torch.tensor(p), torch.tensor(C), torch.tensor(q, dtype=DT), torch.tensor(m.T),
                       P.unpack2(V), c, u, v)
    pg = kf.PlaneGeometry(tab, g.bz, g.mass, dtype=dtype)
    st = _dev(p.T, dtype)
    cv = _dev(_pack(C), dtype)
    qq = torch.as_tensor(q, dtype=torch.int8).cuda()
    chi2, status = ctx.update_plane(st, cv, qq, torch.as_tensor(mod, dtype=torch.int32).cuda(), _dev(m, dtype),
                                    _dev(V, dtype), pg)
    torch.cuda.synchronize()
    gp = st.double().cpu().numpy().T
    gC = sym_unpack(cv.double().cpu().numpy().T)
    tol_p, tol_c = TOL32 if dtype == torch.float32 else TOL64
    ep = param_error(gp, o[0].numpy()).max(axis=1)
    ec = chi2_error(chi2.double().cpu().numpy(), o[3].numpy())
    assert float(ep.max()) < tol_p, float(ep.max())
    assert float(ec.max()) < tol_c, float(ec.max())
    assert np.array_equal(qq.cpu().numpy().astype(np.float64), o[2].numpy())
    assert np.array_equal(status.cpu().numpy().astype(np.int64) & ~O.FP64_FALLBACK, o[4].numpy())
    uu, vv = u.numpy(), v.numpy()
    rel = cov_rel_error(plane_frame_cov(gC, uu, vv), plane_frame_cov(o[1].numpy(), uu, vv))
    eC = rel.reshape(rel.shape[0], -1).max(axis=1)
    say("  max param err", float(ep.max()), "chi2 err", float(ec.max()), "cov err", float(eC.max()),
        "over", int((eC > COV32).sum()))
    if dtype == torch.float32:
        # an FP32 posterior variance carries a relative error of about the
        # prior-to-hit ratio times 2^-23; lanes up to a ratio of 1e4 stay in
        # FP32, so the tail rule of the 3-D update applies: at most 1% of the
        # tracks above 1e-3, none above 1e-2
        assert (eC > COV32).mean() <= 0.01 and float(eC.max()) < 10 * COV32, float(eC.max())
    else:
        assert float(eC.max()) < COV64, float(eC.max())


def _oracle_plane_fit(ev, g, dtype):
    """Seeds from the hits' global positions (the oracle's), rounded to the
    precision, then the oracle fit from those seeds, on inputs rounded the
    same way."""
    tab = rounded(g.modules, dtype)
    uv = rounded(ev.hit_uv, dtype)
    cov = rounded(ev.hit_cov_uv, dtype)
    sp, sC, sq, ok = P.make_seeds_planes(ev.hit_offsets, ev.hit_module, ev.hit_valid, uv, tab, g.bz)
    sp = torch.tensor(rounded(sp.numpy(), dtype))
    out = P.fit_plane_tracks(sp, sC, sq, ev.hit_offsets, ev.hit_module, ev.hit_valid, uv, cov, tab, g)
    return sp, sC, sq, tab, uv, cov, out


def _plane_probes(ev, g, dtype, sp, sC, sq, tab, uv, cov, o, seed=1234):
    """Tracks whose FP64 oracle fit moves by more than half the tolerance, or
    changes its status, ndf or charge, under perturbations at the rounding
    level of ``dtype``: the local hit coordinates moved by one unit in the
    last place (random sign), the state and covariance rounded to FP32 (FP32
    only), and the state and covariance scaled by 1 +- 2^-23 (both sign patterns; FP64: 4e-16)
    element by element after every propagation and update (in FP32 this
    probe counts only where it changes a decision: the status, ndf or
    charge).  No computation in that
    precision can be expected to reproduce such a track (a crossing near
    tangency, say) to the tolerance."""
    tol_p, tol_c = TOL32 if dtype == torch.float32 else TOL64
    rng = np.random.default_rng(seed)
    if dtype == torch.float32:
        ulp = np.spacing(np.abs(uv).astype(np.float32)).astype(np.float64)
    else:
        ulp = 4e-16 * np.maximum(np.abs(uv), 1e-3)
    pert = uv + ulp * rng.choice([-1.0, 1.0], size=uv.shape)
    # (probe, whether it is held to the value tolerance or only to the
    # decisions: status, ndf, charge)
    runs = [(dict(hit_uv=pert), True)]
    if dtype == torch.float32:
        runs += [(dict(state_round=torch.float32), True), (dict(state_jitter=2.0 ** -23), False),
                 (dict(state_jitter=-2.0 ** -23), False)]
    else:
        runs.append((dict(state_jitter=4e-16), True))
    bad = np.zeros(ev.n_tracks, bool)
    for kw, values in runs:
        o2 = P.fit_plane_tracks(sp, sC, sq, ev.hit_offsets, ev.hit_module, ev.hit_valid, kw.get("hit_uv", uv), cov,
                                tab, g, state_round=kw.get("state_round"), state_jitter=kw.get("state_jitter"))
        if values:
            ep = param_error(o2["p"].numpy(), o["p"].numpy()).max(axis=1)
            ec = chi2_error(o2["chi2"].numpy(), o["chi2"].numpy())
            bad |= (ep > 0.5 * tol_p) | (ec > 0.5 * tol_c)
        bad |= (o2["status"].numpy() != o["status"].numpy()) | (o2["ndf"].numpy() != o["ndf"].numpy())
        bad |= o2["q"].numpy() != o["q"].numpy()
    return bad


def _gpu_plane_fit(ctx, kf, ev, g, dtype, sp, sC, sq, tab, uv, cov):
    pg = kf.PlaneGeometry(tab, g.bz, g.mass, dtype=dtype)
    t = kf.plane_event_tensors(ev, dtype)
    t["hit_uv"], t["hit_cov_uv"] = _dev(uv, dtype), _dev(cov, dtype)
    out = ctx.fit_plane_tracks(_dev(sp.numpy().T, dtype), _dev(_pack(sC.numpy()), dtype),
                               torch.as_tensor(sq.numpy(), dtype=torch.int8).cuda(), t["hit_offsets"],
                               t["hit_module"], t["hit_valid"], t["hit_uv"], t["hit_cov_uv"], pg)
    torch.cuda.synchronize()
    return out


def _compare_plane_fit(out, o, ev, g, dtype, tail_frac, bad=None):
    """Parity on the tracks not in ``bad`` (the conditioning probes' flags;
    at most 0.5% of the tracks may be flagged)."""
    ok_t = np.ones(ev.n_tracks, bool) if bad is None else ~bad
    if bad is not None:
        assert bad.mean() <= 0.005, bad.mean()
    gp = out["state"].double().cpu().numpy().T
    gC = sym_unpack(out["cov"].double().cpu().numpy().T)
    tol_p, tol_c = TOL32 if dtype == torch.float32 else TOL64
    ep = param_error(gp, o["p"].numpy()).max(axis=1)
    ec = chi2_error(out["chi2"].double().cpu().numpy(), o["chi2"].numpy())
    gs = out["status"].cpu().numpy().astype(np.int64) & ~O.FP64_FALLBACK
    os_ = o["status"].numpy() & ~O.FP64_FALLBACK
    assert np.array_equal(gs[ok_t], os_[ok_t]), np.nonzero(ok_t & (gs != os_))[0][:10]
    assert np.array_equal(out["ndf"].cpu().numpy()[ok_t], o["ndf"].numpy()[ok_t])
    assert np.array_equal(out["charge"].cpu().numpy().astype(np.float64)[ok_t], o["q"].numpy()[ok_t])
    over = ok_t & ((ep > tol_p) | (ec > tol_c))
    far = ok_t & ((ep > 10 * tol_p) | (ec > 20 * tol_c))
    # the covariance in the frame of the last module each track reached
    last = ev.hit_offsets[1:] - 1
    _, _, u, v, _ = _frames(g.modules, ev.hit_module[last])
    uu, vv = u.numpy(), v.numpy()
    rel = cov_rel_error(plane_frame_cov(gC, uu, vv), plane_frame_cov(o["C"].numpy(), uu, vv))
    eC = np.where(ok_t, rel.reshape(rel.shape[0], -1).max(axis=1), 0.0)
    ctol = COV32 if dtype == torch.float32 else COV64
    summary = dict(n=ev.n_tracks, flagged=int((~ok_t).sum()), max_param_err=float(ep[ok_t].max()),
                   max_chi2_err=float(ec[ok_t].max()), over=int(over.sum()), max_cov_err=float(eC.max()),
                   cov_over=int((eC > ctol).sum()))
    say("  ", summary)
    assert not far.any(), (summary, np.nonzero(far)[0][:10])
    assert over.sum() <= tail_frac * ev.n_tracks, summary
    assert (eC > ctol).sum() <= max(tail_frac, 0.01 if dtype == torch.float32 else 0.0) * ev.n_tracks, summary
    return summary


@pytest.mark.parametrize("dtype,holes", [(torch.float32, 0.0), (torch.float64, 0.0), (torch.float32, 0.1),
                                         (torch.float64, 0.1)])
def test_fit_plane_parity(ctx, kf, dtype, holes):
    wl, ev = _event(3000, holes=holes)
    g = wl.geometry
    say("fit_plane", dtype, "holes", holes, ev.n_tracks, ev.n_hits)
    sp, sC, sq, tab, uv, cov, o = _oracle_plane_fit(ev, g, dtype)
    bad = _plane_probes(ev, g, dtype, sp, sC, sq, tab, uv, cov, o)
    out = _gpu_plane_fit(ctx, kf, ev, g, dtype, sp, sC, sq, tab, uv, cov)
    _compare_plane_fit(out, o, ev, g, dtype, 0.005 if dtype == torch.float32 else 0.0, bad)


def test_fit_plane_full_size(ctx, kf):
    """The whole tilted10 workload (100,000 tracks, FP32), in the launch the
    benchmark times."""
    wl, ev = _event(None)
    g = wl.geometry
    say("fit_plane full", ev.n_tracks, ev.n_hits)
    sp, sC, sq, tab, uv, cov, o = _oracle_plane_fit(ev, g, torch.float32)
    bad = _plane_probes(ev, g, torch.float32, sp, sC, sq, tab, uv, cov, o)
    out = _gpu_plane_fit(ctx, kf, ev, g, torch.float32, sp, sC, sq, tab, uv, cov)
    _compare_plane_fit(out, o, ev, g, torch.float32, 0.005, bad)


def test_fit_plane_empty_and_bad_module(ctx, kf):
    """n = 0 is a no-op; a module id out of range stops its track with
    KF_TRK_BAD_INPUT (the other tracks are unaffected)."""
    wl, ev = _event(64)
    g = wl.geometry
    dtype = torch.float64
    sp, sC, sq, tab, uv, cov, o = _oracle_plane_fit(ev, g, dtype)
    pg = kf.PlaneGeometry(tab, g.bz, g.mass, dtype=dtype)
    t = kf.plane_event_tensors(ev, dtype)
    e = torch.empty(6, 0, dtype=dtype, device="cuda")
    out0 = ctx.fit_plane_tracks(e, torch.empty(21, 0, dtype=dtype, device="cuda"),
                                torch.empty(0, dtype=torch.int8, device="cuda"),
                                torch.zeros(1, dtype=torch.int32, device="cuda"), t["hit_module"], t["hit_valid"],
                                t["hit_uv"], t["hit_cov_uv"], pg)
    assert out0["state"].numel() == 0
    bad = t["hit_module"].clone()
    k = int(ev.hit_offsets[5]) + 4
    bad[k] = g.n_modules
    out = ctx.fit_plane_tracks(_dev(sp.numpy().T, dtype), _dev(_pack(sC.numpy()), dtype),
                               torch.as_tensor(sq.numpy(), dtype=torch.int8).cuda(), t["hit_offsets"], bad,
                               t["hit_valid"], t["hit_uv"], t["hit_cov_uv"], pg)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert st[5] & kf.TRK_BAD_INPUT
    assert int(out["ndf"][5]) == 2 * 4 - 5
    others = np.arange(ev.n_tracks) != 5
    assert not (st[others] & kf.TRK_BAD_INPUT).any()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_plane_to_global_parity(ctx, kf, dtype):
    wl, ev = _event(500)
    g = wl.geometry
    tab = rounded(g.modules, dtype)
    uv = rounded(ev.hit_uv, dtype)
    c, n, u, v, _ = _frames(tab, ev.hit_module)
    want = P.local_to_global(torch.tensor(uv.T), c, u, v).numpy().T
    pg = kf.PlaneGeometry(tab, g.bz, g.mass, dtype=dtype)
    mod = torch.as_tensor(ev.hit_module, dtype=torch.int32).cuda()
    got = ctx.plane_to_global(mod, _dev(uv, dtype), pg).double().cpu().numpy()
    # a coordinate is c + m_u u + m_v v: its rounding is that of the module
    # centre's magnitude, whatever the size of the result
    scale = np.abs(c.numpy()).sum(axis=1) + np.abs(uv).sum(axis=0) + 1.0
    eps = 2.0 ** -23 if dtype == torch.float32 else 2.0 ** -52
    assert float((np.abs(got - want) / scale).max()) < 4 * eps
    # the global positions match the generator's measured points
    assert float(np.abs(got - ev.hit_pos).max()) < (1e-4 if dtype == torch.float32 else 1e-9)
