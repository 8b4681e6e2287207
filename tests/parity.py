"""Helpers shared by the GPU parity tests: run the HIP path through the C
interface and the FP64 oracle on the same inputs, and compare them with the
stated tolerances.

Tolerances (parameters and chi2, FP32 path):
  |dp_i| <= 1e-4 * max(|p_i|, s_i), s = (1 cm, 1 cm, 1 cm, 0.1 c/GeV, 1 rad, 1 rad)
  |dchi2| <= 1e-3 * max(chi2, 1)
The FP64 GPU path is held to 1e-8 on the same scales.

Conditioning: a track whose FP64 result moves by more than half the tolerance
when its hit positions are perturbed at the FP32 rounding level (one unit in
the last place, random sign) cannot be reproduced by any FP32 computation to
that tolerance; such tracks are counted and reported, and held to a loose
bound instead (their fraction must stay small)."""
from __future__ import annotations

import math

import numpy as np
import torch

from oracle import kf_oracle as O

SCALE = np.array([1.0, 1.0, 1.0, 0.1, 1.0, 1.0])


def param_error(a, b):
    """Scaled error |a-b| / max(|b|, s) per track and parameter (phi wrapped)."""
    d = a - b
    d[:, 4] = np.angle(np.exp(1j * d[:, 4]))
    return np.abs(d) / np.maximum(np.abs(b), SCALE)


def chi2_error(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1.0)


def rounded(x, dtype):
    """Inputs as the GPU path of precision ``dtype`` sees them, back in float64."""
    return np.asarray(x).astype(np.float32).astype(np.float64) if dtype == torch.float32 else np.asarray(x, np.float64)


def oracle_fit(ev, dtype, seed_mode=0, hit_pos=None, align=None, state_round=None, state_jitter=None):
    hp = rounded(ev.hit_pos, dtype) if hit_pos is None else np.asarray(hit_pos, np.float64)
    hc = rounded(ev.hit_cov, dtype)
    sp, sC, sq, ok = O.make_seeds(ev.hit_offsets, ev.hit_valid, hp, ev.geometry.bz, mode=seed_mode)
    if state_round is not None:
        sp = sp.to(state_round).to(torch.float64)
    out = O.fit_tracks(sp, sC, sq, ev.hit_offsets, ev.hit_layer, ev.hit_valid, torch.tensor(hp), hc, ev.geometry,
                       align=None if align is None else torch.tensor(rounded(align, dtype)),
                       state_round=state_round, state_jitter=state_jitter)
    return dict(p=out["p"].numpy(), C=out["C"].numpy(), q=out["q"].numpy(), chi2=out["chi2"].numpy(),
                ndf=out["ndf"].numpy(), status=out["status"].numpy(), seed=sp.numpy(), seed_q=sq.numpy())


def ill_conditioned(ev, dtype, ref, seed_mode=0, tol_p=1e-4, tol_c=1e-3, align=None, seed=1234):
    """Tracks whose float64 oracle result moves by more than half the
    tolerance under perturbations at the rounding level of ``dtype``: the hit
    positions perturbed by one unit in the last place (random sign), and the
    state and covariance rounded to ``dtype`` after every propagation and
    update (what storing the running estimate in that precision does at the
    least; for float64, a relative jitter of 4e-16 instead).  No computation
    in that precision can be expected to reproduce such a track to the
    tolerance."""
    rng = np.random.default_rng(seed)
    hp = rounded(ev.hit_pos, dtype)
    if dtype == torch.float32:
        ulp = np.spacing(np.abs(hp).astype(np.float32)).astype(np.float64)
        probe = dict(state_round=torch.float32)
    else:
        ulp = 1e-13 * np.maximum(np.abs(hp), 1.0)
        probe = dict(state_jitter=4e-16)
    pert = hp + ulp * rng.choice([-1.0, 1.0], size=hp.shape)
    bad = np.zeros(ev.n_tracks, bool)
    for kw in (dict(hit_pos=pert), probe):
        o2 = oracle_fit(ev, dtype, seed_mode, align=align, **kw)
        ep = param_error(o2["p"], ref["p"]).max(axis=1)
        ec = chi2_error(o2["chi2"], ref["chi2"])
        bad |= (ep > 0.5 * tol_p) | (ec > 0.5 * tol_c) | (o2["status"] != ref["status"])
    return bad


def gpu_fit(ctx, kf, ev, dtype, seed_mode=0, align=None, checkpoints=None, seg=1, max_len=26):
    dev = ctx.device
    t = kf.event_tensors(ev, dtype, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    st, cov, q, sstat = ctx.make_seeds(t["hit_offsets"], t["hit_valid"], t["hit_pos"], ev.geometry.bz, seed_mode)
    al = None if align is None else torch.as_tensor(np.asarray(align), device=dev).to(dtype).contiguous()
    out = ctx.fit_tracks(st, cov, q, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"],
                         geom, align=al, checkpoints=checkpoints, seg=seg, max_len=max_len)
    torch.cuda.synchronize()
    return dict(p=out["state"].double().cpu().numpy().T, C=out["cov"].double().cpu().numpy().T,
                q=out["charge"].cpu().numpy().astype(np.float64), chi2=out["chi2"].double().cpu().numpy(),
                ndf=out["ndf"].cpu().numpy(), status=out["status"].cpu().numpy().astype(np.int64),
                seed=st.double().cpu().numpy().T, seed_q=q.cpu().numpy().astype(np.float64),
                seed_status=sstat.cpu().numpy())


# covariance tolerance in correlation units on the surface's five directions
COV_TOL32 = 1e-3
COV_TOL64 = 1e-7
COV_TAIL32 = 0.01   # fraction of FP32 tracks allowed above COV_TOL32


def surface_kind(p, geom):
    """0 where the state lies on a barrel cylinder of ``geom``, 1 where it lies
    on a disk (whichever surface is closest)."""
    kinds = np.asarray(geom.kind)
    pos = np.asarray(geom.pos, np.float64)
    r = np.hypot(p[:, 0], p[:, 1])
    db = np.where(kinds[None, :] == 0, np.abs(r[:, None] - pos[None, :]), np.inf).min(axis=1, initial=np.inf)
    dd = np.where(kinds[None, :] == 1, np.abs(p[:, 2:3] - pos[None, :]), np.inf).min(axis=1, initial=np.inf)
    return np.where(db <= dd, 0, 1)


def cov_error(g, o, geom):
    """Per-track maximum over the surface frame of |dC_ab| / sqrt(C_aa C_bb)
    between the GPU covariance g["C"] ([n, 21] packed or [n, 6, 6]) and the
    oracle's o["C"], in the frame of the oracle state's surface."""
    Cg = g["C"] if g["C"].ndim == 3 else sym_unpack(g["C"])
    kind = surface_kind(o["p"], geom)
    rel = cov_rel_error(tangent_frame_cov(Cg, o["p"], kind), tangent_frame_cov(o["C"], o["p"], kind))
    return rel.reshape(rel.shape[0], -1).max(axis=1) if rel.shape[0] else np.zeros(0)


def compare_fit(g, o, tol_p, tol_c, mask=None, ignore_bits=O.FP64_FALLBACK, tail_frac=0.0, tail_factor=10.0,
                tail_factor_chi2=20.0, geom=None, cov_tol=None):
    """Assert parity on the tracks in ``mask`` (default all); return a summary.
    At most ``tail_frac`` of the compared tracks may exceed the tolerance, and
    those only by less than ``tail_factor`` (parameters) or
    ``tail_factor_chi2`` (chi2) times it.  The chi2 tail is set by the FP32
    resolution of absolute positions: at r ~ 100 cm one unit in the last place
    (7.6e-6 cm) is 0.25% of the r-phi resolution, so a residual of a few sigma
    carries a relative chi2 error of that order.
    With ``geom``, the output covariances are compared too, in correlation
    units on the five directions of the output state's surface (its normal is
    a null vector): to ``cov_tol`` (default 1e-3 when tol_p is an FP32
    tolerance, 1e-7 for FP64).  FP64: the tail rule of the parameters (at
    most tail_frac of the tracks above it, none above tail_factor times it).
    FP32: at most max(COV_TAIL32, tail_frac) of the tracks above it, the
    largest error reported."""
    n = g["chi2"].shape[0]
    m = np.ones(n, bool) if mask is None else mask
    ep = param_error(g["p"], o["p"]).max(axis=1)
    ec = chi2_error(g["chi2"], o["chi2"])
    gs = g["status"] & ~ignore_bits
    os_ = o["status"] & ~ignore_bits
    over = m & ((ep > tol_p) | (ec > tol_c))
    summary = dict(n=int(n), compared=int(m.sum()), max_param_err=float(ep[m].max(initial=0.0)),
                   max_chi2_err=float(ec[m].max(initial=0.0)), over_tolerance=int(over.sum()))
    if geom is not None and n > 0:
        fp32 = tol_p > 1e-6
        ctol = cov_tol if cov_tol is not None else (COV_TOL32 if fp32 else COV_TOL64)
        eC = cov_error(g, o, geom)
        overC = m & (eC > ctol)
        summary.update(max_cov_err=float(eC[m].max(initial=0.0)), cov_over_tolerance=int(overC.sum()),
                       cov_err_p99=float(np.quantile(eC[m], 0.99)) if m.any() else 0.0)
        if fp32:
            # FP32: at least 99% of the tracks within the tolerance; the rest
            # is reported (the tail of the FP32 covariance arithmetic)
            assert overC.sum() <= max(COV_TAIL32, tail_frac) * max(m.sum(), 1), (summary, np.nonzero(overC)[0][:10])
        else:
            farC = np.nonzero(m & (eC > tail_factor * ctol))[0]
            assert farC.size == 0, (summary, farC[:10], eC[farC[:10]])
            assert overC.sum() <= tail_frac * max(m.sum(), 1), (summary, np.nonzero(overC)[0][:10])
    far = np.nonzero(m & ((ep > tail_factor * tol_p) | (ec > tail_factor_chi2 * tol_c)))[0]
    assert far.size == 0, (summary, far[:10], ep[far[:10]], ec[far[:10]])
    assert over.sum() <= tail_frac * max(m.sum(), 1), (summary, np.nonzero(over)[0][:10])
    assert np.array_equal(gs[m], os_[m]), np.nonzero(m & (gs != os_))[0][:10]
    assert np.array_equal(g["ndf"][m], o["ndf"][m])
    assert np.array_equal(g["q"][m], o["q"][m])
    return summary


def tangent_frame_cov(C, p, kind):
    """[N,6,6] covariance expressed in the 5 surface coordinates (two in-surface
    position directions, ipt, phi, theta), which removes the normal null vector."""
    N = C.shape[0]
    B = np.zeros((N, 6, 5))
    ph = np.arctan2(p[:, 1], p[:, 0])
    bar = kind == 0
    B[bar, 0, 0] = -np.sin(ph[bar])
    B[bar, 1, 0] = np.cos(ph[bar])
    B[bar, 2, 1] = 1.0
    B[~bar, 0, 0] = 1.0
    B[~bar, 1, 1] = 1.0
    B[:, 3, 2] = B[:, 4, 3] = B[:, 5, 4] = 1.0
    return np.einsum("nia,nij,njb->nab", B, C, B)


def cov_rel_error(Cg, Co):
    """|dC_ab| / sqrt(C_aa C_bb) (correlation units) of two [N,k,k] covariances."""
    d = np.sqrt(np.abs(np.einsum("naa->na", Co)))
    return np.abs(Cg - Co) / (d[:, :, None] * d[:, None, :] + 1e-300)


def sym_unpack(packed_rows):
    """[N, 21] packed -> [N, 6, 6]."""
    N = packed_rows.shape[0]
    M = np.zeros((N, 6, 6))
    k = 0
    for i in range(6):
        for j in range(i + 1):
            M[:, i, j] = packed_rows[:, k]
            M[:, j, i] = packed_rows[:, k]
            k += 1
    return M




# ---- backward fit ------------------------------------------------------------------

BACKWARD_SCALE = 100.0   # covariance scale at the start of the backward pass
IL = [(i, j) for i in range(6) for j in range(i + 1)]


def pack21(C):
    return np.stack([C[:, i, j] for i, j in IL])


def unpack21(P):
    n = P.shape[1]
    M = np.zeros((n, 6, 6))
    for k, (i, j) in enumerate(IL):
        M[:, i, j] = M[:, j, i] = P[k]
    return M


def outputs_np(out):
    return dict(p=out["state"].double().cpu().numpy().T, C=unpack21(out["cov"].double().cpu().numpy()),
                q=out["charge"].cpu().numpy().astype(np.float64), chi2=out["chi2"].double().cpu().numpy(),
                ndf=out["ndf"].cpu().numpy(), status=out["status"].cpu().numpy().astype(np.int64))


def oracle_backward(ev, dtype, fwd, hit_pos=None, state_round=None, state_jitter=None):
    hp = rounded(ev.hit_pos, dtype) if hit_pos is None else np.asarray(hit_pos, np.float64)
    b = O.backward_fit(torch.tensor(fwd["p"]), torch.tensor(fwd["C"]), torch.tensor(fwd["q"]),
                       torch.tensor(fwd["status"]), ev.hit_offsets, ev.hit_layer, ev.hit_valid, torch.tensor(hp),
                       rounded(ev.hit_cov, dtype), ev.geometry, cov_scale=BACKWARD_SCALE, state_round=state_round,
                       state_jitter=state_jitter)
    return dict(p=b["p"].numpy(), C=b["C"].numpy(), q=b["q"].numpy(), chi2=b["chi2"].numpy(), ndf=b["ndf"].numpy(),
                status=b["status"].numpy())


def gpu_backward(c, kf, ev, dtype, fwd, use_status=True, max_len=26):
    """The GPU backward pass from a forward result given as numpy arrays."""
    dev = c.device
    t = kf.event_tensors(ev, dtype, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    f = dict(state=torch.tensor(np.ascontiguousarray(fwd["p"].T), dtype=dtype, device=dev),
             cov=torch.tensor(np.ascontiguousarray(pack21(fwd["C"])), dtype=dtype, device=dev),
             charge=torch.tensor(fwd["q"].astype(np.int8), device=dev),
             status=torch.tensor(fwd["status"].astype(np.int32), device=dev))
    out = c.backward_fit(f, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom,
                         cov_scale=BACKWARD_SCALE, max_len=max_len, use_status=use_status)
    torch.cuda.synchronize()
    return outputs_np(out)


def backward_probes(ev, dtype, run, ref, tol, seed=99):
    """Tracks whose oracle result moves by more than half the tolerance under
    the rounding-level probes (see the module docstring); run(hit_pos=...,
    state_round=...) is the oracle computation being probed."""
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
        o2 = run(**kw)
        ep = param_error(o2["p"], ref["p"]).max(axis=1)
        ec = chi2_error(o2["chi2"], ref["chi2"])
        bad |= (ep > 0.5 * tol[0]) | (ec > 0.5 * tol[1]) | (o2["status"] != ref["status"])
    return bad


def rounded_forward(o, dtype):
    return dict(p=rounded(o["p"], dtype), C=rounded(o["C"], dtype), q=o["q"], status=o["status"])


# ---- smoothing ------------------------------------------------------------------------

def first_valid(ev):
    off = ev.hit_offsets
    return np.array([int(np.argmax(ev.hit_valid[off[t]:off[t + 1]])) for t in range(ev.n_tracks)])


def forward_checkpoints(ev, rec, dtype, max_len):
    """The seg = 1 checkpoints the GPU smoother reads, from the oracle forward
    fit's recorded filtered states (rounded to dtype): slot m of track t holds
    the filtered state after entry k0_t + m."""
    n = ev.n_tracks
    nseg = max(1, max_len - 1)
    ck = np.zeros((28, nseg, n))
    off, lens, k0 = ev.hit_offsets, ev.lengths(), first_valid(ev)
    pe, Ce, qe = rec["pe"].numpy(), rec["Ce"].numpy(), rec["qe"].numpy()
    for t in range(n):
        for m in range(min(lens[t] - k0[t] - 1, nseg)):
            e = off[t] + k0[t] + m
            ck[:6, m, t] = pe[e]
            ck[6:27, m, t] = [Ce[e][i, j] for i, j in [(i, j) for i in range(6) for j in range(i + 1)]]
            ck[27, m, t] = qe[e]
    return rounded(ck.reshape(28, nseg * n), dtype)


def oracle_forward_recorded(ev, dtype, seed_mode, hit_pos=None, state_round=None, state_jitter=None):
    hp = rounded(ev.hit_pos, dtype) if hit_pos is None else np.asarray(hit_pos, np.float64)
    sp, sC, sq, _ = O.make_seeds(ev.hit_offsets, ev.hit_valid, hp, ev.geometry.bz, mode=seed_mode)
    return O.fit_tracks(sp, sC, sq, ev.hit_offsets, ev.hit_layer, ev.hit_valid, torch.tensor(hp),
                        rounded(ev.hit_cov, dtype), ev.geometry, state_round=state_round, state_jitter=state_jitter,
                        record=True)


def oracle_smooth(ev, dtype, rec, hit_pos=None, state_round=None, state_jitter=None):
    """Oracle smoothing from the recorded forward fit `rec`, its inputs rounded to dtype."""
    hp = rounded(ev.hit_pos, dtype) if hit_pos is None else np.asarray(hit_pos, np.float64)
    r = lambda x: torch.tensor(rounded(x.numpy(), dtype))
    return O.backward_fit(r(rec["p"]), r(rec["C"]), rec["q"], rec["status"], ev.hit_offsets, ev.hit_layer,
                          ev.hit_valid, torch.tensor(hp), rounded(ev.hit_cov, dtype), ev.geometry,
                          cov_scale=BACKWARD_SCALE, state_round=state_round, state_jitter=state_jitter,
                          smooth_from=dict(pe=r(rec["pe"]), Ce=r(rec["Ce"])))


def gpu_smooth(c, kf, ev, dtype, rec, max_len=26):
    dev = c.device
    t = kf.event_tensors(ev, dtype, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    r = lambda x: rounded(x.numpy(), dtype)
    fwd = dict(state=torch.tensor(np.ascontiguousarray(r(rec["p"]).T), dtype=dtype, device=dev),
               cov=torch.tensor(np.ascontiguousarray(pack21(r(rec["C"]))), dtype=dtype, device=dev),
               charge=torch.tensor(rec["q"].numpy().astype(np.int8), device=dev),
               status=torch.tensor(rec["status"].numpy().astype(np.int32), device=dev))
    ck = torch.tensor(forward_checkpoints(ev, rec, dtype, max_len), dtype=dtype, device=dev)
    out, sm = c.smooth_tracks(fwd, ck, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"],
                              geom, cov_scale=BACKWARD_SCALE, max_len=max_len)
    torch.cuda.synchronize()
    return outputs_np(out), sm["state"].double().cpu().numpy(), sm["cov"].double().cpu().numpy()


def per_entry(ev, sm_state):
    """GPU smoothed states [6, max_len, n] -> [n_hits, 6] by CSR entry."""
    off, lens = ev.hit_offsets, ev.lengths()
    t = np.repeat(np.arange(ev.n_tracks), lens)
    r = np.arange(ev.n_hits) - off[t]
    return sm_state[:, r, t].T


def smooth_errors(ev, ps_a, ps_b):
    """Per-track maximum over entries of the scaled parameter error (NaN where either is NaN)."""
    ep = param_error(ps_a, ps_b).max(axis=1)
    ep = np.where(np.isnan(ep), 0.0, ep)
    return np.maximum.reduceat(ep, ev.hit_offsets[:-1]) if ev.n_hits else np.zeros(ev.n_tracks)
