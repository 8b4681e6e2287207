"""The per-track code of the HIP path built for the host under the address
and undefined-behaviour sanitizers (tests/hostcheck): seeding and the forward
fit with checkpoints on the mixed barrel + disk detector (with alignment
offsets), the adjoint's reverse sweep with and without its state buffer,
and the forward fit over tilted modules, in FP32 and FP64.  A sanitizer
report ends the program with an error.  The FP64 results are held to the
oracle at the GPU parity tolerances; the FP32 ones, whose host math library
differs from the device's, only to a consistency bound."""
import os
import subprocess

import numpy as np
import pytest
import torch

from oracle import kf_oracle as O
from oracle import kf_plane as P
from toygen import generate, generate_planes, plane_workloads, workloads

from parity import compare_fit, oracle_fit, param_error, unpack21
from hostcheck import build as hostbuild

N_FIT, N_PLANE, SEG, MAX_LEN = 240, 240, 4, 26
TRK_BAD_INPUT = 64   # status bit of the C interface: no seed (fewer than three suitable hits)


def _write(d, name, a, dtype):
    np.ascontiguousarray(a, dtype).tofile(os.path.join(d, name))


def _pack_cols(C):
    i, j = np.tril_indices(6)
    return np.ascontiguousarray(np.asarray(C)[:, i, j].T)


@pytest.fixture(scope="module")
def case(tmp_path_factory):
    if hostbuild.hipcc() is None:
        pytest.skip("hipcc not found")
    d = str(tmp_path_factory.mktemp("hostcheck"))
    exe = hostbuild.build(os.path.join(d, "kf_host_check"))
    ev = generate(workloads()["mixed26"], N_FIT)
    g = ev.geometry
    align = ev.align_true * 0.5
    w = np.linspace(0.5, 2.0, N_FIT)
    pe = generate_planes(plane_workloads()["tilted10"], N_PLANE)
    rng = np.random.default_rng(3)
    pv = pe.hit_valid.copy()
    for t in range(N_PLANE):   # a few holes past the seeding hits
        a, b = pe.hit_offsets[t], pe.hit_offsets[t + 1]
        if rng.random() < 0.3:
            pv[rng.integers(a + 3, b)] = 0
    pe.hit_valid = pv
    pg = pe.geometry
    sp, sC, sq, _ = P.make_seeds_planes(pe.hit_offsets, pe.hit_module, pe.hit_valid, pe.hit_uv, pg.modules, pg.bz)
    meta = dict(n=N_FIT, n_hits=ev.hit_pos.shape[1], n_layers=g.n_layers, bz=g.bz, mass=g.mass, seg=SEG,
                max_len=MAX_LEN, seed_mode=1, align=1, pn=N_PLANE, pn_hits=pe.hit_uv.shape[1],
                pn_modules=pg.modules.shape[1], pbz=pg.bz, pmass=pg.mass)
    with open(os.path.join(d, "meta.txt"), "w") as f:
        for k, v in meta.items():
            f.write(f"{k} {float(v)!r}\n")
    _write(d, "hit_offsets.i32", ev.hit_offsets, np.int32)
    _write(d, "hit_layer.i16", ev.hit_layer, np.int16)
    _write(d, "hit_valid.u8", ev.hit_valid, np.uint8)
    _write(d, "hit_pos.f64", ev.hit_pos, np.float64)
    _write(d, "hit_cov.f64", ev.hit_cov, np.float64)
    _write(d, "layer_kind.i32", g.kind, np.int32)
    _write(d, "layer_pos.f64", g.pos, np.float64)
    _write(d, "layer_x0.f64", g.x_over_x0, np.float64)
    _write(d, "align.f64", align, np.float64)
    _write(d, "weights.f64", w, np.float64)
    _write(d, "p_offsets.i32", pe.hit_offsets, np.int32)
    _write(d, "p_module.i32", pe.hit_module, np.int32)
    _write(d, "p_valid.u8", pe.hit_valid, np.uint8)
    _write(d, "p_uv.f64", pe.hit_uv, np.float64)
    _write(d, "p_cov.f64", pe.hit_cov_uv, np.float64)
    _write(d, "p_table.f64", pg.modules, np.float64)
    _write(d, "p_seed_state.f64", sp.numpy().T, np.float64)
    _write(d, "p_seed_cov.f64", _pack_cols(sC.numpy()), np.float64)
    _write(d, "p_seed_charge.i8", sq.numpy(), np.int8)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=3",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    runs = {}
    for prec in ("32", "64"):
        r = subprocess.run([exe, d, prec], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, (prec, r.returncode, r.stdout[-2000:], r.stderr[-4000:])
        assert "identical" in r.stdout and "runtime error" not in r.stderr, (r.stdout, r.stderr[-4000:])
        runs[prec] = r
    return dict(dir=d, ev=ev, align=align, w=w, pe=pe, seeds=(sp, sC, sq))


def _seeded(ev):
    """Tracks the oracle can seed (three valid hits spaced as the seeding
    mode asks)."""
    return O.make_seeds(ev.hit_offsets, ev.hit_valid, ev.hit_pos, ev.geometry.bz, mode=1)[3].numpy()


def _out(case, prec, name, shape=None, dtype=np.float64):
    a = np.fromfile(os.path.join(case["dir"], f"out{prec}_{name}.bin"), dtype)
    return a if shape is None else a.reshape(shape)


def _fit_out(case, prec):
    ev = case["ev"]
    n = ev.n_tracks
    return dict(p=_out(case, prec, "state", (6, n)).T, C=unpack21(_out(case, prec, "cov", (21, n))),
                q=_out(case, prec, "charge"), chi2=_out(case, prec, "chi2"), ndf=_out(case, prec, "ndf").astype(int),
                status=_out(case, prec, "status", dtype=np.uint32).astype(np.int64),
                seed=_out(case, prec, "seed_state", (6, n)).T, seed_q=_out(case, prec, "seed_charge"))


def test_fit_fp64_matches_oracle(case):
    ev = case["ev"]
    g = _fit_out(case, "64")
    o = oracle_fit(ev, torch.float64, seed_mode=1, align=case["align"])
    # tracks without three suitable hits have no seed (flagged on both sides)
    ok = _seeded(ev)
    assert ok.mean() > 0.9
    assert np.array_equal(g["status"][~ok] & TRK_BAD_INPUT, np.full((~ok).sum(), TRK_BAD_INPUT))
    assert np.allclose(g["seed"][ok], o["seed"][ok], rtol=1e-12, atol=1e-12)
    compare_fit(g, o, 1e-8, 1e-8, mask=ok, geom=ev.geometry)


def test_adjoint_fp64_matches_oracle(case):
    ev = case["ev"]
    n, nh = ev.n_tracks, ev.hit_pos.shape[1]
    g = _fit_out(case, "64")
    gs = _out(case, "64", "grad_seed", (6, n)).T
    gh = _out(case, "64", "grad_hit", (3, nh))
    seed_cov = unpack21(_out(case, "64", "seed_cov", (21, n)))
    _, ogs, ogh, _, out = O.fit_gradients(torch.tensor(g["seed"]), torch.tensor(seed_cov), torch.tensor(g["seed_q"]),
                                          ev.hit_offsets, ev.hit_layer, ev.hit_valid, torch.tensor(ev.hit_pos),
                                          ev.hit_cov, ev.geometry, align=torch.tensor(case["align"]),
                                          weights=torch.tensor(case["w"]))
    ogs, ogh = ogs.numpy(), ogh.numpy()
    ok = _seeded(ev)
    es = np.linalg.norm(gs - ogs, axis=1) / np.maximum(np.linalg.norm(ogs, axis=1), 1e-300)
    off = ev.hit_offsets
    eh = np.array([np.linalg.norm(gh[:, off[t]:off[t + 1]] - ogh[:, off[t]:off[t + 1]])
                   / max(np.linalg.norm(ogh[:, off[t]:off[t + 1]]), 1e-300) for t in range(n)])
    assert es[ok].max() <= 1e-5 and eh[ok].max() <= 1e-6, (es[ok].max(), eh[ok].max())


def test_planes_fp64_matches_oracle(case):
    pe = case["pe"]
    pg = pe.geometry
    n = pe.n_tracks
    sp, sC, sq = case["seeds"]
    o = P.fit_plane_tracks(sp, sC, sq, pe.hit_offsets, pe.hit_module, pe.hit_valid, pe.hit_uv, pe.hit_cov_uv,
                           pg.modules, pg)
    p = _out(case, "64", "p_state", (6, n)).T
    st = _out(case, "64", "p_status", dtype=np.uint32).astype(np.int64)
    assert np.array_equal(st & ~O.FP64_FALLBACK, o["status"].numpy() & ~O.FP64_FALLBACK)
    assert np.array_equal(_out(case, "64", "p_ndf").astype(int), o["ndf"].numpy())
    assert param_error(p, o["p"].numpy()).max() <= 1e-8
    ec = np.abs(_out(case, "64", "p_chi2") - o["chi2"].numpy()) / np.maximum(np.abs(o["chi2"].numpy()), 1.0)
    assert ec.max() <= 1e-8


def test_fp32_consistent_with_fp64(case):
    """The FP32 instantiation ran the same tracks to the same outcome: equal
    statuses and charges on nearly all tracks, states within FP32-sized
    errors of the FP64 run."""
    for pre in ("", "p_"):
        s32 = _out(case, "32", pre + "status", dtype=np.uint32) & ~np.uint32(O.FP64_FALLBACK)
        s64 = _out(case, "64", pre + "status", dtype=np.uint32) & ~np.uint32(O.FP64_FALLBACK)
        assert (s32 == s64).mean() >= 0.98
        ok = (s32 == 0) & (s64 == 0)
        n = s32.shape[0]
        p32 = _out(case, "32", pre + "state", (6, n)).T
        p64 = _out(case, "64", pre + "state", (6, n)).T
        e = param_error(p32, p64).max(axis=1)[ok]
        assert np.quantile(e, 0.99) <= 1e-3, np.quantile(e, 0.99)
        assert np.isfinite(_out(case, "32", pre + "chi2")[ok]).all()
    gh = _out(case, "32", "grad_hit")
    assert np.isfinite(gh).all()
