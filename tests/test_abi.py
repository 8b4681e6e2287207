"""The C interface without a GPU: the library loads, exports every entry
point declared in include/kf.h, and rejects bad arguments before touching the
device (these calls return KF_ERR_ARG from host-side validation)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kf.h")

kf = pytest.importorskip("paper_2312_11728_amd.kf")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(kf_[a-z_0-9]+)\s*\(", txt, re.M)))


def test_header_declares_the_hot_path_entry_points():
    names = _declared()
    for n in ("kf_propagate", "kf_update", "kf_fit_tracks", "kf_score_hits", "kf_fit_adjoint"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = kf.lib()
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) <= set(kf.EXPORTS)


def _geom(n=3):
    return kf.Geometry([0] * n, [4.0 + i for i in range(n)], [-150.0] * n, [150.0] * n, [0.02] * n)


P = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first


def _fit_call(**over):
    args = dict(ctx=P, prec=kf.KF_F32, n=10, ld=10, seed_state=P, seed_cov=P, seed_charge=P, hit_offsets=P,
                hit_layer=P, hit_valid=P, n_hits=100, hit_pos=P, hit_cov=P, geom=ctypes.byref(_geom().struct),
                align=None, state_out=P, cov_out=P, charge_out=P, chi2=P, ndf=P, checkpoints=None, seg=1,
                max_len=26, trk_status=P, stream=None)
    g = over.pop("geometry", None)
    if g is not None:
        args["geom"] = ctypes.byref(g.struct)
    args.update(over)
    return kf.lib().kf_fit_tracks(*args.values())


@pytest.mark.parametrize("over,msg", [
    (dict(n=-1), "n = -1"),
    (dict(ld=5), "ld = 5 < n = 10"),
    (dict(prec=7), "precision 7"),
    (dict(seed_state=None), "seed_state is NULL"),
    (dict(hit_pos=None), "hit_pos is NULL"),
    (dict(trk_status=None), "trk_status is NULL"),
    (dict(n_hits=-3), "n_hits < 0"),
    (dict(checkpoints=P, seg=0), "seg = 0"),
    (dict(checkpoints=P, max_len=0), "max_len = 0"),
    (dict(ctx=None), "ctx is NULL"),
])
def test_fit_tracks_argument_validation(over, msg):
    rc = _fit_call(**over)
    assert rc == kf.KF_ERR_ARG
    assert msg in kf.lib().kf_last_error().decode()


def test_geometry_validation():
    bad = kf.Geometry([0, 2], [4.0, 5.0], [-1, -1], [1, 1], [0.02, 0.02])
    assert _fit_call(geometry=bad) == kf.KF_ERR_ARG
    assert "kind[1]" in kf.lib().kf_last_error().decode()
    bad = kf.Geometry([0], [-4.0], [-1], [1], [0.02])
    assert _fit_call(geometry=bad) == kf.KF_ERR_ARG
    bad = kf.Geometry([0], [4.0], [-1], [1], [0.02], bz=0.0)
    assert _fit_call(geometry=bad) == kf.KF_ERR_ARG
    assert "bz_tesla" in kf.lib().kf_last_error().decode()
    big = kf.Geometry([0] * 65, np.arange(65) + 4.0, [-1] * 65, [1] * 65, [0.02] * 65)
    assert _fit_call(geometry=big) == kf.KF_ERR_ARG
    assert "n_layers" in kf.lib().kf_last_error().decode()


def test_other_entry_points_validate():
    lib = kf.lib()
    g = _geom()
    assert lib.kf_propagate(P, 0, 5, 4, P, P, P, P, None, ctypes.byref(g.struct), 1, P, P, None, P, None) == kf.KF_ERR_ARG
    assert lib.kf_propagate(P, 0, 5, 5, P, P, P, None, None, ctypes.byref(g.struct), 1, P, P, None, P, None) == kf.KF_ERR_ARG
    assert "target_layer" in lib.kf_last_error().decode()
    assert lib.kf_update(P, 0, 5, 5, P, P, P, P, None, P, P, None) == kf.KF_ERR_ARG
    assert "hit_cov" in lib.kf_last_error().decode()
    assert lib.kf_make_seeds(P, 0, 5, 5, P, P, 10, P, 3.8, 2, P, P, P, P, None) == kf.KF_ERR_ARG
    assert "seed mode" in lib.kf_last_error().decode()
    assert lib.kf_set_fit_launch(P, 0, 100, 0, 4, 1, 0) == kf.KF_ERR_ARG
    assert lib.kf_set_fit_launch(P, 0, 128, 2, 4, 1, 0) == kf.KF_ERR_ARG
    assert lib.kf_set_fit_launch(P, 0, 128, 0, 4, 3, 0) == kf.KF_ERR_ARG
    assert lib.kf_set_fit_launch(P, 0, 128, 0, 4, 1, 5) == kf.KF_ERR_ARG
    assert lib.kf_reserve(P, -1, 26) == kf.KF_ERR_ARG
    g2 = ctypes.byref(g.struct)
    assert lib.kf_seed_fit_tracks(P, 0, 5, 5, 2, P, P, P, 10, P, P, g2, None, None, None, None, P, P, P, P, P,
                                  None, 1, 26, P, None) == kf.KF_ERR_ARG
    assert "seed mode" in lib.kf_last_error().decode()
    assert lib.kf_seed_fit_tracks(P, 0, 5, 5, 0, P, P, P, 10, None, P, g2, None, None, None, None, P, P, P, P, P,
                                  None, 1, 26, P, None) == kf.KF_ERR_ARG
    assert "hit_pos" in lib.kf_last_error().decode()
    assert lib.kf_seed_fit_tracks(P, 0, 0, 0, 0, None, None, None, 0, None, None, g2, None, None, None, None, None,
                                  None, None, None, None, None, 1, 26, None, None) == kf.KF_OK
    assert lib.kf_set_kernel_timing(P, -1) == kf.KF_ERR_ARG
    assert lib.kf_set_kernel_timing(P, 4097) == kf.KF_ERR_ARG
    assert "max_launches" in lib.kf_last_error().decode()
    assert lib.kf_set_kernel_timing(None, 8) == kf.KF_ERR_ARG
    assert lib.kf_fit_kernel_time(P, None, None, None) == kf.KF_ERR_ARG
    assert "total_ms" in lib.kf_last_error().decode()
    assert lib.kf_reserve(P, 10, 65) == kf.KF_ERR_ARG


def _adj_call(**over):
    args = dict(ctx=P, prec=kf.KF_F32, n=10, ld=10, seed_state=P, seed_cov=P, seed_charge=P, hit_offsets=P,
                hit_layer=P, hit_valid=P, n_hits=100, hit_pos=P, hit_cov=P, geom=ctypes.byref(_geom().struct),
                align=None, checkpoints=P, seg=4, max_len=26, dL_dchi2=None, grad_seed=P, grad_hit_pos=P,
                grad_align=None, trk_status=P, stream=None)
    args.update(over)
    return kf.lib().kf_fit_adjoint(*args.values())


@pytest.mark.parametrize("over,msg", [
    (dict(n=-1), "n = -1"),
    (dict(prec=3), "precision 3"),
    (dict(seg=0), "seg = 0"),
    (dict(max_len=65), "max_len = 65"),
    (dict(checkpoints=None), "checkpoints is NULL"),
    (dict(grad_seed=None), "grad_seed is NULL"),
    (dict(grad_hit_pos=None), "grad_hit_pos is NULL"),
    (dict(trk_status=None), "trk_status is NULL"),
    (dict(ctx=None), "ctx is NULL"),
])
def test_fit_adjoint_argument_validation(over, msg):
    assert _adj_call(**over) == kf.KF_ERR_ARG
    assert msg in kf.lib().kf_last_error().decode()


def test_fit_adjoint_empty_batch_is_a_no_op():
    assert _adj_call(n=0, ld=0, seed_state=None, grad_seed=None, grad_hit_pos=None, checkpoints=None) == kf.KF_OK


def _search_call(**over):
    nl = 3
    g = _geom(nl)
    wmin = (ctypes.c_float * nl)(*([0.01] * nl))
    wmax = (ctypes.c_float * nl)(*([2.0] * nl))
    prm = kf.KfSearchParams(6, 30.0, 5.0, 10.0, 5.0, 3, 0.003, 0.01, ctypes.cast(wmin, ctypes.c_void_p),
                            ctypes.cast(wmax, ctypes.c_void_p), ctypes.cast(wmin, ctypes.c_void_p),
                            ctypes.cast(wmax, ctypes.c_void_p), 0)
    for k in [k for k in over if k.startswith("prm_")]:
        setattr(prm, k[4:], over.pop(k))
    plan = (ctypes.c_int16 * 2)(1, 2)
    off = (ctypes.c_int32 * (nl + 1))(0, 0, 5, 10)
    args = dict(ctx=P, n=10, ld=10, seed_state=P, seed_cov=P, seed_charge=P, seed_layer=P,
                layer_plan=ctypes.cast(plan, ctypes.c_void_p), plan_len=2, geom=ctypes.byref(g.struct),
                params=ctypes.byref(prm), pool_layer_offsets=ctypes.cast(off, ctypes.c_void_p), n_pool=10,
                pool_pos=P, pool_cov=P, pool_hit_id=P, pool_module=None, cand_hits=P, cand_overlap=None,
                cand_score=P, cand_state=None, trk_status=P, stream=None)
    args.update(over)
    return kf.lib().kf_score_hits(*args.values())


@pytest.mark.parametrize("over,msg", [
    (dict(prm_beam=0), "beam = 0"),
    (dict(prm_beam=9), "beam = 9"),
    (dict(prm_chi2_max=0.0), "chi2_max"),
    (dict(prm_max_miss=-1), "max_miss"),
    (dict(plan_len=0), "plan_len = 0"),
    (dict(n_pool=11), "pool_layer_offsets"),
    (dict(seed_layer=None), "seed_layer is NULL"),
    (dict(cand_hits=None), "cand_hits is NULL"),
    (dict(n=-2), "n = -2"),
    (dict(prm_overlap=2), "overlap = 2"),
    (dict(prm_overlap=1, prm_overlap_bonus=float("nan")), "overlap_bonus"),
    (dict(prm_overlap=1, prm_overlap_bonus=5.0), "pool_module is NULL"),
])
def test_score_hits_argument_validation(over, msg):
    assert _search_call(**over) == kf.KF_ERR_ARG
    assert msg in kf.lib().kf_last_error().decode()


def test_score_hits_rejects_disk_layers_in_the_plan():
    g = kf.Geometry([0, 1, 0], [4.0, 30.0, 6.0], [-150.0, 2.0, -150.0], [150.0, 100.0, 150.0], [0.02] * 3)
    assert _search_call(geom=ctypes.byref(g.struct)) == kf.KF_ERR_ARG
    assert "not a barrel layer" in kf.lib().kf_last_error().decode()


def _backward_call(**over):
    Q = ctypes.c_void_p(0x2000)   # a second fake address (outputs distinct from inputs)
    args = dict(ctx=P, prec=kf.KF_F32, n=10, ld=10, state_in=P, cov_in=P, charge_in=P, fwd_status=P, hit_offsets=P,
                hit_layer=P, hit_valid=P, n_hits=100, hit_pos=P, hit_cov=P, geom=ctypes.byref(_geom().struct),
                cov_scale=100.0, max_len=26, state_out=Q, cov_out=Q, charge_out=Q, chi2=Q, ndf=Q, trk_status=Q,
                stream=None)
    args.update(over)
    return kf.lib().kf_backward_fit(*args.values())


@pytest.mark.parametrize("over,msg", [
    (dict(n=-1), "n = -1"),
    (dict(ld=5), "ld = 5 < n = 10"),
    (dict(prec=3), "precision 3"),
    (dict(cov_scale=0.5), "cov_scale"),
    (dict(cov_scale=float("nan")), "cov_scale"),
    (dict(cov_scale=float("inf")), "cov_scale"),
    (dict(max_len=0), "max_len = 0"),
    (dict(max_len=65), "max_len = 65"),
    (dict(n_hits=-1), "n_hits < 0"),
    (dict(state_in=None), "state_in is NULL"),
    (dict(hit_cov=None), "hit_cov is NULL"),
    (dict(ndf=None), "ndf is NULL"),
    (dict(ctx=None), "ctx is NULL"),
    (dict(state_out=P), "alias"),
    (dict(charge_out=P), "alias"),
])
def test_backward_fit_argument_validation(over, msg):
    assert _backward_call(**over) == kf.KF_ERR_ARG
    assert msg in kf.lib().kf_last_error().decode()


def test_backward_fit_empty_batch_is_a_no_op():
    assert _backward_call(n=0, ld=0, ctx=None, state_in=None) == kf.KF_OK


def _smooth_call(**over):
    Q = ctypes.c_void_p(0x2000)
    R = ctypes.c_void_p(0x3000)
    S = ctypes.c_void_p(0x4000)
    args = dict(ctx=P, prec=kf.KF_F32, n=10, ld=10, state_in=P, cov_in=P, charge_in=P, fwd_status=P,
                fwd_checkpoints=P, hit_offsets=P, hit_layer=P, hit_valid=P, n_hits=100, hit_pos=P, hit_cov=P,
                geom=ctypes.byref(_geom().struct), cov_scale=100.0, max_len=26, state_out=Q, cov_out=Q, charge_out=Q,
                chi2=Q, ndf=Q, trk_status=Q, smooth_state=R, smooth_cov=S, stream=None)
    args.update(over)
    return kf.lib().kf_smooth_tracks(*args.values())


@pytest.mark.parametrize("over,msg", [
    (dict(fwd_checkpoints=None), "needs fwd_checkpoints"),
    (dict(smooth_state=None), "needs fwd_checkpoints"),
    (dict(smooth_cov=None), "needs fwd_checkpoints"),
    (dict(smooth_cov=ctypes.c_void_p(0x3000)), "must not alias"),
    (dict(smooth_state=ctypes.c_void_p(0x2000)), "must not alias"),
    (dict(cov_scale=0.0), "cov_scale"),
    (dict(n=-2), "n = -2"),
    (dict(max_len=0), "max_len = 0"),
])
def test_smooth_tracks_argument_validation(over, msg):
    assert _smooth_call(**over) == kf.KF_ERR_ARG
    assert msg in kf.lib().kf_last_error().decode()


def _final_call(**over):
    Q = ctypes.c_void_p(0x2000)
    args = dict(ctx=P, prec=kf.KF_F32, n=10, ld=10, seed_mode=0, hit_offsets=P, hit_layer=P, hit_valid=P,
                n_hits=100, hit_pos=P, hit_cov=P, geom=ctypes.byref(_geom().struct), cov_scale=100.0, chi2_cut=30.0,
                max_reject=3, min_keep=4, max_len=26, state_out=Q, cov_out=Q, charge_out=Q, chi2=Q, ndf=Q,
                trk_status=Q, outlier=Q, hit_chi2=None, stream=None)
    args.update(over)
    return kf.lib().kf_final_fit(*args.values())


@pytest.mark.parametrize("over,msg", [
    (dict(chi2_cut=0.0), "chi2_cut"),
    (dict(chi2_cut=-1.0), "chi2_cut"),
    (dict(chi2_cut=float("nan")), "chi2_cut"),
    (dict(cov_scale=0.5), "cov_scale"),
    (dict(max_reject=-1), "max_reject"),
    (dict(max_reject=65), "max_reject"),
    (dict(min_keep=2), "min_keep"),
    (dict(seed_mode=2), "seed mode"),
    (dict(n=-1), "n = -1"),
    (dict(ld=5), "ld = 5"),
    (dict(max_len=0), "max_len = 0"),
    (dict(hit_pos=None), "hit_pos is NULL"),
    (dict(outlier=None), "outlier is NULL"),
    (dict(ctx=None), "ctx is NULL"),
])
def test_final_fit_argument_validation(over, msg):
    assert _final_call(**over) == kf.KF_ERR_ARG
    assert msg in kf.lib().kf_last_error().decode()


def test_final_fit_empty_batch_is_a_no_op():
    assert _final_call(n=0, ld=0, ctx=None, hit_offsets=None, chi2_cut=float("inf")) == kf.KF_OK


def _dedup_call(**over):
    args = dict(ctx=P, n=10, track_hits=P, hit_stride=17, n_layers=17, score=P, score_stride=1, frac=0.5, keep=P,
                dup_of=None, stream=None)
    args.update(over)
    return kf.lib().kf_remove_duplicates(*args.values())


@pytest.mark.parametrize("over,msg", [
    (dict(n=-1), "n = -1"),
    (dict(n_layers=0), "n_layers = 0"),
    (dict(n_layers=65, hit_stride=65), "n_layers = 65"),
    (dict(hit_stride=16), "hit_stride = 16"),
    (dict(score_stride=0), "score_stride = 0"),
    (dict(frac=0.0), "frac"),
    (dict(frac=1.5), "frac"),
    (dict(frac=float("nan")), "frac"),
    (dict(n=1 << 30, n_layers=2, hit_stride=2), "2^31"),
    (dict(track_hits=None), "track_hits is NULL"),
    (dict(keep=None), "keep is NULL"),
    (dict(ctx=None), "ctx is NULL"),
])
def test_remove_duplicates_argument_validation(over, msg):
    assert _dedup_call(**over) == kf.KF_ERR_ARG
    assert msg in kf.lib().kf_last_error().decode()


def test_remove_duplicates_empty_is_a_no_op():
    assert _dedup_call(n=0, ctx=None, track_hits=None) == kf.KF_OK


def test_output_dict_is_checked_before_any_launch():
    """A caller's output dict of the wrong size, type or layout is refused
    in the binding (a short buffer would be written past its end)."""
    import torch
    dev = torch.device("cpu")
    good = kf.fit_outputs(5, torch.float32, dev)
    kf._need_outputs(good, 5, torch.float32, dev)
    bad = [kf.fit_outputs(4, torch.float32, dev), kf.fit_outputs(5, torch.float64, dev),
           dict(good, ndf=torch.empty(5, dtype=torch.int64)), dict(good, cov=torch.empty(5, 21).T),
           {k: v for k, v in good.items() if k != "status"}]
    for out in bad:
        with pytest.raises(ValueError):
            kf._need_outputs(out, 5, torch.float32, dev)


def _cpu_context():
    """A binding object whose checks run on CPU tensors (no library context:
    every case below is refused before any call into the library)."""
    import torch
    c = object.__new__(kf.Context)
    c.device = torch.device("cpu")
    c.handle = None
    return c


def _smooth_inputs(n=4, nh=12, max_len=5):
    import torch
    dt = torch.float32
    fwd = kf.fit_outputs(n, dt, torch.device("cpu"))
    hits = (torch.arange(0, nh + 1, nh // n, dtype=torch.int32), torch.zeros(nh, dtype=torch.int16),
            torch.ones(nh, dtype=torch.uint8), torch.zeros(3, nh, dtype=dt), torch.zeros(6, nh, dtype=dt))
    ck = torch.zeros(28, n * (max_len - 1), dtype=dt)
    sm = dict(state=torch.zeros(6, max_len, n, dtype=dt), cov=torch.zeros(21, max_len, n, dtype=dt))
    return fwd, ck, hits, sm


def test_binding_checks_smoother_buffers_status_and_offsets():
    """smooth_tracks refuses a smoothing buffer on another device, a status
    of the wrong type or size, and every entry point refuses CSR offsets that
    do not hold n + 1 entries."""
    import torch
    c = _cpu_context()
    g = _geom(1)
    fwd, ck, hits, sm = _smooth_inputs()
    bad_sm = dict(sm, cov=torch.zeros(21, 5, 4, dtype=torch.float32, device="meta"))
    with pytest.raises(ValueError, match="smooth"):
        c.smooth_tracks(fwd, ck, *hits, g, max_len=5, smooth=bad_sm)
    with pytest.raises(TypeError, match="status"):
        c.smooth_tracks(dict(fwd, status=torch.zeros(4, dtype=torch.int64)), ck, *hits, g, max_len=5, smooth=sm)
    with pytest.raises(ValueError, match="status"):
        c.smooth_tracks(dict(fwd, status=torch.zeros(3, dtype=torch.int32)), ck, *hits, g, max_len=5, smooth=sm)
    short = (hits[0][:-1],) + hits[1:]
    with pytest.raises(ValueError, match="hit_offsets"):
        c.smooth_tracks(fwd, ck, *short, g, max_len=5, smooth=sm)
    with pytest.raises(ValueError, match="hit_offsets"):
        c.backward_fit(fwd, *short, g)
    seeds = (fwd["state"], fwd["cov"], fwd["charge"])
    with pytest.raises(ValueError, match="hit_offsets"):
        c.fit_tracks(*seeds, *short, g)
    with pytest.raises(ValueError, match="hit_offsets"):
        c.fit_adjoint(*seeds, *short, g, ck, 1, 5, fwd["status"])


def _plane_geom(n_modules=10, bz=3.8, mass=0.13957, modules=P):
    return kf.KfPlaneGeometry(n_modules, modules, bz, mass)


def _plane_fit_call(**over):
    g = over.pop("geometry", _plane_geom())
    args = dict(ctx=P, prec=kf.KF_F32, n=10, ld=10, seed_state=P, seed_cov=P, seed_charge=P, hit_offsets=P,
                hit_module=P, hit_valid=P, n_hits=100, hit_uv=P, hit_cov_uv=P,
                geom=None if g is None else ctypes.byref(g), state_out=P, cov_out=P, charge_out=P, chi2=P, ndf=P,
                trk_status=P, stream=None)
    args.update(over)
    return kf.lib().kf_fit_plane_tracks(*args.values())


@pytest.mark.parametrize("over,msg", [
    (dict(n=-1), "n = -1"),
    (dict(ld=5), "ld = 5 < n = 10"),
    (dict(prec=3), "precision 3"),
    (dict(n_hits=-1), "n_hits < 0"),
    (dict(n_hits=1 << 31), "n_hits"),
    (dict(hit_module=None), "hit_module is NULL"),
    (dict(hit_uv=None), "hit_uv is NULL"),
    (dict(seed_cov=None), "seed_cov is NULL"),
    (dict(geometry=None), "plane geometry is NULL"),
    (dict(geometry=_plane_geom(n_modules=0)), "n_modules"),
    (dict(geometry=_plane_geom(modules=None)), "modules is NULL"),
    (dict(geometry=_plane_geom(bz=0.0)), "bz_tesla"),
    (dict(geometry=_plane_geom(mass=-1.0)), "particle_mass_gev"),
])
def test_fit_plane_tracks_argument_validation(over, msg):
    assert _plane_fit_call(**over) == kf.KF_ERR_ARG
    assert msg in kf.lib().kf_last_error().decode()


def test_plane_entry_points_validate():
    lib = kf.lib()
    g = ctypes.byref(_plane_geom())
    assert lib.kf_propagate_plane(P, 0, 5, 5, P, P, P, None, g, 1, P, P, None, P, None) == kf.KF_ERR_ARG
    assert "target_module" in lib.kf_last_error().decode()
    assert lib.kf_propagate_plane(P, 0, 5, 5, P, P, P, P, None, 1, P, P, None, P, None) == kf.KF_ERR_ARG
    assert "plane geometry is NULL" in lib.kf_last_error().decode()
    assert lib.kf_update_plane(P, 1, 5, 5, P, P, P, P, P, None, g, P, P, None) == kf.KF_ERR_ARG
    assert "hit_cov_uv" in lib.kf_last_error().decode()
    assert lib.kf_update_plane(P, 0, 5, 4, P, P, P, P, P, P, g, P, P, None) == kf.KF_ERR_ARG
    assert lib.kf_plane_to_global(P, 0, 10, None, P, g, P, None) == kf.KF_ERR_ARG
    assert "module is NULL" in lib.kf_last_error().decode()
    assert lib.kf_plane_to_global(P, 0, -1, P, P, g, P, None) == kf.KF_ERR_ARG


def test_plane_entry_points_empty_batch_is_a_no_op():
    """n = 0 (n_hits = 0) returns KF_OK before any device work, with NULL arrays."""
    lib = kf.lib()
    g = ctypes.byref(_plane_geom())
    assert lib.kf_propagate_plane(P, 0, 0, 0, None, None, None, None, g, 1, None, None, None, None, None) == kf.KF_OK
    assert lib.kf_update_plane(P, 1, 0, 0, None, None, None, None, None, None, g, None, None, None) == kf.KF_OK
    assert _plane_fit_call(n=0, ld=0, seed_state=None, seed_cov=None, seed_charge=None, hit_offsets=None,
                           hit_module=None, hit_valid=None, n_hits=0, hit_uv=None, hit_cov_uv=None, state_out=None,
                           cov_out=None, charge_out=None, chi2=None, ndf=None, trk_status=None) == kf.KF_OK
    assert lib.kf_plane_to_global(P, 0, 0, None, None, g, None, None) == kf.KF_OK
