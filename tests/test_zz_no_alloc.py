"""The allocation-free adjoint entry point (kf_fit_adjoint_noalloc, through
the C interface) against kf_fit_adjoint on the same inputs.  It runs the
same reverse kernel with the alignment reduction's block partials in the
library's fixed device scratch instead of the context's workspace, and
recomputes each state inside the reverse kernel instead of reading it from
the refill kernel's buffer: the same forward steps compiled in two kernels,
which may round differently in the last bit.  So the outputs are held to
the adjoint's own tolerances (those it meets against the FP64 oracle, per
track, relative L2): FP64 1e-6 (hits), 1e-5 (seed), 1e-8 (alignment); FP32
5e-2 / 1e-1 / 2e-3 with medians below 1e-3.  Every output element must be
written.  Two calls in a row on one context, the second with a smaller batch
(the scratch keeps the first call's partials, which the second must not
read), in FP32 and FP64; and a batch beyond the scratch's size is refused
before any device work."""
import sys

import numpy as np
import pytest
import torch

from toygen import generate, workloads

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


def _inputs(ctx, kf, ev, dt, seg):
    dev = ctx.device
    t = kf.event_tensors(ev, dt, dev)
    geom = kf.Geometry.from_toy(ev.geometry)
    n = ev.n_tracks
    max_len = int(ev.lengths().max())
    seeds = (torch.empty(6, n, dtype=dt, device=dev), torch.empty(21, n, dtype=dt, device=dev),
             torch.empty(n, dtype=torch.int8, device=dev))
    ck = torch.empty(28, n * kf.n_checkpoint_segments(max_len, seg), dtype=dt, device=dev)
    al = torch.as_tensor(np.asarray(ev.align_true) * 0.5, device=dev).to(dt).contiguous()
    out = ctx.seed_fit_tracks(t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom, 0,
                              align=al, seeds=seeds, checkpoints=ck, seg=seg, max_len=max_len)
    w = torch.linspace(0.5, 1.5, n, dtype=dt, device=dev)
    args = (*seeds, t["hit_offsets"], t["hit_layer"], t["hit_valid"], t["hit_pos"], t["hit_cov"], geom, ck, seg,
            max_len, out["status"])
    return args, dict(align=al, dL_dchi2=w)


def _close(ev, ref, got, dt):
    """Per-track relative L2 differences of the seed and hit gradients, and
    of the alignment gradient, within the adjoint's tolerances."""
    r = [x.double().cpu().numpy() for x in ref]
    g = [x.double().cpu().numpy() for x in got]
    es = np.linalg.norm(g[0] - r[0], axis=0) / np.maximum(np.linalg.norm(r[0], axis=0), 1e-300)
    off = ev.hit_offsets
    eh = np.array([np.linalg.norm(g[1][:, off[t]:off[t + 1]] - r[1][:, off[t]:off[t + 1]])
                   / max(np.linalg.norm(r[1][:, off[t]:off[t + 1]]), 1e-300) for t in range(ev.n_tracks)])
    ea = np.linalg.norm(g[2] - r[2]) / max(np.linalg.norm(r[2]), 1e-300)
    say("  seed max %.2e median %.2e; hits max %.2e median %.2e; align %.2e"
        % (es.max(), np.median(es), eh.max(), np.median(eh), ea))
    if dt == torch.float64:
        assert es.max() <= 1e-5 and eh.max() <= 1e-6 and ea <= 1e-8, (es.max(), eh.max(), ea)
    else:
        assert es.max() <= 1e-1 and eh.max() <= 5e-2 and ea <= 2e-3, (es.max(), eh.max(), ea)
        assert np.median(es) <= 1e-3 and np.median(eh) <= 1e-3, (np.median(es), np.median(eh))


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_noalloc_adjoint_equals_adjoint_on_two_calls(kf, dt):
    ctx = kf.Context(0)
    try:
        wl = workloads()["align20"]
        for n, seg in ((6000, 5), (1500, 3)):      # the second call is smaller
            say("noalloc adjoint", dt, "n", n, "seg", seg)
            ev = generate(wl, n)
            args, kw = _inputs(ctx, kf, ev, dt, seg)
            ref = ctx.fit_adjoint(*args, **kw)
            # outputs prefilled with NaN: every element must be written
            pre = tuple(torch.full_like(r, float("nan")) for r in ref)
            got = ctx.fit_adjoint(*args, **kw, no_alloc=True, out=pre)
            torch.cuda.synchronize()
            for x in got:
                assert torch.isfinite(x).all()
            _close(ev, ref, got, dt)
            assert torch.isfinite(got[2]).all()
            assert float(got[2].abs().sum()) > 0.0
    finally:
        ctx.close()


def test_noalloc_adjoint_refuses_a_batch_beyond_its_scratch(kf):
    """n_hits above the fixed scratch's limit is KF_ERR_ARG before any device
    work (the pointers are never read: validation fails first)."""
    ctx = kf.Context(0)
    try:
        g = kf.Geometry([0] * 3, [4.0, 5.0, 6.0], [-150.0] * 3, [150.0] * 3, [0.02] * 3)
        P = 0x1000
        lib = kf.lib()
        n_hits = (1 << 23) + 1     # FP64 limit + 1
        rc = lib.kf_fit_adjoint_noalloc(ctx.handle, kf.KF_F64, 10, 10, P, P, P, P, P, P, n_hits, P, P,
                                        kf.ctypes.byref(g.struct), None, P, 1, 3, None, P, P, P, P, None)
        assert rc == kf.KF_ERR_ARG
        assert "scratch" in lib.kf_last_error().decode()
    finally:
        ctx.close()
