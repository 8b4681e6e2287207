"""Pin for the oracle gradient (reverse-mode autodiff through the oracle fit):
central finite differences of the oracle's summed chi2 with respect to the seed
state, hit positions and per-layer alignment offsets.  Steps balance truncation
and rounding: 1e-6 cm for hits and offsets (large, strongly non-linear
sensitivities, e.g. a track whose curvature passes near zero), 1e-4 cm for the
seed position and 1e-5 for 1/pT and the angles (small sensitivities through
the diffuse prior, where rounding in the summed chi2 dominates)."""
import numpy as np
import torch

from oracle import kf_oracle as O
from toygen import generate, workloads

DT = torch.float64


def test_gradient_matches_central_differences():
    wl = workloads()["align20"]
    ev = generate(wl, 4)
    g = wl.geometry
    sp, sC, sq, _ = O.make_seeds(ev.hit_offsets, ev.hit_valid, ev.hit_pos, g.bz)
    align = torch.tensor(ev.align_true) * 0.5
    w = torch.tensor([1.0, 0.5, 2.0, 1.5], dtype=DT)
    loss, gs, gh, ga, _ = O.fit_gradients(sp, sC, sq, ev.hit_offsets, ev.hit_layer, ev.hit_valid, ev.hit_pos,
                                          ev.hit_cov, g, align=align, weights=w)

    def L(sp_, hp_, al_):
        o = O.fit_tracks(sp_, sC, sq, ev.hit_offsets, ev.hit_layer, ev.hit_valid, hp_, ev.hit_cov, g, align=al_)
        return float((w * o["chi2"]).sum())

    hp = torch.tensor(ev.hit_pos)
    steps = [1e-4, 1e-4, 1e-4, 1e-5, 1e-5, 1e-5]
    for t in range(4):
        for j in range(6):
            d = torch.zeros_like(sp); d[t, j] = steps[j]
            fd = (L(sp + d, hp, align) - L(sp - d, hp, align)) / (2 * steps[j])
            assert abs(fd - float(gs[t, j])) <= 2e-5 * max(1.0, abs(fd)), (t, j, fd, float(gs[t, j]))
    rng = np.random.default_rng(0)
    for e in rng.choice(ev.n_hits, 12, replace=False):
        for c in range(3):
            d = torch.zeros_like(hp); d[c, e] = 1e-6
            fd = (L(sp, hp + d, align) - L(sp, hp - d, align)) / 2e-6
            assert abs(fd - float(gh[c, e])) <= 2e-5 * max(1.0, abs(fd)), (e, c, fd, float(gh[c, e]))
    for lay in (0, 5, 12, 19):
        for c in range(2):
            d = torch.zeros_like(align); d[c, lay] = 1e-6
            fd = (L(sp, hp, align + d) - L(sp, hp, align - d)) / 2e-6
            assert abs(fd - float(ga[c, lay])) <= 2e-5 * max(1.0, abs(fd)), (lay, c, fd, float(ga[c, lay]))
