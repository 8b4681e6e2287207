"""Pins for the oracle's multiple-scattering process noise.

Q must equal theta0^2 J J^T where J is the derivative of (ipt, phi, theta)
with respect to two orthogonal small deflections of the momentum direction at
fixed |p|; J is obtained here by finite differences of the exact 3-D
rotation, independently of the closed-form Q."""
import math

import numpy as np
import torch

from oracle import kf_oracle as O

DT = torch.float64


def _kicked(ipt, phi, th, a, b):
    """Deflect the direction by angles a (along e_theta) and b (along e_phi)
    with |p| fixed; return (ipt', phi', theta')."""
    pmag = 1.0 / (ipt * math.sin(th))
    d = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
    e_th = np.array([math.cos(th) * math.cos(phi), math.cos(th) * math.sin(phi), -math.sin(th)])
    e_ph = np.array([-math.sin(phi), math.cos(phi), 0.0])
    v = d + math.tan(a) * e_th + math.tan(b) * e_ph
    v = v / np.linalg.norm(v)
    th2 = math.acos(v[2])
    ph2 = math.atan2(v[1], v[0])
    return np.array([1.0 / (pmag * math.sin(th2)), ph2, th2])


def test_process_noise_equals_kick_covariance():
    rng = np.random.default_rng(7)
    for _ in range(20):
        ipt = math.exp(rng.uniform(math.log(0.1), math.log(2.0)))
        phi = rng.uniform(-3, 3)
        th = rng.uniform(0.3, math.pi - 0.3)
        R = 30.0
        a = phi + rng.uniform(-0.5, 0.5)
        p = torch.tensor([[R * math.cos(a), R * math.sin(a), 5.0, ipt, phi, th]], dtype=DT)
        kind = torch.tensor([O.BARREL])
        Q, _ = O.process_noise(p, kind, torch.tensor([0.02], dtype=DT), 0.13957)
        th0, _ = O.highland_theta0(p, kind, torch.tensor([0.02], dtype=DT), 0.13957)
        h = 1e-6
        J = np.zeros((3, 2))
        for j in range(2):
            da = (h, 0.0) if j == 0 else (0.0, h)
            fp = _kicked(ipt, phi, th, *da)
            fm = _kicked(ipt, phi, th, -da[0], -da[1])
            J[:, j] = (fp - fm) / (2 * h)
        expect = float(th0[0]) ** 2 * J @ J.T
        got = Q[0, 3:, 3:].numpy()
        assert np.allclose(got, expect, rtol=1e-6, atol=1e-8 * np.abs(expect).max())
        assert np.abs(Q[0, :3, :].numpy()).max() == 0.0
        assert np.linalg.matrix_rank(got, tol=1e-12 * np.abs(got).max()) == 2


def test_highland_incidence_and_momentum_dependence():
    # at fixed |p| = 2 GeV: thicker effective layer (1/cos) at oblique incidence
    kind = torch.tensor([O.BARREL, O.BARREL])
    pm = 2.0
    th = torch.tensor([math.pi / 2, math.pi / 4], dtype=DT)
    p = torch.zeros(2, 6, dtype=DT)
    p[:, 0] = 30.0
    p[:, 3] = 1.0 / (pm * torch.sin(th))
    p[:, 5] = th
    th0, g = O.highland_theta0(p, kind, torch.tensor([0.02, 0.02], dtype=DT), 0.13957)
    assert th0[1] > th0[0] and not g.any()
    # the 45-degree angle equals the normal-incidence angle of a sqrt(2)-thicker layer
    th0c, _ = O.highland_theta0(p[:1], kind[:1], torch.tensor([0.02 * math.sqrt(2)], dtype=DT), 0.13957)
    assert abs(float(th0c[0]) - float(th0[1])) < 1e-15
    # theta0 * beta * p is independent of p for fixed x / beta^2 -> ~1/p at high p
    p2 = p.clone(); p2[:, 3] = p[:, 3] / 10.0
    th0b, _ = O.highland_theta0(p2, kind, torch.tensor([0.02, 0.02], dtype=DT), 0.13957)
    assert torch.allclose(th0b / th0, torch.full((2,), 0.1, dtype=DT), rtol=2e-2)


def test_grazing_flag():
    kind = torch.tensor([O.BARREL])
    p = torch.tensor([[30.0, 0.0, 0.0, 1.0, math.pi / 2 - 0.01, math.pi / 2]], dtype=DT)
    th0, g = O.highland_theta0(p, kind, torch.tensor([0.02], dtype=DT), 0.13957)
    assert bool(g[0]) and math.isfinite(float(th0[0]))
