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


def test_highland_angle_hand_worked_values():
    """theta0 at fixed momentum, velocity and thickness, against numbers
    worked out by hand from the PDG/Highland form
    theta0 = 13.6 MeV / (beta c p) sqrt(x) (1 + 0.038 ln(x / beta^2)):
    (a) beta = 1 (a massless probe), p = 1 GeV/c, x = 0.01 X0:
        13.6e-3 * 0.1 * (1 + 0.038 ln 0.01) = 1.36e-3 * (1 - 0.17499646)
        = 1.1220048e-3 rad;
    (b) a pion (0.13957 GeV) at p = 1 GeV/c, x = 0.02 X0: beta^2 =
        1 / (1 + 0.13957^2) = 1 / 1.01947978 = 0.98089243, beta = 0.99040013;
        13.6e-3 / 0.99040013 = 1.3731824e-2; * sqrt(0.02) = 1.9419731e-3;
        ln(0.02 / 0.98089243) = -3.8927305, * 0.038 = -0.14792376;
        theta0 = 1.9419731e-3 * 0.85207624 = 1.6547092e-3 rad;
    (c) the same pion crossing a barrel at 60 degrees from the normal
        (cos = 0.5): x = 0.04 X0; 1.3731824e-2 * 0.2 = 2.7463647e-3;
        ln(0.04 / 0.98089243) = -3.1995833, * 0.038 = -0.12158417;
        theta0 = 2.7463647e-3 * 0.87841583 = 2.4124503e-3 rad.
    The literals carry 8 digits, so they are compared to 3e-10 rad."""
    kind = torch.tensor([O.BARREL] * 3)
    p = torch.zeros(3, 6, dtype=DT)
    p[:, 0] = 25.0                       # on a barrel at phi_pos = 0
    p[:, 3] = 1.0                        # pT = 1 GeV/c at theta = pi/2: |p| = 1 GeV/c
    p[:, 5] = math.pi / 2
    p[2, 4] = math.pi / 3                # direction 60 degrees from the radial normal
    x0 = torch.tensor([0.01, 0.02, 0.02], dtype=DT)
    th0_a, _ = O.highland_theta0(p[:1], kind[:1], x0[:1], 1e-12)
    th0_bc, _ = O.highland_theta0(p[1:], kind[1:], x0[1:], 0.13957)
    assert abs(float(th0_a[0]) - 1.1220048e-3) < 3e-10
    assert abs(float(th0_bc[0]) - 1.6547092e-3) < 3e-10
    assert abs(float(th0_bc[1]) - 2.4124503e-3) < 3e-10
