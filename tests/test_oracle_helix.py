"""Pins for the oracle's helix and crossing solve (propagation step).

The helix is checked against an independent numerical integration of the
Lorentz force, and the crossing against the surface equation and a brute-force
scan for the first root."""
import math

import numpy as np
import torch

from oracle import kf_oracle as O

BZ = 3.8


def _rk4_lorentz(pos, mom, q, length, h=0.01):
    """Integrate dx/dl = t, dp/dl = q c_B (t x B) with RK4 over 3-D path length."""
    def f(x, p):
        pm = np.linalg.norm(p, axis=1, keepdims=True)
        t = p / pm
        B = np.array([0.0, 0.0, BZ])
        dp = (q[:, None] * O.C_LIGHT) * np.cross(t, B)
        return t, dp
    n_steps = np.ceil(length / h).astype(int)
    hh = length / n_steps
    x, p = pos.copy(), mom.copy()
    for i in range(n_steps.max()):
        act = i < n_steps
        hs = np.where(act, hh, 0.0)[:, None]
        k1x, k1p = f(x, p)
        k2x, k2p = f(x + 0.5 * hs * k1x, p + 0.5 * hs * k1p)
        k3x, k3p = f(x + 0.5 * hs * k2x, p + 0.5 * hs * k2p)
        k4x, k4p = f(x + hs * k3x, p + hs * k3p)
        x = x + hs / 6.0 * (k1x + 2 * k2x + 2 * k3x + k4x)
        p = p + hs / 6.0 * (k1p + 2 * k2p + 2 * k3p + k4p)
    return x, p


def _random_states(n, seed, rmax=30.0):
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.0, rmax, n)
    a = rng.uniform(-math.pi, math.pi, n)
    p = np.stack([r * np.cos(a), r * np.sin(a), rng.uniform(-50, 50, n),
                  1.0 / np.exp(rng.uniform(np.log(0.5), np.log(10.0), n)),
                  rng.uniform(-math.pi, math.pi, n), rng.uniform(0.4, math.pi - 0.4, n)], axis=1)
    q = np.where(rng.uniform(size=n) < 0.5, 1.0, -1.0)
    return torch.tensor(p), torch.tensor(q)


def test_helix_matches_lorentz_force_integration():
    p, q = _random_states(12, 1)
    s = torch.tensor(np.random.default_rng(2).uniform(1.0, 80.0, 12))
    out = O.helix_at(p, q, s, BZ).numpy()
    pn = p.numpy()
    pt = 1.0 / pn[:, 3]
    mom = np.stack([pt * np.cos(pn[:, 4]), pt * np.sin(pn[:, 4]), pt / np.tan(pn[:, 5])], axis=1)
    length = s.numpy() / np.sin(pn[:, 5])
    x, pm = _rk4_lorentz(pn[:, :3], mom, q.numpy(), length)
    assert np.abs(out[:, :3] - x).max() < 1e-8
    phi_rk = np.arctan2(pm[:, 1], pm[:, 0])
    dphi = np.angle(np.exp(1j * (out[:, 4] - phi_rk)))
    assert np.abs(dphi).max() < 1e-9
    # pT and theta conserved by both
    assert np.allclose(np.hypot(pm[:, 0], pm[:, 1]), pt, rtol=1e-10)


def test_positive_charge_turns_clockwise():
    p = torch.tensor([[0.0, 0.0, 0.0, 1.0, 0.0, math.pi / 2]])
    out = O.helix_at(p, torch.tensor([1.0]), torch.tensor([1.0]), BZ)
    assert out[0, 4] < 0 and out[0, 1] < 0


def test_barrel_crossing_on_surface_and_first_root():
    p, q = _random_states(64, 3, rmax=20.0)
    R = 25.0 + 10.0 * torch.rand(64, dtype=torch.float64, generator=torch.Generator().manual_seed(4))
    s, ok = O.crossing_barrel(p, q, R, BZ)
    h = O.helix_at(p, q, s, BZ)
    r = torch.hypot(h[:, 0], h[:, 1])
    assert ok.any()
    assert (r[ok] - R[ok]).abs().max() < 1e-9
    # brute-force scan of r(s)^2 - R^2 for its first sign change
    for i in torch.nonzero(ok)[:, 0].tolist():
        grid = torch.linspace(1e-4, float(s[i]) * 1.5 + 1.0, 20001, dtype=torch.float64)
        hh = O.helix_at(p[i:i + 1].expand(grid.shape[0], 6), q[i:i + 1].expand(grid.shape[0]), grid, BZ)
        f = hh[:, 0] ** 2 + hh[:, 1] ** 2 - float(R[i]) ** 2
        ch = torch.nonzero(torch.sign(f[1:]) != torch.sign(f[:-1]))[:, 0]
        first = float(grid[ch[0]])
        step = float(grid[1] - grid[0])
        assert abs(first - float(s[i])) <= 1.01 * step


def test_barrel_crossing_unreachable():
    # pT = 0.5 GeV: 2 rho = 87.8 cm; from the origin r = 100 cannot be reached
    p = torch.tensor([[0.0, 0.0, 0.0, 2.0, 0.3, 1.2]])
    s, ok = O.crossing_barrel(p, torch.tensor([1.0]), 100.0, BZ)
    assert not bool(ok[0])
    s, ok = O.crossing_barrel(p, torch.tensor([1.0]), 80.0, BZ)
    assert bool(ok[0])


def test_looper_second_crossing():
    # starting on r = 30 heading inwards-tangentially: the first crossing of
    # r = 30 along the path is the re-crossing, not s = 0
    p = torch.tensor([[30.0, 0.0, 0.0, 1.0, math.pi / 2 + 0.3, 1.2]])
    s, ok = O.crossing_barrel(p, torch.tensor([-1.0]), 30.0, BZ, same=torch.tensor([True]))
    assert bool(ok[0]) and float(s[0]) > 1.0
    h = O.helix_at(p, torch.tensor([-1.0]), s, BZ)
    assert abs(math.hypot(float(h[0, 0]), float(h[0, 1])) - 30.0) < 1e-9


def test_disk_crossing():
    p, q = _random_states(32, 5)
    Z = torch.full((32,), 120.0, dtype=torch.float64)
    s, ok = O.crossing_disk(p, Z)
    h = O.helix_at(p, q, s, BZ)
    assert (h[ok, 2] - 120.0).abs().max() < 1e-10
    fwd = torch.cos(p[:, 5]) > 0
    assert bool((ok == fwd).all())


def test_surface_just_behind_is_reached_backwards():
    # an estimate that overshot r = 7 by 50 um (different layer): short backward step
    p = torch.tensor([[7.005, 0.0, 0.0, 0.2, 0.05, 1.0]], dtype=torch.float64)
    s, ok = O.crossing_barrel(p, torch.tensor([1.0]), 7.0, BZ)
    assert bool(ok[0]) and -0.01 < float(s[0]) < 0.0
    h = O.helix_at(p, torch.tensor([1.0]), s, BZ)
    assert abs(math.hypot(float(h[0, 0]), float(h[0, 1])) - 7.0) < 1e-10
    # the same state asked to re-cross a layer it sits on goes round instead
    p2 = torch.tensor([[7.0, 0.0, 0.0, 2.0, 1.2, 1.0]], dtype=torch.float64)
    s2, ok2 = O.crossing_barrel(p2, torch.tensor([1.0]), 7.0, BZ, same=torch.tensor([True]))
    assert bool(ok2[0]) and float(s2[0]) > 1.0
    # disks: a plane 0.5 cm behind in z (0.15 cm of transverse path) is reached
    # backwards, one 5.5 cm behind (1.7 cm of path) is not
    p3 = torch.tensor([[5.0, 0.0, 30.5, 0.2, 0.1, 0.3]], dtype=torch.float64)
    s3, ok3 = O.crossing_disk(p3, torch.tensor([30.0], dtype=torch.float64))
    assert bool(ok3[0]) and -1.0 < float(s3[0]) < 0
    s4, ok4 = O.crossing_disk(p3, torch.tensor([25.0], dtype=torch.float64))
    assert not bool(ok4[0])
