"""Pins for the oracle's surface-to-surface transport Jacobian and the
covariance propagation: central finite differences of the full propagation
map, and the null vector that a state confined to a surface must have."""
import math

import numpy as np
import torch

from oracle import kf_oracle as O

BZ = 3.8
DT = torch.float64


def _states(n, seed):
    rng = np.random.default_rng(seed)
    r = rng.uniform(3.0, 20.0, n)
    a = rng.uniform(-math.pi, math.pi, n)
    phi = a + rng.uniform(-0.6, 0.6, n)   # moving roughly outwards
    p = np.stack([r * np.cos(a), r * np.sin(a), rng.uniform(-20, 20, n),
                  1.0 / np.exp(rng.uniform(np.log(0.7), np.log(10.0), n)), phi,
                  rng.uniform(0.5, math.pi - 0.5, n)], axis=1)
    q = np.where(rng.uniform(size=n) < 0.5, 1.0, -1.0)
    return torch.tensor(p, dtype=DT), torch.tensor(q, dtype=DT)


def _map(p, q, kind, pos):
    s, ok = O.crossing(p, q, kind, pos, BZ)
    return O.helix_at(p, q, s, BZ), ok


STEPS = torch.tensor([1e-5, 1e-5, 1e-5, 1e-6, 1e-7, 1e-7], dtype=DT)


def _fd_jacobian(p, q, kind, pos):
    n = p.shape[0]
    J = torch.zeros(n, 6, 6, dtype=DT)
    for j in range(6):
        d = torch.zeros(6, dtype=DT)
        d[j] = STEPS[j]
        fp, _ = _map(p + d, q, kind, pos)
        fm, _ = _map(p - d, q, kind, pos)
        J[:, :, j] = (fp - fm) / (2 * STEPS[j])
    return J


def _check(kind_v, pos_v, seed):
    p, q = _states(40, seed)
    n = p.shape[0]
    kind = torch.full((n,), kind_v, dtype=torch.int64)
    pos = torch.full((n,), pos_v, dtype=DT)
    if kind_v == O.DISK:
        # point every track at the disk
        p[:, 5] = torch.where(torch.tensor(pos_v) > p[:, 2], 0.6, math.pi - 0.6)
    _, ok = _map(p, q, kind, pos)
    s, _ = O.crossing(p, q, kind, pos, BZ)
    F = O.jacobian(p, q, s, kind, BZ)
    Jfd = _fd_jacobian(p, q, kind, pos)
    scale = torch.clamp(Jfd.abs(), min=1.0)
    err = ((F - Jfd).abs() / scale)[ok]
    assert ok.sum() > 20
    assert err.max() < 2e-6, float(err.max())
    return p, q, s, F, ok, kind


def test_jacobian_barrel_matches_finite_differences():
    _check(O.BARREL, 45.0, 11)


def test_jacobian_disk_matches_finite_differences():
    _check(O.DISK, 80.0, 12)


def test_null_vector_barrel():
    p, q, s, F, ok, kind = _check(O.BARREL, 45.0, 13)
    h = O.helix_at(p, q, s, BZ)
    nhat = torch.stack([h[:, 0], h[:, 1], torch.zeros_like(h[:, 0])], 1) / 45.0
    # position rows projected on the surface normal vanish for every column
    res = torch.einsum("ni,nij->nj", nhat, F[:, :3, :])
    assert res[ok].abs().max() < 1e-9
    # and the propagated covariance inherits the null vector
    A = torch.randn(p.shape[0], 6, 6, dtype=DT, generator=torch.Generator().manual_seed(0))
    C = A @ A.transpose(1, 2)
    C2 = F @ C @ F.transpose(1, 2)
    next_ = torch.cat([nhat, torch.zeros(p.shape[0], 3, dtype=DT)], 1)
    v = torch.einsum("ni,nij->nj", next_, C2)
    tr = torch.diagonal(C2, dim1=1, dim2=2).sum(1)
    assert (v.abs().max(1).values / tr)[ok].max() < 1e-11


def test_null_vector_disk():
    p, q, s, F, ok, kind = _check(O.DISK, 80.0, 14)
    assert F[ok][:, 2, :].abs().max() < 1e-10


def test_jacobian_unit_rows():
    p, q, s, F, ok, kind = _check(O.BARREL, 45.0, 15)
    e3 = torch.zeros(6, dtype=DT); e3[3] = 1
    e5 = torch.zeros(6, dtype=DT); e5[5] = 1
    assert torch.allclose(F[:, 3, :], e3.expand(F.shape[0], 6))
    assert torch.allclose(F[:, 5, :], e5.expand(F.shape[0], 6))
