"""Invariants of the oracle's covariance after every update: symmetric, and
positive definite on the directions a state on its surface can move in.

A state on a detector surface has five degrees of freedom, so after a
propagation its 6x6 covariance has the surface normal as a null vector and a
strict 6x6 positive-definiteness check cannot hold.  The check is made in
the surface's own frame, built here from the geometry alone (barrel: the
transverse tangent (-y, x)/R and z; disk: x and y; then 1/pT, phi, theta):
with B that 6x5 basis, B^T C B must have a Cholesky factor after every entry
of every track, and the normal n must satisfy |n^T C n| <= 1e-9 tr(C_pos)
after every propagated entry (the seed entry is not propagated: there the
full 6x6 covariance is positive definite instead).  The frame is taken at
the predicted crossing, where the propagation made the normal a null
vector: the update keeps that null vector (n^T K = (C n)^T H^T S^-1 = 0),
while it moves the position along the tangent plane, so the normal at the
filtered position is tilted against it by the update's step over R."""
import numpy as np
import pytest
import torch

from oracle import kf_oracle as O
from toygen import generate, workloads

DT = torch.float64


def _frames(pos_xyz, kind):
    """[m, 6, 5] surface frames and [m, 6] normals from positions and kinds."""
    m = pos_xyz.shape[0]
    x, y = pos_xyz[:, 0], pos_xyz[:, 1]
    r = torch.sqrt(x * x + y * y)
    bar = torch.as_tensor(kind) == 0
    B = torch.zeros(m, 6, 5, dtype=DT)
    n = torch.zeros(m, 6, dtype=DT)
    B[:, 0, 0] = torch.where(bar, -y / r, torch.ones_like(r))
    B[:, 1, 0] = torch.where(bar, x / r, torch.zeros_like(r))
    B[:, 2, 1] = torch.where(bar, torch.ones_like(r), torch.zeros_like(r))
    B[:, 1, 1] = torch.where(bar, torch.zeros_like(r), torch.ones_like(r))
    B[:, 3, 2] = B[:, 4, 3] = B[:, 5, 4] = 1.0
    n[:, 0] = torch.where(bar, x / r, torch.zeros_like(r))
    n[:, 1] = torch.where(bar, y / r, torch.zeros_like(r))
    n[:, 2] = torch.where(bar, torch.zeros_like(r), torch.ones_like(r))
    return B, n


@pytest.mark.parametrize("name,mode", [("barrel10", O.SEED_FIRST_THREE), ("mixed26", 1)])
def test_covariance_is_positive_definite_on_the_surface_after_every_update(name, mode):
    wl = workloads()[name]
    ev = generate(wl, 400)
    g = wl.geometry
    sp, sC, sq, _ = O.make_seeds(ev.hit_offsets, ev.hit_valid, ev.hit_pos, g.bz, mode=mode)
    fo = O.fit_tracks(sp, sC, sq, ev.hit_offsets, ev.hit_layer, ev.hit_valid, torch.tensor(ev.hit_pos), ev.hit_cov,
                      g, record=True)
    reached = torch.isfinite(fo["pe"]).all(dim=1)
    e = torch.nonzero(reached)[:, 0]
    assert e.numel() > 0.9 * ev.n_hits
    C = fo["Ce"][e]
    # symmetric: exactly after an update (it symmetrises), to rounding after
    # a hole (propagation and material only)
    upd = torch.as_tensor(ev.hit_valid[e.numpy()] == 1)
    assert torch.equal(C[upd], C[upd].transpose(1, 2))
    sd0 = torch.sqrt(torch.diagonal(C, dim1=1, dim2=2).abs())
    asym = (C - C.transpose(1, 2)).abs() / (sd0[:, :, None] * sd0[:, None, :] + 1e-300)
    assert float(asym.max()) < 1e-12
    lay = ev.hit_layer[e.numpy()]
    kind = torch.as_tensor(g.kind[lay].astype(np.int64))
    # predicted crossing of every entry whose previous entry was reached: the
    # previous filtered state carried to this entry's layer
    en = e.numpy()
    prev_ok = np.zeros(en.size, bool)
    prev_ok[1:] = (en[1:] - 1 == en[:-1]) & np.isin(en[1:], ev.hit_offsets[:-1], invert=True)
    at = torch.as_tensor(np.nonzero(prev_ok)[0])
    same = torch.as_tensor(ev.hit_layer[en[at] - 1] == ev.hit_layer[en[at]])
    pp, _, _, st = O.propagate(fo["pe"][e[at] - 1], fo["Ce"][e[at] - 1], fo["qe"][e[at] - 1], kind[at],
                               torch.as_tensor(g.pos[lay[at]], dtype=DT), torch.as_tensor(g.x_over_x0[lay[at]]), g,
                               same=same)
    assert int((st & O.NO_CROSSING).sum()) == 0
    where = fo["pe"][e][:, :3].clone()
    where[at] = pp[:, :3]
    B, nv = _frames(where, kind)
    C5 = B.transpose(1, 2) @ C @ B
    # scale to unit diagonal so that the factorisation tests the shape, not the units
    d = torch.sqrt(torch.diagonal(C5, dim1=1, dim2=2))
    assert (d > 0).all()
    _, info = torch.linalg.cholesky_ex(C5 / (d[:, :, None] * d[:, None, :]))
    assert int((info != 0).sum()) == 0
    # first reached entry of each track: the seed entry (not propagated)
    first = np.full(ev.n_tracks, -1)
    track_of = np.searchsorted(ev.hit_offsets, en, side="right") - 1
    for t, x in zip(track_of[::-1], en[::-1]):
        first[t] = x
    is_first = en == first[track_of]
    assert np.array_equal(prev_ok, ~is_first)
    nn = torch.einsum("ni,nij,nj->n", nv, C, nv)
    trp = C[:, 0, 0] + C[:, 1, 1] + C[:, 2, 2]
    prop = torch.as_tensor(~is_first)
    assert (nn[prop].abs() <= 1e-9 * trp[prop]).all(), float((nn[prop].abs() / trp[prop]).max())
    _, info6 = torch.linalg.cholesky_ex(C[torch.as_tensor(is_first)])
    assert int((info6 != 0).sum()) == 0


def test_the_check_fails_on_a_broken_covariance():
    """The check above is sharp: a covariance with one negative direction on
    the surface, or a non-zero normal variance, is caught."""
    pos = torch.tensor([[3.0, 4.0, 1.0]], dtype=DT)
    B, nv = _frames(pos, torch.tensor([0]))
    A = torch.randn(5, 5, dtype=DT, generator=torch.Generator().manual_seed(1))
    good5 = A @ A.T + 0.1 * torch.eye(5, dtype=DT)
    C = B[0] @ good5 @ B[0].T
    C5 = B.transpose(1, 2) @ C[None] @ B
    assert int(torch.linalg.cholesky_ex(C5)[1][0]) == 0
    assert float(nv[0] @ C @ nv[0]) < 1e-12
    bad5 = good5 - 2.0 * float(torch.linalg.eigvalsh(good5)[0]) * torch.outer(
        torch.linalg.eigh(good5)[1][:, 0], torch.linalg.eigh(good5)[1][:, 0])
    Cb = B[0] @ bad5 @ B[0].T
    assert int(torch.linalg.cholesky_ex(B.transpose(1, 2) @ Cb[None] @ B)[1][0]) != 0
    Cn = C + 1e-3 * torch.outer(nv[0], nv[0])
    assert float(nv[0] @ Cn @ nv[0]) > 1e-9 * float(Cn[0, 0] + Cn[1, 1] + Cn[2, 2])
