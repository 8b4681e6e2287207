"""Pins for the oracle's Kalman update: a diagonal hand case, the Joseph form
against the short form, the 3-D update with a thickness term against the 2-D
update in the surface's local frame, the whole recursion against batch
Gaussian conditioning of the linearised problem, and the charge flip against
an update in signed-curvature parameters."""
import math

import numpy as np
import torch

from oracle import kf_oracle as O
from toygen import workloads, generate

DT = torch.float64


def test_diagonal_hand_case():
    c = np.array([0.5, 0.2, 0.3, 0.4, 0.01, 0.02])
    v = np.array([0.1, 0.05, 0.2])
    p = torch.tensor([[1.0, 2.0, 3.0, 0.5, 0.1, 1.0]], dtype=DT)
    C = torch.diag(torch.tensor(c, dtype=DT))[None]
    V = torch.diag(torch.tensor(v, dtype=DT))[None]
    m = torch.tensor([[1.3, 1.9, 3.4]], dtype=DT)
    p2, C2, q2, chi2, st = O.update(p, C, torch.tensor([1.0]), m, V)
    r = np.array([0.3, -0.1, 0.4])
    k = c[:3] / (c[:3] + v)
    assert np.allclose(p2[0, :3].numpy(), p[0, :3].numpy() + k * r, rtol=0, atol=1e-15)
    assert np.allclose(p2[0, 3:].numpy(), p[0, 3:].numpy(), rtol=0, atol=0)
    assert abs(float(chi2[0]) - float(np.sum(r * r / (c[:3] + v)))) < 1e-13
    assert np.allclose(np.diag(C2[0].numpy())[:3], c[:3] * v / (c[:3] + v), rtol=1e-14)
    assert np.allclose(np.diag(C2[0].numpy())[3:], c[3:], rtol=1e-14)
    assert int(st[0]) == 0 and float(q2[0]) == 1.0


def _random_spd(n, k, seed, scale=1.0):
    g = torch.Generator().manual_seed(seed)
    A = torch.randn(n, k, k, dtype=DT, generator=g) * scale
    return A @ A.transpose(1, 2) + 1e-3 * scale * scale * torch.eye(k, dtype=DT)


def test_joseph_equals_short_form_for_optimal_gain():
    n = 50
    C = _random_spd(n, 6, 1)
    V = _random_spd(n, 3, 2, 0.1)
    p = torch.zeros(n, 6, dtype=DT); p[:, 3] = 5.0
    m = torch.randn(n, 3, dtype=DT, generator=torch.Generator().manual_seed(3))
    _, C2, _, _, _ = O.update(p, C, torch.ones(n, dtype=DT), m, V)
    Cn, Vn = C.numpy(), V.numpy()
    for i in range(n):
        S = Cn[i, :3, :3] + Vn[i]
        K = Cn[i, :, :3] @ np.linalg.inv(S)
        short = Cn[i] - K @ Cn[i, :3, :]
        assert np.allclose(C2[i].numpy(), short, rtol=1e-10, atol=1e-12 * np.abs(short).max())


def test_3d_update_with_thickness_equals_2d_local_update():
    wl = workloads()["barrel20"]
    ev = generate(wl, 40)
    sp, sC, sq, _ = O.make_seeds(ev.hit_offsets, ev.hit_valid, ev.hit_pos, 3.8)
    # propagate the seeds to layer 10 (covariance acquires the normal null vector)
    kind = torch.zeros(40, dtype=torch.int64)
    pos = torch.full((40,), float(wl.geometry.pos[10]), dtype=DT)
    p, C, s, st = O.propagate(sp, sC, sq, kind, pos, torch.full((40,), 0.02, dtype=DT), wl.geometry)
    ok = st == 0
    x, y = p[:, 0], p[:, 1]
    R = torch.hypot(x, y)
    nh = torch.stack([x / R, y / R, torch.zeros_like(x)], 1)
    th = torch.stack([-y / R, x / R, torch.zeros_like(x)], 1)
    zh = torch.tensor([0.0, 0.0, 1.0], dtype=DT).expand(40, 3)
    g = torch.Generator().manual_seed(5)
    a = 0.01 * torch.randn(40, dtype=DT, generator=g)
    b = 0.03 * torch.randn(40, dtype=DT, generator=g)
    m = p[:, :3] + a[:, None] * th + b[:, None] * zh
    srp, sz, sn = 0.003, 0.01, 0.03 / math.sqrt(12)
    V = (srp ** 2 * th[:, :, None] * th[:, None, :] + sz ** 2 * zh[:, :, None] * zh[:, None, :]
         + sn ** 2 * nh[:, :, None] * nh[:, None, :])
    p3, C3, _, chi3, _ = O.update(p, C, sq, m, V)
    for i in torch.nonzero(ok)[:, 0].tolist():
        P2 = torch.stack([th[i], zh[i]]).numpy()                       # 2x3
        H2 = np.concatenate([P2, np.zeros((2, 3))], 1)                 # 2x6
        Ci = C[i].numpy()
        S2 = H2 @ Ci @ H2.T + np.diag([srp ** 2, sz ** 2])
        K2 = Ci @ H2.T @ np.linalg.inv(S2)
        r2 = np.array([float(a[i]), float(b[i])])
        p2 = p[i].numpy() + K2 @ r2
        C2 = (np.eye(6) - K2 @ H2) @ Ci
        chi2 = r2 @ np.linalg.inv(S2) @ r2
        assert abs(chi2 - float(chi3[i])) <= 1e-9 * max(1.0, chi2)
        assert np.allclose(p3[i].numpy(), p2, rtol=1e-10, atol=1e-12)
        sc = np.sqrt(np.outer(np.diag(C2), np.diag(C2))) + 1e-300
        assert np.abs((C3[i].numpy() - C2) / sc).max() < 1e-7


def test_recursion_equals_batch_conditioning():
    """Linearised problem x_k = F_k x_{k-1} + w_k, y_k = H x_k + v_k with the
    oracle's own F_k, Q_k, V_k: the filter's last state and covariance and its
    summed chi2 equal Gaussian conditioning of the stacked problem."""
    wl = workloads()["barrel10"]
    ev = generate(wl, 3)
    g = wl.geometry
    sp, sC, sq, _ = O.make_seeds(ev.hit_offsets, ev.hit_valid, ev.hit_pos, g.bz)
    H = np.concatenate([np.eye(3), np.zeros((3, 3))], 1)
    for t in range(3):
        e0, e1 = int(ev.hit_offsets[t]), int(ev.hit_offsets[t + 1])
        N = e1 - e0
        # reference trajectory (noise-free propagation of the seed) and the
        # matrices along it; the linearised model is affine about it:
        # x_k = ref_k + F_k (x_{k-1} - ref_{k-1}) + w_k
        p = sp[t:t + 1].clone(); q = sq[t:t + 1]
        Fs, Qs, Vs, refs = [], [], [], []
        for k in range(N):
            lay = int(ev.hit_layer[e0 + k])
            kind = torch.tensor([int(g.kind[lay])]); pos = torch.tensor([float(g.pos[lay])], dtype=DT)
            if k == 0:
                F = torch.eye(6, dtype=DT)[None]
                p2 = p
            else:
                s, _ = O.crossing(p, q, kind, pos, g.bz)
                F = O.jacobian(p, q, s, kind, g.bz)
                p2 = O.helix_at(p, q, s, g.bz)
            Q, _ = O.process_noise(p2, kind, torch.tensor([0.02], dtype=DT), g.mass)
            Fs.append(F[0].numpy()); Qs.append(Q[0].numpy()); refs.append(p2[0].numpy())
            Vs.append(O.unpack_sym(ev.hit_cov[:, e0 + k:e0 + k + 1], 3)[0].numpy())
            p = p2
        y = ev.hit_pos[:, e0:e0 + N].T
        m0 = sp[t].numpy()
        P0 = sC[t].numpy()

        def dev(a, b):
            d = a - b
            d[4] = math.remainder(d[4], 2 * math.pi)
            return d

        # recursive filter using the oracle's update on the affine model
        x = m0.copy(); C = P0.copy(); chi_sum = 0.0; prev = refs[0]
        for k in range(N):
            x = refs[k] + Fs[k] @ dev(x, prev)
            prev = refs[k]
            C = Fs[k] @ C @ Fs[k].T + Qs[k]
            xt, Ct, _, c2, st = O.update(torch.tensor(x[None]), torch.tensor(C[None]), q,
                                         torch.tensor(y[k][None]), torch.tensor(Vs[k][None]))
            assert int(st[0]) == 0
            x, C = xt[0].numpy(), Ct[0].numpy()
            chi_sum += float(c2[0])
        # batch: z = (x0, w_1..w_N); x_k - ref_k is linear in z - (ref_0, 0, ...)
        nz = 6 * (N + 1)
        Cz = np.zeros((nz, nz))
        Cz[:6, :6] = P0
        for k in range(N):
            Cz[6 * (k + 1):6 * (k + 2), 6 * (k + 1):6 * (k + 2)] = Qs[k]
        maps = []
        M = np.zeros((6, nz)); M[:, :6] = np.eye(6)
        for k in range(N):
            M = Fs[k] @ M
            M[:, 6 * (k + 1):6 * (k + 2)] += np.eye(6)
            maps.append(M.copy())
        dz = np.zeros(nz); dz[:6] = dev(m0, refs[0])
        mu = [refs[k] + maps[k] @ dz for k in range(N)]
        A_y = np.concatenate([H @ Mk for Mk in maps], 0)
        Vy = np.zeros((3 * N, 3 * N))
        for k in range(N):
            Vy[3 * k:3 * k + 3, 3 * k:3 * k + 3] = Vs[k]
        Syy = A_y @ Cz @ A_y.T + Vy
        Sxy = maps[-1] @ Cz @ A_y.T
        Sxx = maps[-1] @ Cz @ maps[-1].T
        dy = y.reshape(-1) - np.concatenate([H @ m for m in mu])
        sol = np.linalg.solve(Syy, dy)
        x_b = mu[-1] + Sxy @ sol
        C_b = Sxx - Sxy @ np.linalg.solve(Syy, Sxy.T)
        chi_b = float(dy @ sol)
        x = torch.tensor(x[None]); C = torch.tensor(C[None])
        xf = x[0].numpy().copy()
        xf[4] = x_b[4] + math.remainder(xf[4] - x_b[4], 2 * math.pi)
        assert np.allclose(xf, x_b, rtol=1e-8, atol=1e-9)
        sc = np.sqrt(np.outer(np.diag(C_b), np.diag(C_b)))
        assert np.abs((C[0].numpy() - C_b) / sc).max() < 1e-6
        assert abs(chi_sum - chi_b) < 1e-7 * max(1.0, chi_b)


def test_charge_flip_equals_signed_curvature_update():
    p = torch.tensor([[10.0, 1.0, 2.0, 0.02, 0.1, 1.2]], dtype=DT)
    C = _random_spd(1, 6, 9, 0.1)
    C[0, 3, 3] = 0.04
    C[0, 0, 3] = C[0, 3, 0] = 0.01      # strong position-curvature correlation
    m = torch.tensor([[10.0, 1.0 - 0.3, 2.0]], dtype=DT)
    V = torch.diag(torch.tensor([1e-4, 1e-4, 1e-4], dtype=DT))[None]
    for q0 in (1.0, -1.0):
        p2, C2, q2, chi2, st = O.update(p, C, torch.tensor([q0], dtype=DT), m, V)
        # signed parameters: k = q * ipt, covariance D C D
        D = np.diag([1, 1, 1, q0, 1, 1.0])
        ps = p[0].numpy() * np.diag(D)
        Cs = D @ C[0].numpy() @ D
        S = Cs[:3, :3] + V[0].numpy()
        K = Cs[:, :3] @ np.linalg.inv(S)
        r = m[0].numpy() - ps[:3]
        ps2 = ps + K @ r
        Cs2 = Cs - K @ Cs[:3, :]
        qn = 1.0 if ps2[3] >= 0 else -1.0
        assert float(q2[0]) == qn
        flipped = qn != q0
        assert bool(int(st[0]) & O.CHARGE_FLIP) == flipped
        Dn = np.diag([1, 1, 1, qn, 1, 1.0])
        assert np.allclose(p2[0, :4].numpy(), (Dn @ ps2)[:4], rtol=1e-12, atol=1e-14)
        assert abs(math.remainder(float(p2[0, 4]) - ps2[4], 2 * math.pi)) < 1e-14
        assert np.allclose(C2[0].numpy(), Dn @ Cs2 @ Dn, rtol=1e-9, atol=1e-13)
    # at least one of the two charges must actually flip in this setup
    _, _, qa, _, _ = O.update(p, C, torch.tensor([1.0], dtype=DT), m, V)
    _, _, qb, _, _ = O.update(p, C, torch.tensor([-1.0], dtype=DT), m, V)
    assert float(qa[0]) != 1.0 or float(qb[0]) != -1.0


def test_phi_wrap_range():
    x = torch.tensor([math.pi, -math.pi, 3.5, -3.5, 0.0, 7.0, -7.0], dtype=DT)
    w = O.wrap_phi(x)
    assert float(w[0]) == math.pi and float(w[1]) == math.pi
    assert bool(((w > -math.pi) & (w <= math.pi)).all())
    assert torch.allclose(torch.cos(w), torch.cos(x)) and torch.allclose(torch.sin(w), torch.sin(x))
