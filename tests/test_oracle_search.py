"""Pins of the search oracle (oracle/kf_search.py) against independent
statements of what it computes: exhaustive enumeration of every path when the
beam exceeds their number, exact ties from duplicated hits, the miss rule,
and the efficiency on noise-free and noisy pools."""
import copy
import math

import numpy as np
import pytest
import torch

from oracle import kf_oracle as O
from oracle import kf_search as KS
from search_common import PLAN, SEED_LAYER, default_params, search_inputs

IL = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]


def _V(cov6):
    V = np.zeros((3, 3))
    for c, (i, j) in enumerate(IL):
        V[i, j] = V[j, i] = cov6[c]
    return V


def _window_scan(p2, C2, L, R, prm, pools):
    """(pool index, chi2) of every hit of layer L inside the window of the
    state (p2, C2) with chi2 <= chi2_max, by a scan over all of the layer's
    hits."""
    phi = math.atan2(p2[1], p2[0])
    t = np.array([-math.sin(phi), math.cos(phi), 0.0])
    w_r = np.clip(prm.n_sigma * math.sqrt(t @ C2[:3, :3] @ t + prm.sigma_rphi[L] ** 2), prm.win_min_rphi[L],
                  prm.win_max_rphi[L])
    w_z = np.clip(prm.n_sigma * math.sqrt(C2[2, 2] + prm.sigma_z[L] ** 2), prm.win_min_z[L], prm.win_max_z[L])
    kids = []
    for h in range(int(pools.layer_offsets[L]), int(pools.layer_offsets[L + 1])):
        m = pools.pos[:, h]
        d = (math.atan2(m[1], m[0]) - phi + math.pi) % (2 * math.pi) - math.pi
        if abs(d) * R > w_r or abs(m[2] - p2[2]) > w_z:
            continue
        r = m - p2[:3]
        chi2 = float(r @ np.linalg.solve(C2[:3, :3] + _V(pools.cov[:, h]), r))
        if chi2 <= prm.chi2_max:
            kids.append((h, chi2))
    return kids


def _update(p, C, q, pools, h):
    pu, Cu, qu, _, _ = O.update(torch.tensor(p[None]), torch.tensor(C[None]), torch.tensor([q], dtype=torch.float64),
                                torch.tensor(pools.pos[:, h][None]), torch.tensor(_V(pools.cov[:, h])[None]))
    return pu[0].numpy(), Cu[0].numpy(), float(qu[0])


def enumerate_paths(p, C, q, plan, g, pools, prm):
    """Every path the search rules allow for one seed, by depth-first
    recursion; windows by a scan over all pool hits of the layer.  With
    prm.overlap, a path that takes hit h then takes the overlap hit: of the
    layer's hits on modules with a higher id inside the window of the updated state
    with chi2 <= chi2_max, the smallest chi2 (lower id among equals); the
    overlap hit's score term counts in the ranking from the next layer on.
    Returns (score in the last ranking, final score, hits, overlap hits) per
    path."""
    out = []

    def rec(k, p, C, q, layer, score, misses, hist, ovl, last_ovl=0.0):
        if k == len(plan):
            out.append((score - last_ovl, score, hist, ovl))
            return
        L = plan[k]
        R = float(g.pos[L])
        f64 = lambda v: torch.tensor([v], dtype=torch.float64)
        p2, C2, _, st = O.propagate(torch.tensor(p[None]), torch.tensor(C[None]), f64(q), torch.tensor([0]), f64(R),
                                    f64(float(g.x_over_x0[L])), g, same=torch.tensor([layer == L]))
        if int(st[0]) & O.NO_CROSSING:
            return
        p2, C2 = p2[0].numpy(), C2[0].numpy()
        kids = _window_scan(p2, C2, L, R, prm, pools)
        if not kids:
            if misses < prm.max_miss:
                rec(k + 1, p2, C2, q, L, score - prm.miss_penalty, misses + 1, hist + [KS.MISS], ovl + [KS.MISS])
            return
        for h, chi2 in kids:
            pu, Cu, qu = _update(p2, C2, q, pools, h)
            sc, oid, term = score + prm.hit_bonus - chi2, KS.MISS, 0.0
            if prm.overlap:
                ok = [x for x in _window_scan(pu, Cu, L, R, prm, pools) if pools.module[x[0]] > pools.module[h]]
                if ok:
                    h2, c2 = min(ok, key=lambda x: (x[1], int(pools.hit_id[x[0]])))
                    pu, Cu, qu = _update(pu, Cu, qu, pools, h2)
                    term, oid = prm.overlap_bonus - c2, int(pools.hit_id[h2])
            rec(k + 1, pu, Cu, qu, L, sc + term, misses, hist + [int(pools.hit_id[h])], ovl + [oid], term)

    rec(0, p, C, q, SEED_LAYER, 0.0, 0, [], [])
    return out


def _tiny_pools(ev, pools, tracks, layers, offsets, rotate=0.0):
    """Pools of the given layers holding, for each listed track, its true hit
    and copies moved along the layer by each of `offsets` (cm); hit positions
    rotated about z by `rotate`.  Copy c of a hit is on module c."""
    P = copy.copy(pools)
    pos, cov, tid, mod, off = [], [], [], [], [0]
    c, s = math.cos(rotate), math.sin(rotate)
    for L in range(int(ev.geometry.n_layers)):
        if L in layers:
            for t in tracks:
                sel = np.nonzero((pools.track == t) & (np.arange(pools.track.size) >= pools.layer_offsets[L]) &
                                 (np.arange(pools.track.size) < pools.layer_offsets[L + 1]))[0]
                for h in sel:
                    m = pools.pos[:, h]
                    phi = math.atan2(m[1], m[0])
                    for ci, dl in enumerate([0.0] + list(offsets)):
                        R = math.hypot(m[0], m[1])
                        ph = phi + dl / R + rotate
                        pos.append([R * math.cos(ph), R * math.sin(ph), m[2] + 0.3 * dl])
                        cov6 = pools.cov[:, h].copy()
                        # rotate the covariance with the hit
                        V = _V(cov6)
                        a = dl / R + rotate
                        Rm = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
                        V = Rm @ V @ Rm.T
                        cov.append([V[i, j] for i, j in IL])
                        tid.append(t)
                        mod.append(ci)
        off.append(len(pos))
    P.pos = np.asarray(pos, np.float64).T.reshape(3, -1)
    P.cov = np.asarray(cov, np.float64).T.reshape(6, -1)
    P.track = np.asarray(tid, np.int32)
    P.module = np.asarray(mod, np.int32)   # each copy of a hit on a module of its own
    P.hit_id = np.arange(len(pos), dtype=np.int32)[::-1].copy()   # ids not in pool order
    P.layer_offsets = np.asarray(off, np.int32)
    return P


def _rotate_seed(p, C, a):
    c, s = math.cos(a), math.sin(a)
    p = p.copy()
    p[0], p[1] = c * p[0] - s * p[1], s * p[0] + c * p[1]
    p[4] = (p[4] + a + math.pi) % (2 * math.pi) - math.pi
    J = np.eye(6)
    J[:2, :2] = [[c, -s], [s, c]]
    return p, J @ C @ J.T


@pytest.mark.parametrize("rotate", [0.0, "wrap"])
def test_search_equals_exhaustive_enumeration_when_the_beam_holds_every_path(rotate):
    wl, ev, g, pools, p, C, q = search_inputs(40, noise=False)
    plan = PLAN[:4]
    prm = default_params(g, beam=200)
    checked = 0
    for t in range(6):
        a = 0.0
        if rotate == "wrap":
            # turn the track so that its second plan-layer hit sits 1e-4 rad below +pi
            h = int(np.nonzero((pools.track == t) & (np.arange(pools.track.size) >= pools.layer_offsets[plan[1]]) &
                               (np.arange(pools.track.size) < pools.layer_offsets[plan[1] + 1]))[0][0])
            a = math.pi - 1e-4 - math.atan2(pools.pos[1, h], pools.pos[0, h])
        P = _tiny_pools(ev, pools, [t], set(plan), offsets=(0.004, -0.006), rotate=a)
        ps, Cs = _rotate_seed(p[t], C[t], a)
        paths = enumerate_paths(ps, Cs, float(q[t]), plan, g, P, prm)
        res = KS.score_hits(ps[None], Cs[None], q[t:t + 1], [SEED_LAYER], plan, g, P, prm)
        assert 1 <= len(paths) <= prm.beam
        paths.sort(key=lambda x: -x[0])
        for r, (sc, _, hist, _) in enumerate(paths):
            assert list(res["hits"][0, r]) == hist, (t, r)
            assert abs(res["score"][0, r] - sc) <= 1e-9 * max(1.0, abs(sc))
        assert (res["hits"][0, len(paths):] == KS.NO_CAND).all()
        checked += len(paths) > 1
    assert checked >= 3   # the cases do branch


def test_duplicated_hits_tie_exactly_and_the_lower_id_wins():
    wl, ev, g, pools, p, C, q = search_inputs(50, noise=False)
    P = _tiny_pools(ev, pools, list(range(50)), set(PLAN), offsets=(0.0,))   # each true hit twice, same values
    prm = default_params(g)
    res = KS.score_hits(p, C, q, np.full(50, SEED_LAYER), PLAN, g, P, prm)
    for t in range(50):
        s = res["score"][t]
        assert (s == s[0]).all()                  # every kept candidate ties exactly
        # rank 0 takes the lower id at every layer (ids run opposite to pool order)
        h = res["hits"][t, 0]
        idx = {int(i): k for k, i in enumerate(P.hit_id)}
        for L, hid in zip(PLAN, h):
            if hid < 0:
                continue
            k = idx[int(hid)]
            twin = k + 1 if (k - P.layer_offsets[L]) % 2 == 0 else k - 1
            assert hid < P.hit_id[twin]
    assert not res["flagged"].any()


def test_noise_free_pools_are_found_with_full_efficiency():
    wl, ev, g, pools, p, C, q = search_inputs(400, noise=False)
    res = KS.score_hits(p, C, q, np.full(400, SEED_LAYER), PLAN, g, pools, default_params(g))
    best = res["hits"][:, 0]
    ok = np.array([[h >= 0 and pools.track[h] == t for h in best[t]] for t in range(400)])
    assert ok.mean() >= 0.99, ok.mean()


def test_noisy_pools_keep_most_true_hits():
    wl, ev, g, pools, p, C, q = search_inputs(300, noise=True)
    res = KS.score_hits(p, C, q, np.full(300, SEED_LAYER), PLAN, g, pools, default_params(g))
    best = res["hits"][:, 0]
    ok = np.array([[h >= 0 and pools.track[h] == t for h in best[t]] for t in range(300)])
    assert ok.mean() >= 0.9, ok.mean()
    assert res["n_window_hits"] > 300 * len(PLAN)


def _drop_layers(pools, layers):
    P = copy.copy(pools)
    keep = np.ones(pools.track.size, bool)
    for L in layers:
        keep[pools.layer_offsets[L]:pools.layer_offsets[L + 1]] = False
    P.pos, P.cov, P.track, P.hit_id = pools.pos[:, keep], pools.cov[:, keep], pools.track[keep], pools.hit_id[keep]
    cnt = np.add.reduceat(keep.astype(int), pools.layer_offsets[:-1]) * (np.diff(pools.layer_offsets) > 0)
    P.layer_offsets = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int32)
    return P


def test_missed_layers_cost_the_penalty_and_stop_the_candidate_beyond_the_limit():
    wl, ev, g, pools, p, C, q = search_inputs(30, noise=False)
    prm = default_params(g)
    P = _drop_layers(pools, [6, 7])
    res = KS.score_hits(p, C, q, np.full(30, SEED_LAYER), PLAN, g, P, prm)
    full = KS.score_hits(p, C, q, np.full(30, SEED_LAYER), PLAN, g, pools, prm)
    for t in range(30):
        h = res["hits"][t, 0]
        assert h[PLAN.index(6)] == KS.MISS and h[PLAN.index(7)] == KS.MISS
        assert (np.delete(h, [PLAN.index(6), PLAN.index(7)]) >= 0).all()
        # two misses replace two accepted hits: the score drops by at least 2 (bonus + penalty - chi2 each)
        assert res["score"][t, 0] < full["score"][t, 0]
    # four empty layers in a row: three misses, then the candidate stops and
    # keeps its score; every later layer reads STOP
    P4 = _drop_layers(pools, [6, 7, 8, 9])
    res4 = KS.score_hits(p, C, q, np.full(30, SEED_LAYER), PLAN, g, P4, prm)
    k6 = PLAN.index(6)
    for t in range(30):
        h = res4["hits"][t, 0]
        assert (h[:k6] >= 0).all()
        assert (h[k6:k6 + 3] == KS.MISS).all() and (h[k6 + 3:] == KS.STOP).all()
        assert (res4["hits"][t, 1:] == KS.NO_CAND).all()   # one path only


def test_near_ties_are_flagged():
    """A hit mirrored through the predicted point has the same chi2 up to
    rounding (here often exactly, in FP64): the ranking decision between the
    two is flagged near, since FP32 rounds the two differently."""
    wl, ev, g, pools, p, C, q = search_inputs(20, noise=False)
    prm = default_params(g)
    plan = PLAN[:1]
    L = plan[0]
    flagged = 0
    for t in range(20):
        p2, C2, _, _ = O.propagate(torch.tensor(p[t][None]), torch.tensor(C[t][None]), torch.tensor(q[t:t + 1]),
                                   torch.tensor([0]), torch.tensor([float(g.pos[L])], dtype=torch.float64),
                                   torch.tensor([float(g.x_over_x0[L])], dtype=torch.float64), g)
        pp = p2[0].numpy()
        P = _tiny_pools(ev, pools, [t], {L}, offsets=())
        m1 = P.pos[:, 0]
        m2 = 2 * pp[:3] - m1
        P.pos = np.stack([m1, m2], axis=1)
        P.cov = np.stack([P.cov[:, 0], P.cov[:, 0]], axis=1)
        P.hit_id = np.array([5, 3], np.int32)
        P.track = np.array([t, t], np.int32)
        P.layer_offsets = np.array([0] * (L + 1) + [2] * (g.n_layers - L), np.int32)
        res = KS.score_hits(p[t:t + 1], C[t:t + 1], q[t:t + 1], [SEED_LAYER], plan, g, P, prm)
        s = res["score"][0]
        if np.isfinite(s[1]):
            assert res["flagged"][0], (t, s)   # equal or not, the two differ only by rounding
            flagged += 1
    assert flagged >= 5


def test_flipped_near_ties_give_the_other_valid_order():
    """The mirrored-hit near tie above, taken the other way (flips): the two
    candidates trade ranks and nothing else changes; either order is a valid
    result (valid_alternative finds both), while a made-up order is not."""
    wl, ev, g, pools, p, C, q = search_inputs(20, noise=False)
    prm = default_params(g)
    plan = PLAN[:1]
    L = plan[0]
    checked = 0
    for t in range(20):
        p2, C2, _, _ = O.propagate(torch.tensor(p[t][None]), torch.tensor(C[t][None]), torch.tensor(q[t:t + 1]),
                                   torch.tensor([0]), torch.tensor([float(g.pos[L])], dtype=torch.float64),
                                   torch.tensor([float(g.x_over_x0[L])], dtype=torch.float64), g)
        pp = p2[0].numpy()
        P = _tiny_pools(ev, pools, [t], {L}, offsets=())
        m1 = P.pos[:, 0]
        P.pos = np.stack([m1, 2 * pp[:3] - m1], axis=1)
        P.cov = np.stack([P.cov[:, 0], P.cov[:, 0]], axis=1)
        P.hit_id = np.array([5, 3], np.int32)
        P.track = np.array([t, t], np.int32)
        P.layer_offsets = np.array([0] * (L + 1) + [2] * (g.n_layers - L), np.int32)
        args = (p[t:t + 1], C[t:t + 1], q[t:t + 1], [SEED_LAYER], plan, g, P, prm)
        base = KS.score_hits(*args)
        if not np.isfinite(base["score"][0][1]):
            continue
        ranks = [k for k in base["near"][0] if k[0] == "rank"]
        assert ranks
        flipped = KS.score_hits(*args, flips={ranks[0]})
        assert np.array_equal(flipped["hits"][0, 0], base["hits"][0, 1])
        assert np.array_equal(flipped["hits"][0, 1], base["hits"][0, 0])
        assert np.array_equal(flipped["hits"][0, 2:], base["hits"][0, 2:])
        for h in (base["hits"][0], flipped["hits"][0]):
            ok, runs = KS.valid_alternative(h, p[t], C[t], q[t], SEED_LAYER, plan, g, P, prm)
            assert ok
        bogus = base["hits"][0].copy()
        bogus[0, 0] = 999999
        assert not KS.valid_alternative(bogus, p[t], C[t], q[t], SEED_LAYER, plan, g, P, prm)[0]
        checked += 1
    assert checked >= 5


def test_no_flips_is_the_plain_search_and_every_flagged_seed_has_its_own_result():
    """flips = {} reproduces the plain run; the plain result of a flagged
    seed is found by valid_alternative on its first run; a cut flip on a
    flagged seed changes only what follows from that one decision."""
    wl, ev, g, pools, p, C, q = search_inputs(150)
    prm = default_params(g)
    a = KS.score_hits(p, C, q, np.full(150, SEED_LAYER), PLAN, g, pools, prm)
    b = KS.score_hits(p, C, q, np.full(150, SEED_LAYER), PLAN, g, pools, prm, flips=set())
    assert np.array_equal(a["hits"], b["hits"]) and np.array_equal(a["score"], b["score"])
    fl = np.nonzero(a["flagged"])[0]
    assert fl.size > 0
    for s in fl[:5]:
        ok, runs = KS.valid_alternative(a["hits"][s], p[s], C[s], q[s], SEED_LAYER, PLAN, g, pools, prm)
        assert ok and runs == 1
    cuts = [(s, k) for s in fl for k in a["near"][s] if k[0] == "cut"]
    if cuts:
        s, key = cuts[0]
        one = lambda fl_: KS.score_hits(p[s:s + 1], C[s:s + 1], q[s:s + 1], [SEED_LAYER], PLAN, g, pools, prm,
                                        flips=fl_)
        f = one({key})
        # the decision named by the key is taken the other way: its hit is
        # (or is no longer) among the children of that candidate at that layer
        step, hist, hid = key[1], key[2], key[3]
        had = any(tuple(x[:step]) == hist and x[step] == hid for x in a["hits"][s])
        has = any(tuple(x[:step]) == hist and x[step] == hid for x in f["hits"][0])
        assert not (had and has)


def test_valid_alternative_finds_results_of_several_flips():
    """A result made by taking two or three near decisions of a flagged seed
    the other way is recognised as a valid alternative (the guided search
    reaches it within its budget), and a result with one hit changed is not."""
    wl, ev, g, pools, p, C, q = search_inputs(300)
    prm = default_params(g)
    a = KS.score_hits(p, C, q, np.full(300, SEED_LAYER), PLAN, g, pools, prm)
    rng = np.random.default_rng(1)
    cand = [s for s in np.nonzero(a["flagged"])[0] if len(a["near"][s]) >= 2]
    checked = 0
    for s in cand[:6]:
        keys = a["near"][s]
        k = min(len(keys), int(rng.integers(2, 4)))
        pick = {keys[i] for i in rng.choice(len(keys), k, replace=False)}
        tgt = KS.score_hits(p[s:s + 1], C[s:s + 1], q[s:s + 1], [SEED_LAYER], PLAN, g, pools, prm,
                            flips=pick)["hits"][0]
        ok, runs = KS.valid_alternative(tgt, p[s], C[s], q[s], SEED_LAYER, PLAN, g, pools, prm)
        assert ok, (s, pick, runs)
        checked += 1
    assert checked >= 3
    s = cand[0]
    bogus = a["hits"][s].copy()
    row = int(np.nonzero((bogus >= 0).any(axis=1))[0][0])
    col = int(np.nonzero(bogus[row] >= 0)[0][0])
    bogus[row, col] = 987654321
    assert not KS.valid_alternative(bogus, p[s], C[s], q[s], SEED_LAYER, PLAN, g, pools, prm, budget=8)[0]


def test_replay_reproduces_the_search_and_rejects_impossible_lists():
    """replay of every list the search keeps gives that list's score
    exactly, and consistent_result accepts the oracle's own result; a list
    with a hit swapped for one outside the window, a miss where a hit is
    surely accepted, or a score off by more than the margin is rejected."""
    wl, ev, g, pools, p, C, q = search_inputs(40)
    prm = default_params(g)
    o = KS.score_hits(p, C, q, np.full(40, SEED_LAYER), PLAN, g, pools, prm)
    checked = 0
    for s in range(40):
        rows = o["hits"][s]
        for r in range(rows.shape[0]):
            if rows[r, 0] == KS.NO_CAND:
                continue
            rp = KS.replay(rows[r], p[s], C[s], q[s], SEED_LAYER, PLAN, g, pools, prm)
            assert rp["valid"], (s, r, rp["reason"])
            assert abs(rp["score"] - o["score"][s, r]) <= 1e-9 * max(1.0, abs(o["score"][s, r]))
            assert abs(rp["err"] - o["score_err"][s, r]) <= 1e-9 * max(1.0, o["score_err"][s, r])
        ok, why = KS.consistent_result(rows, o["score"][s], p[s], C[s], q[s], SEED_LAYER, PLAN, g, pools, prm,
                                       rows, o["score"][s], o["score_err"][s])
        assert ok, (s, why)
        checked += 1
    assert checked == 40
    # impossible lists on the first seed whose best list has hits on its first two steps
    s = next(i for i in range(40) if (o["hits"][i, 0, :2] >= 0).all())
    row = o["hits"][s, 0].copy()
    # the pool hit of the first layer farthest from the seed in phi
    a, b = int(pools.layer_offsets[PLAN[0]]), int(pools.layer_offsets[PLAN[0] + 1])
    dphi = np.angle(np.exp(1j * (np.arctan2(pools.pos[1, a:b], pools.pos[0, a:b]) - np.arctan2(p[s, 1], p[s, 0]))))
    far = int(pools.hit_id[a + int(np.argmax(np.abs(dphi)))])
    bad = row.copy()
    bad[0] = far
    assert not KS.replay(bad, p[s], C[s], q[s], SEED_LAYER, PLAN, g, pools, prm)["valid"]
    miss = row.copy()
    miss[0] = KS.MISS
    rp = KS.replay(miss, p[s], C[s], q[s], SEED_LAYER, PLAN, g, pools, prm)
    assert not rp["valid"] and "accepted hit" in rp["reason"]
    sc = o["score"][s].copy()
    sc[0] += 1.0 + 10 * KS.RANK_SIGMAS * o["score_err"][s, 0]
    assert not KS.consistent_result(o["hits"][s], sc, p[s], C[s], q[s], SEED_LAYER, PLAN, g, pools, prm,
                                    o["hits"][s], o["score"][s], o["score_err"][s])[0]


@pytest.mark.parametrize("rotate", [0.0, "wrap"])
def test_overlap_search_equals_exhaustive_enumeration(rotate):
    """With the overlap step, every path (hits and overlap hits), its rank
    (by the score of the last ranking, which does not hold that layer's
    overlap term) and its final score equal the exhaustive enumeration of the
    rules (each copy of a hit on a module of its own, so the copies are each
    other's overlap candidates)."""
    wl, ev, g, pools, p, C, q = search_inputs(40, noise=False)
    plan = PLAN[:4]
    prm = default_params(g, beam=200)
    prm.overlap = True
    checked = 0
    for t in range(6):
        a = 0.0
        if rotate == "wrap":
            h = int(np.nonzero((pools.track == t) & (np.arange(pools.track.size) >= pools.layer_offsets[plan[1]]) &
                               (np.arange(pools.track.size) < pools.layer_offsets[plan[1] + 1]))[0][0])
            a = math.pi - 1e-4 - math.atan2(pools.pos[1, h], pools.pos[0, h])
        P = _tiny_pools(ev, pools, [t], set(plan), offsets=(0.004, -0.006), rotate=a)
        ps, Cs = _rotate_seed(p[t], C[t], a)
        paths = enumerate_paths(ps, Cs, float(q[t]), plan, g, P, prm)
        res = KS.score_hits(ps[None], Cs[None], q[t:t + 1], [SEED_LAYER], plan, g, P, prm)
        assert 1 <= len(paths) <= prm.beam
        # the same set of paths with the same scores, in the order of the
        # last ranking (taking a hit and its overlap hit in either order gives
        # the same final state and, in the linear model, the same chi2 sum:
        # such paths tie up to rounding, so only the scores' order is checked)
        want = {(tuple(hist), tuple(ovl)): (rs, sc) for rs, sc, hist, ovl in paths}
        got = [(tuple(int(x) for x in res["hits"][0, r]), tuple(int(x) for x in res["overlap"][0, r]))
               for r in range(len(paths))]
        assert set(got) == set(want), t
        for r, key in enumerate(got):
            assert abs(res["score"][0, r] - want[key][1]) <= 1e-9 * max(1.0, abs(want[key][1]))
        rs = [want[key][0] for key in got]
        assert all(a >= b - 1e-9 * max(1.0, abs(a)) for a, b in zip(rs[:-1], rs[1:])), t
        assert (res["hits"][0, len(paths):] == KS.NO_CAND).all()
        checked += sum(o >= 0 for o in max(paths)[3])
    assert checked >= 6   # overlap hits are taken


def test_overlap_hits_on_modules_with_overlaps():
    """Pools split into modules with overlap hits (toygen.with_modules), no
    noise: where the best candidate of a seed took its track's hit on the
    lower of two overlapping modules, it takes the track's second hit (on
    the higher module) as its overlap hit (>= 95%);
    every overlap hit it takes is on a higher module than its layer's hit and
    belongs to the same track; and without the overlap step no overlap hit
    is reported."""
    from toygen import with_modules, workloads
    wl, ev, g, pools, p, C, q = search_inputs(150, noise=False)
    P = with_modules(workloads()["search20"], ev, pools)
    prm = default_params(g)
    prm.overlap = True
    res = KS.score_hits(p, C, q, np.full(150, SEED_LAYER), PLAN, g, P, prm)
    idx = {int(h): k for k, h in enumerate(P.hit_id)}
    avail = took = 0
    for t in range(150):
        for hid, oid in zip(res["hits"][t, 0], res["overlap"][t, 0]):
            if hid < 0:
                continue
            k = idx[int(hid)]
            L = int(np.searchsorted(P.layer_offsets, k, side="right") - 1)
            a, b = int(P.layer_offsets[L]), int(P.layer_offsets[L + 1])
            twins = [j for j in range(a, b) if P.track[j] == P.track[k] and j != k and P.module[j] > P.module[k]]
            if oid >= 0:
                j = idx[int(oid)]
                assert P.module[j] > P.module[k] and P.track[j] == P.track[k]
            if P.track[k] == t and twins:
                avail += 1
                took += oid >= 0
    assert avail >= 50 and took >= 0.95 * avail, (took, avail)
    prm.overlap = False
    res0 = KS.score_hits(p, C, q, np.full(150, SEED_LAYER), PLAN, g, P, prm)
    assert ((res0["overlap"] == KS.MISS) | (res0["overlap"] == KS.NO_CAND)).all()


def test_replay_with_overlap_hits_reproduces_the_search():
    """With the overlap step, replay of every kept list (hits and overlap
    hits) gives its score and error exactly and consistent_result accepts
    the oracle's own result; a list whose overlap hit is dropped where one
    is surely accepted is rejected."""
    from search_common import module_inputs
    wl, ev, g, pools, p, C, q = module_inputs(40)
    prm = default_params(g)
    prm.overlap = True
    o = KS.score_hits(p, C, q, np.full(40, SEED_LAYER), PLAN, g, pools, prm)
    dropped = 0
    for s in range(40):
        rows, ov = o["hits"][s], o["overlap"][s]
        for r in range(rows.shape[0]):
            if rows[r, 0] == KS.NO_CAND:
                continue
            rp = KS.replay(rows[r], p[s], C[s], q[s], SEED_LAYER, PLAN, g, pools, prm, ovl_row=ov[r])
            assert rp["valid"], (s, r, rp["reason"])
            assert abs(rp["score"] - o["score"][s, r]) <= 1e-9 * max(1.0, abs(o["score"][s, r]))
            assert abs(rp["err"] - o["score_err"][s, r]) <= 1e-9 * max(1.0, o["score_err"][s, r])
        ok, why = KS.consistent_result(rows, o["score"][s], p[s], C[s], q[s], SEED_LAYER, PLAN, g, pools, prm, rows,
                                       o["score"][s], o["score_err"][s], overlap=ov, oracle_overlap=ov)
        assert ok, (s, why)
        k = np.nonzero(ov[0] >= 0)[0]
        if k.size and not o["flagged"][s]:
            bad = ov[0].copy()
            bad[k[0]] = KS.MISS
            rp = KS.replay(rows[0], p[s], C[s], q[s], SEED_LAYER, PLAN, g, pools, prm, ovl_row=bad)
            assert not rp["valid"] and "surely accepted" in rp["reason"], rp
            dropped += 1
    assert dropped >= 5
