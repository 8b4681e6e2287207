"""FP64 CPU oracle of the combinatorial candidate search (kf_score_hits).
TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; it shares no code with the HIP
kernels.

What the paper fixes (Sec. 2.2, forward search; Sec. 3.1, layers and layer
plans): each seed proceeds outwards layer by layer along a layer plan; every
candidate is propagated to the layer, the layer's hits compatible with it are
selected, and the Kalman-filter calculations are done for them; a seed keeps
at most a fixed number of concurrent candidates, a candidate may miss a
limited number of layers, and the best-scoring candidate represents the seed.
The window, the chi2 cut, the score function and the tie-break are
per-iteration parameters and standard functions that the paper does not
spell out (Sec. 3.2, 3.3).  Readings taken here, step by step, for every
layer L of the plan and every live candidate of a seed:

1. Propagate the candidate (state and covariance, with the layer's material)
   to layer L (kf_oracle.propagate; `same` = the candidate is on L already).
   A candidate without a crossing stops (see below).
2. Window around the predicted point (x, y, z), phi_p = atan2(y, x):
     w_rphi = clamp(n_sigma sqrt(t^T C_pos t + sigma_rphi^2), win_min_rphi, win_max_rphi)
     w_z    = clamp(n_sigma sqrt(C_zz + sigma_z^2),            win_min_z,    win_max_z)
   with t = (-sin phi_p, cos phi_p, 0) the transverse tangent of the layer.
   A pool hit of layer L is inside iff |wrap(phi_h - phi_p)| <= w_rphi / R_L
   and |z_h - z_p| <= w_z, phi_h = atan2(y_h, x_h).
3. chi2 of every hit inside (the update's r^T S^-1 r, no update); the hit is
   accepted iff chi2 <= chi2_max.
4. Children: one per accepted hit with score = parent score + hit_bonus -
   chi2.  If no hit is accepted, one miss child with score = parent score -
   miss_penalty, unless the parent has already missed max_miss layers: then
   the candidate stops.
5. Per seed, all children of all its candidates are ranked by (score
   descending; then hit id ascending, a miss after every hit and a stop
   after a miss; then parent rank ascending) and the first `beam` are kept,
   in that order (their ranks).
6. A kept child with a hit gets the Kalman update with it (kf_oracle.update);
   a miss child keeps the propagated state.

Stopping (the search ends for a candidate at the tracker edge or when no
more hits are found, Sec. 2.2): a candidate that stops keeps its score and
the state it entered the layer with, and from then on has, at every layer,
exactly one child -- itself, marked STOP (-3) in the hit list -- which
competes in the ranking like any other child.

A seed starts with one candidate (rank 0, score 0, no misses) holding the
seed state, on the seed's layer.

Several results are correct where FP32 and FP64 rounding can decide
differently.  The oracle therefore flags a seed when any of its decisions is
near, against an error model of FP32 at that decision:
* position: a point at radius R predicted in FP32 is off by about
  4 ulp32(R) (1 + 1/|cos a|) along the layer, a the incidence angle (the
  crossing of a cylinder is resolved only to ulp/|cos a| near tangency);
* chi2 of one hit: 2 sqrt(chi2 + 1) (position error) / s_r
  + (1e-4 + COND_K eps32 kappa(S)) chi2, with s_r = sqrt(t^T C_pos t +
  sigma_rphi^2) the residual's r-phi spread and kappa(S) the condition number
  of the residual covariance (near a tangent crossing the predicted position
  is spread along the layer, S is nearly singular and its FP32 form resolves
  the small eigenvalue only to eps32 kappa);
* window edge: a pool hit within EDGE_REL w + (position error) of an edge;
* chi2 cut: a chi2 within the chi2 error (at the cut) of chi2_max;
* ranking: two children adjacent in the ranking at positions up to `beam`
  (order inside the kept set and the cut after it) whose scores differ by a
  non-zero amount of at most the summed chi2 errors of the terms in which
  they differ.  Two children whose histories agree up to some layer share
  the score of that common ancestor (in any precision the same computed
  value), so only the terms since they diverged count.  Exactly equal scores
  are near too, unless every term since the divergence takes identical hits
  (same position and covariance: a duplicated hit) or a miss or stop in both:
  such a tie holds in every precision and step 5 breaks it the same way.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import kf_oracle as O

MISS = -1        # hit id of a miss in the output
NO_CAND = -2     # hit id where the seed has no candidate of that rank
STOP = -3        # hit id of the layers after a candidate stopped
_KEY = {MISS: np.iinfo(np.int64).max - 1, STOP: np.iinfo(np.int64).max}
EDGE_REL = 1e-4      # relative error of a window half-width
CHI2_REL = 1e-4      # relative error of a chi2 from the covariance
ULP_FACTOR = 1.0     # FP32 position error in units of ulp32(R)
RANK_SIGMAS = 3.0    # score margin: this many root-sum-squares of the term errors


def ulp32(x):
    x = np.float32(abs(x))
    return float(np.spacing(x))


def pos_error(R, cos_a):
    """FP32 error of a predicted point at radius R along the layer."""
    return ULP_FACTOR * ulp32(R) * (1.0 + 1.0 / max(abs(cos_a), 1e-6))


COND_K = 4.0        # chi2 relative error per unit of eps32 * kappa(S)
EPS32 = float(np.finfo(np.float32).eps)


def chi2_error(chi2, epos, sigma, kappa=1.0):
    return 2.0 * math.sqrt(max(chi2, 0.0) + 1.0) * epos / sigma + (CHI2_REL + COND_K * EPS32 * kappa) * chi2


@dataclasses.dataclass
class SearchParams:
    """Parameters of the search (defaults: the 20-layer barrel workload)."""
    n_layers: int
    beam: int = 6
    chi2_max: float = 30.0
    n_sigma: float = 5.0
    hit_bonus: float = 10.0
    miss_penalty: float = 5.0
    max_miss: int = 3
    win_min_rphi: np.ndarray = None   # [n_layers] cm
    win_max_rphi: np.ndarray = None
    win_min_z: np.ndarray = None
    win_max_z: np.ndarray = None
    sigma_rphi: np.ndarray = None     # [n_layers] nominal hit resolution, cm
    sigma_z: np.ndarray = None
    overlap: bool = False             # pick up one overlap hit per layer (step 7)
    overlap_bonus: float = 5.0        # score of an overlap hit: + overlap_bonus - chi2

    def __post_init__(self):
        L = self.n_layers
        d = dict(win_min_rphi=0.01, win_max_rphi=2.0, win_min_z=0.03, win_max_z=2.0, sigma_rphi=0.003, sigma_z=0.01)
        for k, v in d.items():
            if getattr(self, k) is None:
                setattr(self, k, np.full(L, v))
            else:
                setattr(self, k, np.asarray(getattr(self, k), np.float64))


def _wrap(a):
    return a - 2.0 * math.pi * np.ceil((a - math.pi) / (2.0 * math.pi))


class _LayerPool:
    """Hits of one layer sorted by phi for window queries."""

    def __init__(self, pos, cov, ids, mods=None):
        phi = np.arctan2(pos[1], pos[0])
        o = np.argsort(phi, kind="stable")
        self.phi = phi[o]
        self.pos = pos[:, o]
        self.cov = cov[:, o]
        self.ids = ids[o]
        self.mods = None if mods is None else mods[o]

    def query(self, phi_c, half):
        """Indices of hits with |wrap(phi - phi_c)| <= half (half < pi)."""
        lo, hi = phi_c - half, phi_c + half
        segs = []
        if lo < -math.pi:
            segs.append((lo + 2 * math.pi, math.pi))
            lo = -math.pi
        if hi > math.pi:
            segs.append((-math.pi, hi - 2 * math.pi))
            hi = math.pi
        segs.append((lo, hi))
        idx = [np.arange(np.searchsorted(self.phi, a, "left"), np.searchsorted(self.phi, b, "right")) for a, b in segs]
        return np.unique(np.concatenate(idx))


def _chi2(p_pos, C_pos, m, V6):
    """r^T (C_pos + V)^-1 r for hits m [k, 3] with packed covariances V6 [6, k],
    and the condition number of each C_pos + V."""
    k = m.shape[0]
    V = np.zeros((k, 3, 3))
    il = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
    for c, (i, j) in enumerate(il):
        V[:, i, j] = V[:, j, i] = V6[c]
    S = C_pos[None] + V
    r = m - p_pos[None]
    ev = np.linalg.eigvalsh(S)
    return np.einsum("ni,nij,nj->n", r, np.linalg.inv(S), r), ev[:, -1] / ev[:, 0]


def _round(p, C, dtype):
    return p.to(dtype).to(torch.float64), C.to(dtype).to(torch.float64)


def score_hits(seed_p, seed_C, seed_q, seed_layer, layer_plan, geom, pools, prm: SearchParams, state_round=None,
               flips=None):
    """Run the search.  seed_p [n, 6], seed_C [n, 6, 6], seed_q [n], seed_layer
    [n] (layer index the seed state is on), layer_plan: layer indices in
    order, geom: a detector Geometry (barrel layers), pools: object with
    layer_offsets [L+1], pos [3, np], cov [6, np], hit_id [np].
    state_round: None, or a dtype for the conditioning probe.
    flips: None, or a set of near-decision keys (as listed in `near`) to be
    taken the other way: a hit near a window edge counted on the other side
    of it, a chi2 near the cut accepted if it was rejected and the other way
    round, two near-tied neighbours of a ranking swapped.  A key names the
    layer step, the candidate by its history and the hit (or the two
    children by their histories), so it names the same decision in any run
    that reaches that candidate.
    Returns dict(hits [n, beam, P] int64, score [n, beam], p [n, beam, 6],
    C [n, beam, 6, 6], status [n], flagged [n] bool, flags [n] (near
    decisions: 1 window edge, 2 chi2 cut, 4 ranking), near [n] (list of the
    seed's near-decision keys), score_err [n, beam] (root-sum-square of the
    FP32 error model over the candidate's terms), n_window_hits)."""
    flips = frozenset() if flips is None else frozenset(flips)
    seed_p = np.asarray(seed_p, np.float64)
    seed_C = np.asarray(seed_C, np.float64)
    n, B, P = seed_p.shape[0], prm.beam, len(layer_plan)
    lp = {}
    for L in set(int(x) for x in layer_plan):
        a, b = int(pools.layer_offsets[L]), int(pools.layer_offsets[L + 1])
        mods = getattr(pools, "module", None) if prm.overlap else None
        if prm.overlap and mods is None:
            raise ValueError("the overlap step needs the pools' module ids")
        lp[L] = _LayerPool(np.asarray(pools.pos[:, a:b], np.float64), np.asarray(pools.cov[:, a:b], np.float64),
                           np.asarray(pools.hit_id[a:b], np.int64),
                           None if mods is None else np.asarray(mods[a:b], np.int64))
    # live candidates: parallel lists
    c_seed = list(range(n))
    c_rank = [0] * n
    c_p = [seed_p[i] for i in range(n)]
    c_C = [seed_C[i] for i in range(n)]
    c_q = [float(seed_q[i]) for i in range(n)]
    c_score = [0.0] * n
    c_miss = [0] * n
    c_layer = [int(seed_layer[i]) for i in range(n)]
    c_hist = [[] for _ in range(n)]
    c_ovl = [[] for _ in range(n)]   # overlap hit id of each step (MISS: none)
    c_err = [[] for _ in range(n)]   # FP32 error of each score term
    where = {}   # hit id -> index into pools, for comparing the inputs of exact ties

    def _same_input(x, y):
        if x == y:
            return True
        if x < 0 or y < 0:
            return False
        if not where:
            where.update({int(h): k for k, h in enumerate(np.asarray(pools.hit_id))})
        i, j = where[int(x)], where[int(y)]
        return bool(np.array_equal(pools.pos[:, i], pools.pos[:, j]) and np.array_equal(pools.cov[:, i], pools.cov[:, j]))

    status = np.zeros(n, np.int64)
    flags = np.zeros(n, np.int64)   # near decisions: 1 window edge, 2 chi2 cut, 4 ranking
    near = [[] for _ in range(n)]
    n_window = 0
    c_stop = [False] * n
    for step, L in enumerate(layer_plan):
        L = int(L)
        m = len(c_seed)
        if m == 0:
            break
        R = float(geom.pos[L])
        live = [i for i in range(m) if not c_stop[i]]
        p2 = np.zeros((m, 6))
        C2 = np.zeros((m, 6, 6))
        st = np.zeros(m, np.int64)
        if live:
            k_ = len(live)
            pp, CC, _, ss = O.propagate(torch.tensor(np.stack([c_p[i] for i in live])),
                                        torch.tensor(np.stack([c_C[i] for i in live])),
                                        torch.tensor([c_q[i] for i in live], dtype=torch.float64),
                                        torch.full((k_,), int(geom.kind[L]), dtype=torch.int64),
                                        torch.full((k_,), R, dtype=torch.float64),
                                        torch.full((k_,), float(geom.x_over_x0[L]), dtype=torch.float64), geom,
                                        same=torch.tensor([c_layer[i] == L for i in live]))
            if state_round is not None:
                pp, CC = _round(pp, CC, state_round)
            p2[live], C2[live], st[live] = pp.numpy(), CC.numpy(), ss.numpy()
        children = {}
        pool = lp[L]
        for i in range(m):
            s = c_seed[i]
            stop_child = (c_score[i], STOP, c_rank[i], i, -1, 0.0)
            if c_stop[i]:
                children.setdefault(s, []).append(stop_child)
                continue
            status[s] |= st[i]
            if st[i] & O.NO_CROSSING:
                children.setdefault(s, []).append(stop_child)
                continue
            x, y, z = p2[i, 0], p2[i, 1], p2[i, 2]
            phi_p = math.atan2(y, x)
            cos_a = math.sin(p2[i, 5]) * (math.cos(p2[i, 4]) * x + math.sin(p2[i, 4]) * y) / math.hypot(x, y)
            epos = pos_error(R, cos_a)
            t = np.array([-math.sin(phi_p), math.cos(phi_p), 0.0])
            Cp = C2[i, :3, :3]
            w_r = min(max(prm.n_sigma * math.sqrt(t @ Cp @ t + prm.sigma_rphi[L] ** 2), prm.win_min_rphi[L]),
                      prm.win_max_rphi[L])
            w_z = min(max(prm.n_sigma * math.sqrt(Cp[2, 2] + prm.sigma_z[L] ** 2), prm.win_min_z[L]), prm.win_max_z[L])
            # hits up to the edge margin beyond the window, for the near-decision flags
            mr = EDGE_REL * w_r + epos
            mz = EDGE_REL * w_z + epos
            cand = pool.query(phi_p, (w_r + mr) / R)
            if cand.size:
                dz = np.abs(pool.pos[2, cand] - z)
                cand = cand[dz <= w_z + mz]
            kids = []
            hist = tuple(c_hist[i])
            if cand.size:
                darc = np.abs(_wrap(pool.phi[cand] - phi_p)) * R
                dz = np.abs(pool.pos[2, cand] - z)
                inside_m = (darc <= w_r) & (dz <= w_z)
                edge = (np.abs(darc - w_r) <= mr) | (np.abs(dz - w_z) <= mz)
                for a in np.nonzero(edge)[0]:
                    key = ("edge", step, hist, int(pool.ids[cand[a]]))
                    flags[s] |= 1
                    near[s].append(key)
                    if key in flips:
                        inside_m[a] = not inside_m[a]
                inside = cand[inside_m]
                n_window += int(inside.size)
                if inside.size:
                    chi2, kap = _chi2(p2[i, :3], Cp, pool.pos[:, inside].T, pool.cov[:, inside])
                    sig = math.sqrt(t @ Cp @ t + prm.sigma_rphi[L] ** 2)
                    for h, c2, kp in zip(inside, chi2, kap):
                        accept = c2 <= prm.chi2_max
                        if abs(c2 - prm.chi2_max) <= chi2_error(prm.chi2_max, epos, sig, kp):
                            key = ("cut", step, hist, int(pool.ids[h]))
                            flags[s] |= 2
                            near[s].append(key)
                            if key in flips:
                                accept = not accept
                        if accept:
                            kids.append((c_score[i] + prm.hit_bonus - c2, int(pool.ids[h]), c_rank[i], i, int(h),
                                         chi2_error(c2, epos, sig, kp)))
            if not kids:
                if c_miss[i] < prm.max_miss:
                    kids.append((c_score[i] - prm.miss_penalty, MISS, c_rank[i], i, -1, 0.0))
                else:
                    kids.append(stop_child)
            children.setdefault(s, []).extend(kids)
        # ranking and selection per seed
        n_p, n_C, n_q, n_score, n_miss, n_hist, n_seed, n_rank, n_err, n_stop = [], [], [], [], [], [], [], [], [], []
        n_ovl = []
        upd = []
        for s in sorted(children):
            kids = children[s]
            kids.sort(key=lambda k: (-k[0], _KEY.get(k[1], k[1]), k[2]))
            for a in range(min(B, len(kids) - 1)):
                ka, kb = kids[a], kids[a + 1]
                d = abs(ka[0] - kb[0])
                ha, hb = c_hist[ka[3]] + [ka[1]], c_hist[kb[3]] + [kb[1]]
                ea, eb = c_err[ka[3]] + [ka[5]], c_err[kb[3]] + [kb[5]]
                d0 = next((k for k in range(len(ha)) if ha[k] != hb[k]), len(ha))
                if d == 0.0:
                    is_near = not all(_same_input(x, y) for x, y in zip(ha[d0:], hb[d0:]))
                else:
                    is_near = d <= RANK_SIGMAS * math.sqrt(sum(e * e for e in ea[d0:] + eb[d0:]))
                if is_near:
                    key = ("rank", step, tuple(ha), tuple(hb))
                    flags[s] |= 4
                    near[s].append(key)
                    if key in flips:
                        kids[a], kids[a + 1] = kb, ka
            for r, (sc, hid, prank, i, h, err) in enumerate(kids[:B]):
                n_seed.append(s)
                n_rank.append(r)
                n_score.append(sc)
                n_miss.append(c_miss[i] + (1 if hid == MISS else 0))
                n_hist.append(c_hist[i] + [hid])
                n_ovl.append(c_ovl[i] + [MISS])
                n_err.append(c_err[i] + [err])
                n_stop.append(hid == STOP)
                if hid == STOP:
                    # the state it entered the layer with (unchanged after a stop)
                    n_p.append(c_p[i])
                    n_C.append(c_C[i])
                else:
                    n_p.append(p2[i])
                    n_C.append(C2[i])
                n_q.append(c_q[i])
                if hid >= 0:
                    upd.append((len(n_p) - 1, h))
        if upd:
            k = [u[0] for u in upd]
            hs = np.array([u[1] for u in upd])
            il = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
            V = np.zeros((len(k), 3, 3))
            for c, (a, b) in enumerate(il):
                V[:, a, b] = V[:, b, a] = pool.cov[c, hs]
            pu, Cu, qu, _, su = O.update(torch.tensor(np.stack([n_p[j] for j in k])),
                                         torch.tensor(np.stack([n_C[j] for j in k])),
                                         torch.tensor([n_q[j] for j in k], dtype=torch.float64),
                                         torch.tensor(pool.pos[:, hs].T), torch.tensor(V))
            if state_round is not None:
                pu, Cu = _round(pu, Cu, state_round)
            for a, j in enumerate(k):
                n_p[j] = pu[a].numpy()
                n_C[j] = Cu[a].numpy()
                n_q[j] = float(qu[a])
                status[n_seed[j]] |= int(su[a])
            if prm.overlap:
                for j, h in upd:
                    _overlap_step(j, h, step, L, R, pool, prm, n_p, n_C, n_q, n_score, n_hist, n_ovl, n_err, n_seed,
                                  flags, near, status, flips, state_round)
        c_seed, c_rank, c_p, c_C, c_q = n_seed, n_rank, n_p, n_C, n_q
        c_score, c_miss, c_hist, c_err, c_stop = n_score, n_miss, n_hist, n_err, n_stop
        c_ovl = n_ovl
        c_layer = [L] * len(c_seed)
    hits = np.full((n, B, P), NO_CAND, np.int64)
    ovl = np.full((n, B, P), NO_CAND, np.int64)
    score = np.full((n, B), -np.inf)
    pout = np.full((n, B, 6), np.nan)
    Cout = np.full((n, B, 6, 6), np.nan)
    serr = np.zeros((n, B))
    for j, s in enumerate(c_seed):
        r = c_rank[j]
        h = c_hist[j]
        hits[s, r, :len(h)] = h
        ovl[s, r, :len(h)] = c_ovl[j]
        score[s, r] = c_score[j]
        pout[s, r] = c_p[j]
        Cout[s, r] = c_C[j]
        serr[s, r] = math.sqrt(sum(e * e for e in c_err[j]))
    return dict(hits=hits, score=score, p=pout, C=Cout, status=status, flagged=flags != 0, flags=flags, near=near,
                score_err=serr, n_window_hits=n_window, overlap=ovl)


def _window(p, C, L, R, prm):
    """The window of steps 2 (or 7) around the state p with covariance C on
    layer L of radius R: (phi_p, w_rphi, w_z, position error, r-phi spread)."""
    x, y = p[0], p[1]
    phi_p = math.atan2(y, x)
    cos_a = math.sin(p[5]) * (math.cos(p[4]) * x + math.sin(p[4]) * y) / math.hypot(x, y)
    epos = pos_error(R, cos_a)
    t = np.array([-math.sin(phi_p), math.cos(phi_p), 0.0])
    Cp = C[:3, :3]
    sig = math.sqrt(t @ Cp @ t + prm.sigma_rphi[L] ** 2)
    w_r = min(max(prm.n_sigma * sig, prm.win_min_rphi[L]), prm.win_max_rphi[L])
    w_z = min(max(prm.n_sigma * math.sqrt(Cp[2, 2] + prm.sigma_z[L] ** 2), prm.win_min_z[L]), prm.win_max_z[L])
    return phi_p, w_r, w_z, epos, sig


def _overlap_step(j, h, step, L, R, pool, prm, n_p, n_C, n_q, n_score, n_hist, n_ovl, n_err, n_seed, flags, near,
                  status, flips, state_round):
    """Step 7: the kept child j took pool hit h (layer-pool index) at this
    layer and has been updated with it.  Its overlap hit is, among the
    layer's hits on a module with a higher id than h's that lie inside the
    window around the updated state (step 2's formulas with the updated
    covariance) and have chi2 <= chi2_max against it, the one with the
    smallest chi2 (the lower hit id among equals).  The module order counts
    each pair of overlapping hits once: the child that took the pair's hit
    on the lower module can add the other, the child that took the other
    cannot add it back (two such children would carry the same two hits and,
    to rounding, the same state and score).  If there is one, the
    child is updated with it too, its score gains overlap_bonus - chi2 and
    the hit is recorded as the step's overlap hit.  Near decisions: window
    edges and the cut as in steps 2-3 (keys "ovl-edge", "ovl-cut"), and a
    second-smallest chi2 within the chi2 errors of the smallest ("ovl-pick":
    taken the other way, the second is picked)."""
    s = n_seed[j]
    p, C = n_p[j], n_C[j]
    phi_p, w_r, w_z, epos, sig = _window(p, C, L, R, prm)
    mr, mz = EDGE_REL * w_r + epos, EDGE_REL * w_z + epos
    hist = tuple(n_hist[j])
    cand = pool.query(phi_p, (w_r + mr) / R)
    if cand.size:
        cand = cand[(np.abs(pool.pos[2, cand] - p[2]) <= w_z + mz) & (pool.mods[cand] > pool.mods[h])]
    if cand.size == 0:
        return
    darc = np.abs(_wrap(pool.phi[cand] - phi_p)) * R
    dz = np.abs(pool.pos[2, cand] - p[2])
    inside = (darc <= w_r) & (dz <= w_z)
    for a in np.nonzero((np.abs(darc - w_r) <= mr) | (np.abs(dz - w_z) <= mz))[0]:
        key = ("ovl-edge", step, hist, int(pool.ids[cand[a]]))
        flags[s] |= 1
        near[s].append(key)
        if key in flips:
            inside[a] = not inside[a]
    cand = cand[inside]
    if cand.size == 0:
        return
    chi2, kap = _chi2(p[:3], C[:3, :3], pool.pos[:, cand].T, pool.cov[:, cand])
    acc = []
    for hh, c2, kp in zip(cand, chi2, kap):
        ok = c2 <= prm.chi2_max
        if abs(c2 - prm.chi2_max) <= chi2_error(prm.chi2_max, epos, sig, kp):
            key = ("ovl-cut", step, hist, int(pool.ids[hh]))
            flags[s] |= 2
            near[s].append(key)
            if key in flips:
                ok = not ok
        if ok:
            acc.append((float(c2), int(pool.ids[hh]), int(hh), chi2_error(c2, epos, sig, kp)))
    if not acc:
        return
    acc.sort(key=lambda x: (x[0], x[1]))
    pick = acc[0]
    if len(acc) > 1:
        a0, a1 = acc[0], acc[1]
        d = a1[0] - a0[0]
        if d <= RANK_SIGMAS * math.hypot(a0[3], a1[3]) and not (d == 0.0 and _same_hit(pool, a0[2], a1[2])):
            key = ("ovl-pick", step, hist, (a0[1], a1[1]))
            flags[s] |= 4
            near[s].append(key)
            if key in flips:
                pick = a1
    c2, hid, hh, err = pick
    il = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
    V = np.zeros((1, 3, 3))
    for c_, (u, v) in enumerate(il):
        V[0, u, v] = V[0, v, u] = pool.cov[c_, hh]
    pu, Cu, qu, _, su = O.update(torch.tensor(p[None]), torch.tensor(C[None]), torch.tensor([n_q[j]], dtype=torch.float64),
                                 torch.tensor(pool.pos[:, hh][None]), torch.tensor(V))
    if state_round is not None:
        pu, Cu = _round(pu, Cu, state_round)
    n_p[j], n_C[j], n_q[j] = pu[0].numpy(), Cu[0].numpy(), float(qu[0])
    status[s] |= int(su[0])
    n_score[j] = n_score[j] + prm.overlap_bonus - c2
    n_ovl[j][-1] = hid
    n_err[j][-1] = math.hypot(n_err[j][-1], err)


def _same_hit(pool, i, j):
    return bool(np.array_equal(pool.pos[:, i], pool.pos[:, j]) and np.array_equal(pool.cov[:, i], pool.cov[:, j]))


def _bears_on(key, target, current, target_ovl=None, current_ovl=None):
    """Whether taking near decision `key` the other way could move the result
    `current` [beam, P] towards `target`: an edge or cut decision on hit h
    after history H matters when exactly one of the two results has a row
    continuing H with h; a ranking between histories A and B matters when
    the two results do not hold the same rows starting with A and with B; an
    overlap decision at step k after history H (its hit at k included)
    matters when the two results' rows continuing H differ in their overlap
    hit at k (or only one has such a row)."""
    kind, step = key[0], key[1]
    if kind.startswith("ovl"):
        if target_ovl is None:
            return True
        hist = key[2]
        n = len(hist)
        at = lambda rows, ov: sorted(int(o[n - 1]) for r, o in zip(rows, ov) if tuple(r[:n]) == hist)
        return at(target, target_ovl) != at(current, current_ovl)
    if kind in ("edge", "cut"):
        hist, hid = key[2], key[3]
        has = lambda rows: any(tuple(r[:step]) == hist and r[step] == hid for r in rows)
        return has(target) != has(current)
    pre = lambda rows, h: sorted(i for i, r in enumerate(rows) if tuple(r[:len(h)]) == h)
    return any(pre(target, h) != pre(current, h) for h in (key[2], key[3]))


def valid_alternative(hits, seed_p, seed_C, seed_q, seed_layer, layer_plan, geom, pools, prm: SearchParams,
                      budget=64, overlap=None):
    """Whether the hit lists `hits` [beam, P] of one seed are one of the
    results its near decisions allow: the search is re-run with sets of its
    near decisions taken the other way, up to `budget` runs, fewest flips
    first; from each run only the near decisions that bear on the difference
    between its result and `hits` (_bears_on) are added to its flip set (all
    of them when none does).  A decision that bears on no difference cannot
    be the one that explains it, so this visits the runs that can reach
    `hits` before the others.  With `overlap` [beam, P] (the overlap hits of
    the result, prm.overlap on) the overlap hits must match too.  Returns
    (found, runs)."""
    one = lambda flips: score_hits(np.asarray(seed_p)[None], np.asarray(seed_C)[None], np.asarray([seed_q]),
                                   np.asarray([seed_layer]), layer_plan, geom, pools, prm, flips=flips)
    target = [tuple(int(x) for x in r) for r in np.asarray(hits)]
    t_ovl = None if overlap is None else [tuple(int(x) for x in r) for r in np.asarray(overlap)]
    seen = {frozenset()}
    queue = [frozenset()]
    runs = 0
    while queue and runs < budget:
        queue.sort(key=len)
        f = queue.pop(0)
        o = one(f)
        runs += 1
        if np.array_equal(o["hits"][0], hits) and (overlap is None or np.array_equal(o["overlap"][0], overlap)):
            return True, runs
        cur = [tuple(int(x) for x in r) for r in o["hits"][0]]
        c_ovl = [tuple(int(x) for x in r) for r in o["overlap"][0]]
        keys = [k for k in o["near"][0] if k not in f]
        rel = [k for k in keys if _bears_on(k, target, cur, t_ovl, c_ovl)]
        for key in (rel or keys):
            g = f | {key}
            if g not in seen:
                seen.add(g)
                queue.append(g)
    return False, runs


def replay(row, seed_p, seed_C, seed_q, seed_layer, layer_plan, geom, pools, prm: SearchParams, ovl_row=None):
    """Follow one candidate history `row` [P] (hit ids, MISS, STOP, NO_CAND)
    of one seed through the search's steps 1-6 and report whether every one
    of its decisions is one the search can take, allowing each near decision
    either way: the hit of a step lies inside its window (or near an edge)
    and has chi2 <= chi2_max (or near the cut); a miss is taken only when no
    hit of the window is accepted (up to near decisions) and the misses do
    not exceed max_miss; a stop only where the candidate cannot continue
    (no crossing, or no accepted hit with its misses spent).  Returns
    dict(valid, reason, score, err): the score the search gives that history
    and the root-sum-square of its FP32 term errors (RANK_SIGMAS of it is the
    ranking margin).  With prm.overlap, `ovl_row` [P] gives the overlap hit
    of every step (MISS for none), checked by step 7's rule with the same
    allowance: an overlap hit must be a candidate (a higher module than the
    step's hit, inside the window up to an edge, chi2 within the cut up to
    near) whose chi2 is not surely above another candidate's (by more than
    the ranking margin of the two); none may be taken only when no candidate
    is surely accepted."""
    p = torch.tensor(np.asarray(seed_p, np.float64))[None]
    C = torch.tensor(np.asarray(seed_C, np.float64))[None]
    q = torch.tensor([float(seed_q)], dtype=torch.float64)
    layer, score, errs, misses, stopped = int(seed_layer), 0.0, [], 0, False
    last_term = 0.0   # the last step's overlap term (not in the last ranking)
    row = [int(x) for x in row]
    if row and row[0] == NO_CAND:
        return dict(valid=False, reason="no candidate", score=-math.inf, err=0.0)
    for step, L in enumerate(layer_plan):
        L = int(L)
        hid = row[step]
        if stopped:
            if hid != STOP:
                return dict(valid=False, reason="continues after a stop at step %d" % step, score=score, err=0.0)
            continue
        R = float(geom.pos[L])
        p2, C2, _, st = O.propagate(p, C, q, torch.tensor([int(geom.kind[L])]), torch.tensor([R], dtype=torch.float64),
                                    torch.tensor([float(geom.x_over_x0[L])], dtype=torch.float64), geom,
                                    same=torch.tensor([layer == L]))
        if int(st[0]) & O.NO_CROSSING:
            if hid != STOP:
                return dict(valid=False, reason="no crossing at step %d" % step, score=score, err=0.0)
            stopped = True
            continue
        pp, Cp = p2[0].numpy(), C2[0].numpy()[:3, :3]
        x, y, z = pp[0], pp[1], pp[2]
        phi_p = math.atan2(y, x)
        cos_a = math.sin(pp[5]) * (math.cos(pp[4]) * x + math.sin(pp[4]) * y) / math.hypot(x, y)
        epos = pos_error(R, cos_a)
        t = np.array([-math.sin(phi_p), math.cos(phi_p), 0.0])
        sig = math.sqrt(t @ Cp @ t + prm.sigma_rphi[L] ** 2)
        w_r = min(max(prm.n_sigma * sig, prm.win_min_rphi[L]), prm.win_max_rphi[L])
        w_z = min(max(prm.n_sigma * math.sqrt(Cp[2, 2] + prm.sigma_z[L] ** 2), prm.win_min_z[L]), prm.win_max_z[L])
        mr, mz = EDGE_REL * w_r + epos, EDGE_REL * w_z + epos
        a, b = int(pools.layer_offsets[L]), int(pools.layer_offsets[L + 1])
        pos = np.asarray(pools.pos[:, a:b], np.float64)
        cov = np.asarray(pools.cov[:, a:b], np.float64)
        ids = np.asarray(pools.hit_id[a:b], np.int64)
        darc = np.abs(_wrap(np.arctan2(pos[1], pos[0]) - phi_p)) * R
        dz = np.abs(pos[2] - z)
        surely_in = (darc <= w_r - mr) & (dz <= w_z - mz)
        maybe_in = (darc <= w_r + mr) & (dz <= w_z + mz)
        sel = np.nonzero(maybe_in)[0]
        chi2 = np.zeros(0)
        kap = np.zeros(0)
        if sel.size:
            chi2, kap = _chi2(pp[:3], Cp, pos[:, sel].T, cov[:, sel])
        cerr = np.array([chi2_error(prm.chi2_max, epos, sig, k_) for k_ in kap])
        surely_acc = surely_in[sel] & (chi2 < prm.chi2_max - cerr)
        if hid >= 0:
            j = np.nonzero(ids[sel] == hid)[0]
            if j.size == 0:
                return dict(valid=False, reason="hit %d outside the window at step %d" % (hid, step), score=score,
                            err=0.0)
            j = int(j[0])
            if not chi2[j] <= prm.chi2_max + cerr[j]:
                return dict(valid=False, reason="hit %d above the cut at step %d" % (hid, step), score=score, err=0.0)
            score += prm.hit_bonus - float(chi2[j])
            errs.append(chi2_error(float(chi2[j]), epos, sig, float(kap[j])))
            il = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
            V = torch.zeros(1, 3, 3, dtype=torch.float64)
            for c_, (u, v) in enumerate(il):
                V[0, u, v] = V[0, v, u] = float(cov[c_, sel[j]])
            p, C, q, _, _ = O.update(p2, C2, q, torch.tensor(pos[:, sel[j]][None]), V)
            if prm.overlap:
                mods = np.asarray(pools.module[a:b], np.int64)
                r_ = _replay_overlap(int(ovl_row[step]) if ovl_row is not None else MISS, int(mods[sel[j]]), p, C, q,
                                     L, R, pos, cov, ids, mods, prm)
                if not r_["valid"]:
                    return dict(valid=False, reason="%s at step %d" % (r_["reason"], step), score=score, err=0.0)
                if r_["taken"]:
                    p, C, q = r_["p"], r_["C"], r_["q"]
                    score += prm.overlap_bonus - r_["chi2"]
                    errs[-1] = math.hypot(errs[-1], r_["err"])
                    if step == len(layer_plan) - 1:
                        last_term = prm.overlap_bonus - r_["chi2"]
        elif hid == MISS:
            if surely_acc.any():
                return dict(valid=False, reason="miss at step %d with an accepted hit" % step, score=score, err=0.0)
            if misses >= prm.max_miss:
                return dict(valid=False, reason="miss beyond max_miss at step %d" % step, score=score, err=0.0)
            misses += 1
            score -= prm.miss_penalty
            errs.append(0.0)
            p, C = p2, C2
        elif hid == STOP:
            if surely_acc.any() or misses < prm.max_miss:
                return dict(valid=False, reason="stop at step %d where the candidate can continue" % step,
                            score=score, err=0.0)
            stopped = True
        else:
            return dict(valid=False, reason="no candidate at step %d" % step, score=score, err=0.0)
        layer = L
    return dict(valid=True, reason="", score=score, err=math.sqrt(sum(e * e for e in errs)),
                rank_score=score - last_term)


def _replay_overlap(oid, mod_h, p, C, q, L, R, pos, cov, ids, mods, prm):
    """Step 7 for replay: whether overlap hit `oid` (MISS: none) is one the
    step can take after the update (p, C, q) with a hit on module mod_h."""
    pp, Cp = p[0].numpy(), C[0].numpy()
    phi_p, w_r, w_z, epos, sig = _window(pp, Cp, L, R, prm)
    mr, mz = EDGE_REL * w_r + epos, EDGE_REL * w_z + epos
    darc = np.abs(_wrap(np.arctan2(pos[1], pos[0]) - phi_p)) * R
    dz = np.abs(pos[2] - pp[2])
    maybe = np.nonzero((darc <= w_r + mr) & (dz <= w_z + mz) & (mods > mod_h))[0]
    surely_in = (darc[maybe] <= w_r - mr) & (dz[maybe] <= w_z - mz)
    if maybe.size:
        chi2, kap = _chi2(pp[:3], Cp[:3, :3], pos[:, maybe].T, cov[:, maybe])
    else:
        chi2, kap = np.zeros(0), np.zeros(0)
    cerr = np.array([chi2_error(prm.chi2_max, epos, sig, k_) for k_ in kap])
    terr = np.array([chi2_error(float(c_), epos, sig, float(k_)) for c_, k_ in zip(chi2, kap)])
    maybe_acc = chi2 <= prm.chi2_max + cerr
    surely_acc = surely_in & (chi2 < prm.chi2_max - cerr)
    if oid == MISS:
        if surely_acc.any():
            return dict(valid=False, reason="no overlap hit with one surely accepted", taken=False)
        return dict(valid=True, taken=False)
    j = np.nonzero(ids[maybe] == oid)[0]
    if j.size == 0:
        return dict(valid=False, reason="overlap hit %d not a candidate" % oid, taken=False)
    j = int(j[0])
    if not maybe_acc[j]:
        return dict(valid=False, reason="overlap hit %d above the cut" % oid, taken=False)
    for k in np.nonzero(surely_acc)[0]:
        if chi2[k] < chi2[j] - RANK_SIGMAS * math.hypot(terr[k], terr[j]):
            return dict(valid=False, reason="overlap hit %d surely worse than %d" % (oid, int(ids[maybe][k])),
                        taken=False)
    il = [(0, 0), (1, 0), (1, 1), (2, 0), (2, 1), (2, 2)]
    V = torch.zeros(1, 3, 3, dtype=torch.float64)
    for c_, (u, v) in enumerate(il):
        V[0, u, v] = V[0, v, u] = float(cov[c_, maybe[j]])
    p2, C2, q2, _, _ = O.update(p, C, q, torch.tensor(pos[:, maybe[j]][None]), V)
    return dict(valid=True, taken=True, p=p2, C=C2, q=q2, chi2=float(chi2[j]), err=float(terr[j]))


def consistent_result(hits, scores, seed_p, seed_C, seed_q, seed_layer, layer_plan, geom, pools, prm: SearchParams,
                      oracle_hits, oracle_scores, oracle_err, overlap=None, oracle_overlap=None):
    """Whether one seed's lists `hits` [beam, P] with their `scores` [beam]
    are a result the search can give when its near decisions and its
    rankings are resolved within the FP32 error model, against the oracle's
    own result for that seed (oracle_hits, oracle_scores, oracle_err):
    * every list is a history the search can take (replay), and its score
      agrees with the replayed score to 1e-3 + RANK_SIGMAS * its error;
    * the lists are distinct and in score order (descending, to the same
      margin);
    * an oracle list missing from `hits` scores no more than the lowest of
      `hits` (replayed) plus the ranking margin of the two, and a list of
      `hits` missing from the oracle's scores no less than the oracle's
      lowest kept list minus that margin: within the error model either
      could take the other's place.
    With prm.overlap, a list is its hits and overlap hits together
    (`overlap`, `oracle_overlap` [beam, P]).
    Returns (ok, reason)."""
    if overlap is not None:
        rows = [tuple(int(x) for x in r) + tuple(int(x) for x in o) for r, o in zip(np.asarray(hits), overlap)]
        orows_ = [tuple(int(x) for x in r) + tuple(int(x) for x in o)
                  for r, o in zip(np.asarray(oracle_hits), oracle_overlap)]
    else:
        rows = [tuple(int(x) for x in r) for r in np.asarray(hits)]
        orows_ = None
    P_ = np.asarray(hits).shape[1]
    live = [i for i, r in enumerate(rows) if r[0] != NO_CAND]
    if len(set(rows[i] for i in live)) != len(live):
        return False, "duplicate lists"
    rep = {}
    for i in live:
        r = replay(rows[i][:P_], seed_p, seed_C, seed_q, seed_layer, layer_plan, geom, pools, prm,
                   ovl_row=rows[i][P_:] if overlap is not None else None)
        if not r["valid"]:
            return False, "list %d: %s" % (i, r["reason"])
        if abs(float(scores[i]) - r["score"]) > 1e-3 + RANK_SIGMAS * r["err"]:
            return False, "list %d: score %.6f against %.6f +- %.3g" % (i, float(scores[i]), r["score"], r["err"])
        rep[rows[i]] = r
    for a, b in zip(live[:-1], live[1:]):
        # the order of the last ranking (its scores hold no overlap term of
        # the last layer)
        m = 1e-3 + RANK_SIGMAS * math.hypot(rep[rows[a]]["err"], rep[rows[b]]["err"])
        if rep[rows[a]]["rank_score"] < rep[rows[b]]["rank_score"] - m:
            return False, "lists %d and %d out of score order" % (a, b)
    orows = orows_ if orows_ is not None else [tuple(int(x) for x in r) for r in np.asarray(oracle_hits)]
    olive = [i for i, r in enumerate(orows) if r[0] != NO_CAND]
    if len(olive) != len(live):
        return False, "%d lists against the oracle's %d" % (len(live), len(olive))
    if not live:
        return True, ""
    low = min(live, key=lambda i: rep[rows[i]]["score"])
    olow = min(olive, key=lambda i: float(oracle_scores[i]))
    for i in olive:
        if orows[i] in rep:
            continue
        m = 1e-3 + RANK_SIGMAS * math.hypot(float(oracle_err[i]), rep[rows[low]]["err"])
        if float(oracle_scores[i]) > rep[rows[low]]["score"] + m:
            return False, "oracle list %d (score %.6f) missing above the lowest kept %.6f" % (
                i, float(oracle_scores[i]), rep[rows[low]]["score"])
    for i in live:
        if rows[i] in orows:
            continue
        m = 1e-3 + RANK_SIGMAS * math.hypot(rep[rows[i]]["err"], float(oracle_err[olow]))
        if rep[rows[i]]["score"] < float(oracle_scores[olow]) - m:
            return False, "list %d (score %.6f) below the oracle's lowest kept %.6f" % (
                i, rep[rows[i]]["score"], float(oracle_scores[olow]))
    return True, ""
