"""Seeded synthetic lists of found tracks (one hit id per layer of a plan)
with planted duplicates, as a track finder hands them to duplicate removal."""
from __future__ import annotations

import numpy as np


def duplicate_candidates(n, n_layers=17, dup_frac=0.3, miss_prob=0.05, none_prob=0.01, seed=0):
    """hits [n, n_layers] int32 and score [n] float32.  Base tracks carry
    distinct hit ids (layer l uses ids l * 2^24 + k); a fraction dup_frac of
    the tracks copy a random earlier track and replace a random number of its
    hits (0 .. n_layers / 2) by misses or fresh ids; misses (-1) at random;
    a fraction none_prob have no candidate (all -2, score -inf).  Scores:
    10 per hit minus a chi2-like term, rounded to 1/8 so that ties occur."""
    rng = np.random.default_rng(seed)
    hits = np.empty((n, n_layers), np.int64)
    fresh = np.zeros(n_layers, np.int64)

    def new_id(l):
        fresh[l] += 1
        return l * (1 << 24) + fresh[l]

    for t in range(n):
        if t > 0 and rng.random() < dup_frac:
            src = int(rng.integers(0, t))
            hits[t] = hits[src]
            k = int(rng.integers(0, n_layers // 2 + 1))
            for l in rng.choice(n_layers, size=k, replace=False):
                hits[t, l] = -1 if rng.random() < 0.5 else new_id(l)
        else:
            for l in range(n_layers):
                hits[t, l] = -1 if rng.random() < miss_prob else new_id(l)
    nh = (hits >= 0).sum(axis=1)
    score = np.round((10.0 * nh - rng.gamma(nh.clip(1), 1.0)) * 8.0) / 8.0
    none = rng.random(n) < none_prob
    hits[none] = -2
    score[none] = -np.inf
    return hits.astype(np.int32), score.astype(np.float32)
