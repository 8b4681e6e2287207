"""FP64 CPU oracle of duplicate removal among found tracks (kf_remove_duplicates).
TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module; it shares no code with the HIP
kernels.

The paper's track finding ends, per seed, with the best-scoring candidate,
and removes duplicate tracks, found from different seeds, by the hits they
share (Sec. 2.2); it gives no rule.  Reading taken here:

* Each seed contributes one track: its best candidate (rank 0 of the
  search), a list of hit ids with one entry per layer of the plan (-1 a miss,
  -2 no candidate at all).
* n(t) is the number of hit ids >= 0 of track t; shared(t, u) the number of
  layers at which t and u carry the same hit id >= 0.
* t and u are duplicates iff shared(t, u) >= 1 and
  shared(t, u) >= frac * min(n(t), n(u)).
* u outranks t iff score(u) > score(t), or the scores are equal and u < t.
* t is removed iff some u that outranks it is its duplicate (pairwise rule:
  whether that u is itself removed does not matter).  dup_of(t) is then the
  highest-ranked such u, else -1.  A track without a candidate (score
  -inf) is removed and cannot remove others (dup_of = -1).

Consequences, pinned in the tests: no two kept tracks are duplicates; a set
of identical tracks keeps exactly its highest-ranked member; disjoint tracks
are all kept.
"""
from __future__ import annotations

import numpy as np


def _outranks(score, u, t):
    return score[u] > score[t] or (score[u] == score[t] and u < t)


def remove_duplicates(hits, score, frac):
    """hits [n, L] int (hit id, -1 miss, -2 none), score [n] float, 0 < frac
    <= 1.  Returns keep [n] bool, dup_of [n] int64.  Candidate pairs come from
    an index of hit id -> tracks carrying it at that layer."""
    hits = np.asarray(hits, np.int64)
    score = np.asarray(score, np.float64)
    n, L = hits.shape
    nh = (hits >= 0).sum(axis=1)
    none = ~(score > -np.inf)
    index = {}
    for t in range(n):
        if none[t]:
            continue
        for l in range(L):
            h = hits[t, l]
            if h >= 0:
                index.setdefault((l, int(h)), []).append(t)
    keep = ~none
    dup_of = np.full(n, -1, np.int64)
    for t in range(n):
        if none[t]:
            continue
        partners = set()
        for l in range(L):
            h = hits[t, l]
            if h >= 0:
                partners.update(index[(l, int(h))])
        partners.discard(t)
        best = -1
        for u in sorted(partners):
            shared = int(((hits[t] == hits[u]) & (hits[t] >= 0)).sum())
            if shared >= 1 and shared >= frac * min(nh[t], nh[u]) and _outranks(score, u, t):
                if best < 0 or _outranks(score, u, best):
                    best = u
        if best >= 0:
            keep[t] = False
            dup_of[t] = best
    return keep, dup_of


def remove_duplicates_brute(hits, score, frac):
    """The same rule over all pairs (small inputs only)."""
    hits = np.asarray(hits, np.int64)
    score = np.asarray(score, np.float64)
    n, _ = hits.shape
    nh = (hits >= 0).sum(axis=1)
    none = ~(score > -np.inf)
    keep = ~none
    dup_of = np.full(n, -1, np.int64)
    for t in range(n):
        if none[t]:
            continue
        for u in range(n):
            if u == t or none[u]:
                continue
            shared = int(((hits[t] == hits[u]) & (hits[t] >= 0)).sum())
            if shared >= 1 and shared >= frac * min(nh[t], nh[u]) and _outranks(score, u, t):
                if dup_of[t] < 0 or _outranks(score, u, dup_of[t]):
                    dup_of[t] = u
        keep[t] = keep[t] and dup_of[t] < 0
    return keep, dup_of
