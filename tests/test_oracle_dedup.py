"""Pins for the duplicate-removal oracle (oracle/kf_dedup.py): a hand-worked
example, brute force over all pairs on small inputs, the invariants the rule
implies (no two kept tracks are duplicates; every removed track names a
higher-ranked duplicate), exact copies, and the subset case frac = 1."""
import numpy as np
import pytest

from oracle import kf_dedup as D
from toygen import duplicate_candidates


def _shared(a, b):
    return int(((a == b) & (a >= 0)).sum())


def _is_dup(hits, t, u, frac):
    s = _shared(hits[t], hits[u])
    return s >= 1 and s >= frac * min((hits[t] >= 0).sum(), (hits[u] >= 0).sum())


def test_hand_worked_example():
    """Five tracks over four layers, frac 0.5 (worked by hand):
    t1 shares 3 of its 3 hits with t0 and t4 (both outrank it; t0 ranks
    higher on the index) -> removed, dup_of 0; t2 shares 1 hit (< 2) with t0
    and 2 of 2 with t3, which outranks it -> removed, dup_of 3; t3 and t0
    kept; t4 is a copy of t0 with the same score -> removed, dup_of 0."""
    hits = np.array([[1, 2, 3, 4], [1, 2, 3, -1], [7, 8, 3, 9], [7, 8, -1, -1], [1, 2, 3, 4]])
    score = np.array([40.0, 30.0, 35.0, 50.0, 40.0])
    keep, dup_of = D.remove_duplicates(hits, score, 0.5)
    assert keep.tolist() == [True, False, False, True, False]
    assert dup_of.tolist() == [-1, 0, 3, -1, 0]


@pytest.mark.parametrize("seed,frac", [(1, 0.5), (2, 0.3), (3, 0.75), (4, 1.0)])
def test_brute_force_agrees(seed, frac):
    hits, score = duplicate_candidates(250, n_layers=9, seed=seed)
    a = D.remove_duplicates(hits, score, frac)
    b = D.remove_duplicates_brute(hits, score, frac)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_invariants():
    frac = 0.5
    hits, score = duplicate_candidates(600, seed=5)
    keep, dup_of = D.remove_duplicates(hits, score, frac)
    none = score == -np.inf
    assert not keep[none].any() and (dup_of[none] == -1).all()
    kept = np.nonzero(keep)[0]
    for i, t in enumerate(kept):
        for u in kept[i + 1:]:
            assert not _is_dup(hits, t, u, frac), (t, u)
    for t in np.nonzero(~keep & ~none)[0]:
        u = dup_of[t]
        assert u >= 0 and _is_dup(hits, t, u, frac)
        assert score[u] > score[t] or (score[u] == score[t] and u < t)
    assert 0.3 < keep.mean() < 0.95


def test_exact_copies_keep_the_first():
    base, s = duplicate_candidates(200, dup_frac=0.0, none_prob=0.0, seed=6)
    hits = np.concatenate([base, base])
    score = np.concatenate([s, s])
    keep, dup_of = D.remove_duplicates(hits, score, 0.5)
    has = (base >= 0).any(axis=1)
    assert keep[:200][has].all() and not keep[200:][has].any()
    assert np.array_equal(dup_of[200:][has], np.arange(200)[has])


def test_frac_one_means_contained():
    """With frac = 1 a pair is a duplicate only if the shorter track's hits
    all lie on the longer one."""
    hits = np.array([[1, 2, 3, 4], [1, 2, -1, -1], [1, 2, 5, -1]])
    score = np.array([40.0, 20.0, 30.0])
    keep, dup_of = D.remove_duplicates(hits, score, 1.0)
    assert keep.tolist() == [True, False, True]
    assert dup_of.tolist() == [-1, 0, -1]
