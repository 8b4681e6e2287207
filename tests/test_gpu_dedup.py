"""GPU parity of duplicate removal (kf_remove_duplicates) with the oracle
(oracle/kf_dedup.py) on seeded candidate lists with planted duplicates and
score ties: keep and dup_of bit-exact, at sizes from one track to beyond the
search benchmark's 20,000 seeds, for several sharing fractions, from
contiguous and from strided inputs (the rank-0 slice of a search output)."""
from __future__ import annotations

import os
import sys

import numpy as np
import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from oracle import kf_dedup as D
from toygen import duplicate_candidates

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def kf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_11728_amd import kf as _kf
    return _kf


@pytest.fixture(scope="module")
def ctx(kf):
    c = kf.Context(0)
    yield c
    c.close()


def _gpu(ctx, hits, score, frac):
    dev = ctx.device
    keep, dup = ctx.remove_duplicates(torch.tensor(hits, device=dev), torch.tensor(score, device=dev), frac)
    torch.cuda.synchronize()
    return keep.cpu().numpy().astype(bool), dup.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("n,frac,seed", [(1, 0.5, 1), (63, 0.5, 2), (300, 0.3, 3), (5000, 0.5, 4), (5000, 1.0, 5),
                                         (20000, 0.5, 6), (50000, 0.75, 7), (200000, 0.5, 12)])
def test_dedup_parity(ctx, kf, n, frac, seed):
    say("dedup", n, frac)
    hits, score = duplicate_candidates(n, seed=seed)
    ok, od = D.remove_duplicates(hits, score, np.float32(frac))
    gk, gd = _gpu(ctx, hits, score, frac)
    assert np.array_equal(gk, ok), int((gk != ok).sum())
    assert np.array_equal(gd, od), int((gd != od).sum())
    say("kept", int(gk.sum()), "of", n)


def test_dedup_strided_rank0_of_a_search_output(ctx, kf):
    """The tracks as rank 0 of [n, beam, L] hits and [n, beam] scores."""
    n, beam, L = 3000, 6, 17
    hits, score = duplicate_candidates(n, n_layers=L, seed=8)
    rng = np.random.default_rng(9)
    H = rng.integers(-2, 1 << 20, size=(n, beam, L)).astype(np.int32)
    S = rng.random((n, beam)).astype(np.float32)
    H[:, 0, :] = hits
    S[:, 0] = score
    dev = ctx.device
    Ht, St = torch.tensor(H, device=dev), torch.tensor(S, device=dev)
    keep, dup = ctx.remove_duplicates(Ht[:, 0, :], St[:, 0], 0.5)
    torch.cuda.synchronize()
    ok, od = D.remove_duplicates(hits, score, 0.5)
    assert np.array_equal(keep.cpu().numpy().astype(bool), ok)
    assert np.array_equal(dup.cpu().numpy().astype(np.int64), od)


def test_dedup_repeated_calls_and_sizes(ctx, kf):
    """The workspace grows and is reused: a large call, a small one, the
    large one again; same answers each time."""
    big = duplicate_candidates(30000, seed=10)
    small = duplicate_candidates(100, seed=11)
    r1 = _gpu(ctx, *big, 0.5)
    r2 = _gpu(ctx, *small, 0.5)
    r3 = _gpu(ctx, *big, 0.5)
    assert np.array_equal(r1[0], r3[0]) and np.array_equal(r1[1], r3[1])
    o2 = D.remove_duplicates(*small, 0.5)
    assert np.array_equal(r2[0], o2[0]) and np.array_equal(r2[1], o2[1])
