"""Inputs of the combinatorial-search tests: seeded toy tracks through the
20-layer barrel, per-layer pools of their hits plus uniform noise, and seeds
= the FP64 oracle's Kalman fit of each track's first three hits (state on the
third layer), rounded to FP32 so that the oracle and the FP32 GPU path start
from identical values."""
from __future__ import annotations

import numpy as np
import torch

from oracle import kf_oracle as O
from oracle.kf_search import SearchParams
from toygen import generate, truncate, with_modules, workloads
from toygen.generate import make_pools

PLAN = list(range(3, 20))
SEED_LAYER = 2


def f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def seeds_from_three_hits(ev, geom):
    tr = truncate(ev, np.full(ev.n_tracks, 3))
    hp = f32(tr.hit_pos)
    sp, sC, sq, _ = O.make_seeds(tr.hit_offsets, tr.hit_valid, hp, geom.bz)
    fo = O.fit_tracks(sp, sC, sq, tr.hit_offsets, tr.hit_layer, tr.hit_valid, torch.tensor(hp), f32(tr.hit_cov), geom)
    return f32(fo["p"].numpy()), f32(fo["C"].numpy()), fo["q"].numpy().astype(np.float64)


def search_inputs(n=None, noise=True):
    """(workload, event, geometry, pools, seed_p [n,6], seed_C [n,6,6], seed_q [n]);
    pool positions and covariances are FP32-representable."""
    wl = workloads()["search20"]
    ev = generate(wl, n)
    g = wl.geometry
    pools = make_pools(wl, ev, first_layer=3, noise=noise)
    pools.pos = f32(pools.pos)
    pools.cov = f32(pools.cov)
    p, C, q = seeds_from_three_hits(ev, g)
    return wl, ev, g, pools, p, C, q


def default_params(g, beam=6):
    return SearchParams(g.n_layers, beam=beam)


def module_inputs(n=None, noise=True):
    """search_inputs with the pools split into detector modules with overlap
    hits (toygen.with_modules), FP32-representable."""
    wl, ev, g, pools, p, C, q = search_inputs(n, noise)
    P = with_modules(wl, ev, pools)
    P.pos = f32(P.pos)
    P.cov = f32(P.cov)
    return wl, ev, g, P, p, C, q
