"""Autotuner for the fused fit launch.

Within a family of hit layouts every launch shape of kf_fit_tracks computes
bit-identical results, and the two families (direct reads, LDS staging) agree
to rounding, so the tuner only measures: it times each candidate (threads per block, plain or
persistent grid, blocks per compute unit for the persistent grid, and the
kernel variant compiled for one or two waves per SIMD) on the caller's own
inputs with HIP events on the current stream, together with the hit layout
(track order, length-sorted, length-sorted and packed, or either order
staged through LDS by the fit kernel -- the sorting and packing passes are
part of the timed call), keeps the fastest, sets it in
the context and records it in a JSON cache keyed by (operation, precision,
track-count class, device name)."""
from __future__ import annotations

import json
import math
import os

import torch

from . import kf as K

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "kf_autotune.json")


def candidates(layouts=(0, 1, 2, 3, 4)):
    """(block, persistent, blocks_per_cu, waves, layout) shapes to time."""
    out = []
    for layout in layouts:
        for waves in (1, 2):
            for block in (64, 128, 256):
                out.append((block, 0, 1, waves, layout))
                for bpc in (4, 8):
                    out.append((block, 1, bpc, waves, layout))
    return out


def size_class(n: int) -> int:
    """Tracks rounded to a power of two (the key of the cache)."""
    return 1 << max(0, int(math.ceil(math.log2(max(n, 1)))))


def _key(dtype, n, device_name):
    return f"fit_tracks|{str(dtype).replace('torch.', '')}|{size_class(n)}|{device_name}"


def load_cache(path=DEFAULT_CACHE):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache, path=DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_ms(fn, reps=5, warmup=2):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune_fit(ctx: K.Context, fit_fn, dtype, n, reps=5, cands=None, cache_path=DEFAULT_CACHE, use_cache=True):
    """Time ``fit_fn()`` (a closure that calls ctx.fit_tracks on fixed inputs)
    for every candidate launch shape; set and return the fastest.
    Returns (best, table) with table = [(shape, ms), ...]."""
    dev_name = torch.cuda.get_device_name(ctx.device)
    key = _key(dtype, n, dev_name)
    cache = load_cache(cache_path) if use_cache else {}
    if use_cache and key in cache:
        best = tuple(cache[key]["shape"])
        ctx.set_fit_launch(dtype, *best)
        return best, cache[key].get("table", [])
    table = []
    for shape in (cands or candidates()):
        ctx.set_fit_launch(dtype, *shape)
        table.append((shape, time_ms(fit_fn, reps)))
    best = min(table, key=lambda x: x[1])[0]
    ctx.set_fit_launch(dtype, *best)
    if cache_path:
        cache = load_cache(cache_path)
        cache[key] = {"shape": list(best), "table": [[list(s), ms] for s, ms in table]}
        save_cache(cache, cache_path)
    return best, table
