"""The seeded generator: determinism, hits on their surfaces, plausible
length distributions and noise pools."""
import numpy as np

from toygen import generate, make_pools, workloads


def test_deterministic():
    wl = workloads()["mixed26"]
    a = generate(wl, 500)
    b = generate(wl, 500)
    assert np.array_equal(a.hit_pos, b.hit_pos) and np.array_equal(a.hit_valid, b.hit_valid)


def test_hits_on_surfaces_and_lengths():
    for name in ("barrel10", "mixed26"):
        wl = workloads()[name]
        ev = generate(wl, 2000)
        g = wl.geometry
        kind = g.kind[ev.hit_layer]
        r = np.hypot(ev.hit_pos[0], ev.hit_pos[1])
        b = kind == 0
        assert np.abs(r[b] - g.pos[ev.hit_layer[b]]).max() < 1e-9
        if (~b).any():
            assert np.abs(ev.hit_pos[2, ~b] - g.pos[ev.hit_layer[~b]]).max() < 1e-12
        L = ev.lengths()
        assert L.min() >= 3 and L.max() <= 26
        nv = np.add.reduceat(ev.hit_valid.astype(int), ev.hit_offsets[:-1])
        assert nv.min() >= 3
    wl = workloads()["barrel10"]
    L = generate(wl).lengths()
    # pT < 0.63 GeV cannot reach r = 110 cm: ~7.5% of tracks stop at nine hits
    assert 0.05 < (L == 9).mean() < 0.10 and set(np.unique(L)) <= {9, 10}


def test_early_stops_cover_short_lengths():
    """A quarter of the mixed-detector batch's central tracks end after
    3 .. n of their n crossings, so that the batch holds every length from 3
    to 26, and every track can still be seeded."""
    wl = workloads()["mixed26"]
    L = generate(wl, 20_000).lengths()
    assert L.min() == 3 and L.max() <= 26
    assert set(range(3, 9)) <= set(np.unique(L).tolist())
    assert 0.03 < (L < 9).mean() < 0.09


def test_hole_fraction():
    wl = workloads()["mixed26"]
    ev = generate(wl, 5000)
    assert 0.04 < 1.0 - ev.hit_valid.mean() < 0.06


def test_noise_pool_density():
    wl = workloads()["search20"]
    ev = generate(wl, 200)
    pools = make_pools(wl, ev)
    g = wl.geometry
    for lay in (3, 10, 19):
        n = pools.layer_offsets[lay + 1] - pools.layer_offsets[lay]
        area = 2 * np.pi * g.pos[lay] * 300.0
        ntrue = ((ev.hit_layer == lay) & (ev.hit_valid == 1)).sum()
        assert abs(n - ntrue - 2.0 * area) <= 1
