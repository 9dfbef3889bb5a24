"""The seeded input recipes produce the statistics their docstrings state
(CPU).  These pin the stand-ins for the paper's unpublished geometries."""
import math

import numpy as np

from paper_2407_03343_amd import workloads as wl


def _pair_gaps(c):
    d = np.sqrt(((c[:, None, :] - c[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    return d - 2.0


def test_two_sphere_gap():
    pk, rbm = wl.workload_two_sphere_gap001()
    assert abs(_pair_gaps(pk.centers)[0, 1] - 0.01) < 1e-14
    assert np.allclose(rbm[0, 1, :3] - rbm[0, 0, :3], [1.0, 0, 0])


def test_cluster100_recipe():
    pk, rbm = wl.workload_cluster100(0)
    g = pk.min_gaps()
    assert pk.P == 100 and rbm.shape == (1, 100, 6)
    assert g.min() >= 1e-3 * (1 - 1e-9) and np.all(g <= 1e-1 + 1e-9)
    assert np.all(pk.centers >= 1.0 - 1e-12) and np.all(pk.centers <= pk.box - 1.0 + 1e-12)
    phi = 100 * 4 * math.pi / 3 / pk.box ** 3
    assert abs(phi - 0.2) < 1e-12


def test_packing_recipe_pairs_and_gaps():
    pk = wl.workload_packing2000(400, seed=3)
    G = _pair_gaps(pk.centers)
    assert G.min() >= 1e-3 * (1 - 1e-9)
    close = np.where(G.min(1) < 1e-2 + 1e-12)[0]
    # 5% of the spheres in pairs (up to the ones the pull could not place)
    assert 0.03 * pk.P <= close.size <= 0.05 * pk.P + 1
    # every other gap stays at least 0.1 (the pulled pairs keep 0.1 to the rest)
    others = np.setdiff1d(np.arange(pk.P), close)
    assert G[np.ix_(others, others)].min() >= 0.2 - 1e-9


def test_block500_recipe():
    pk, rbm = wl.workload_block500(500, seed=0)
    g = pk.min_gaps()
    assert rbm.shape == (64, 500, 6)
    assert abs(500 * 4 * math.pi / 3 / pk.box ** 3 - 0.35) < 1e-12
    assert 0.35 <= np.mean(g < 5e-2 + 1e-12) <= 0.42
    assert g.min() >= 1e-3 * (1 - 1e-9)


def test_serving_stream_statistics():
    reqs = wl.serving_stream(n=40, rate=200.0, seed=1)
    t = np.array([r["t"] for r in reqs])
    assert t[0] == 0.0 and np.all(np.diff(t) > 0)
    # mean inter-arrival 1/200 s within sampling error of 39 draws
    assert 0.5 / 200 < np.diff(t).mean() < 2.0 / 200
    for r in reqs:
        assert 2 <= r["P"] <= 200
        assert 0.1 <= r["phi"] <= 0.3 and r["phi_actual"] <= r["phi"] + 1e-12
        assert 1e-3 <= r["gap_min"] <= 1e-1
        if r["P"] > 1:
            assert _pair_gaps(r["centers"]).min() >= r["gap_min"] * (1 - 1e-9)
        assert r["rbm"].shape == (r["P"], 6)
