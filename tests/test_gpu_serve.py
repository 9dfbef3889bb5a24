"""Serving (continuous batching of independent solves) through the C-ABI.

A request's result must not depend on the company it keeps: every request
of a mixed stream is compared with the same request served alone, with the
library's single-problem solve, and one request with the FP64 oracle.
Requests use a small discretisation so that the per-contact SVDs of the
set-up stay cheap.
"""
import numpy as np
import pytest

from oracle import geometry as geo, mfs
from paper_2407_03343_amd import workloads as wl

from gpu_common import _say, _t, _n

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DISC = dict(n_proxy=60, n_colloc_base=80, n_image=4, n_check_base=0)
# the single-problem comparison solves stop on the recursive estimate, as the
# served requests do (true-residual guard off)
SOLVER = dict(gmres_tol=1e-10, gmres_restart=60, gmres_max_it=3000, gmres_check_every=0)


@pytest.fixture(scope="module")
def stream():
    return wl.serving_stream(n=10, rate=200.0, P_lo=2, P_hi=12, seed=5)


@pytest.fixture(scope="module")
def mixed_run(dev, stream):
    _say("serving: 10 requests (2..12 spheres) through one server, 8 slots")
    srv = dev.Server(arena_bytes=2 << 30, max_active=8, **DISC, **SOLVER)
    ids = [srv.submit(r["centers"], r["rbm"]) for r in stream]
    srv.drain(timeout_s=120)
    res = [srv.poll(i, r["P"]) for i, r in zip(ids, stream)]
    st = srv.stats()
    srv.close()
    _say(f"  stats {st}")
    return res, st


def test_serving_completes_and_batches(mixed_run, stream):
    res, st = mixed_run
    assert all(r is not None and r["status"] == 0 for r in res)
    assert st["completed"] == len(stream) and st["failed"] == 0
    assert st["peak_active"] > 1                      # requests shared launches
    for r in res:
        assert r["true_rel_residual"] < 1e-6
        assert r["t_arrival"] <= r["t_admitted"] <= r["t_started"] <= r["t_done"]


def test_serving_alone_equals_in_mix(dev, mixed_run, stream):
    res, _ = mixed_run
    for k in (0, 4, 9):
        r = stream[k]
        _say(f"  request {k} (P={r['P']}) alone")
        srv = dev.Server(arena_bytes=1 << 30, max_active=1, **DISC, **SOLVER)
        i = srv.submit(r["centers"], r["rbm"])
        srv.drain(timeout_s=60)
        alone = srv.poll(i, r["P"])
        srv.close()
        assert alone["iterations"] == res[k]["iterations"]
        scale = np.abs(alone["ft"]).max()
        assert np.abs(alone["ft"] - res[k]["ft"]).max() <= 1e-12 * scale


def test_serving_matches_single_problem_solve(dev, mixed_run, stream):
    res, _ = mixed_run
    for k in (1, 6):
        r = stream[k]
        pb = dev.Problem(r["centers"], 1.0, **DISC, **SOLVER).bind().setup()
        out = pb.solve_resistance(_t(r["rbm"]), want_check=False)
        ft = _n(out["ft"]).reshape(-1, 6)
        scale = np.abs(ft).max()
        d = np.abs(ft - res[k]["ft"]).max() / scale
        _say(f"  request {k}: served vs single-problem solve {d:.2e}")
        assert d < 1e-7


def test_serving_matches_oracle(dev, oracle_pairsum_built, mixed_run, stream):
    res, _ = mixed_run
    k = 2
    r = stream[k]
    g = geo.build(r["centers"], 1.0, geo.Params(**DISC))
    pbo = mfs.Problem(g).setup()
    ref = mfs.solve_resistance(pbo, r["rbm"], tol=1e-10)["ft"]
    d = np.abs(res[k]["ft"] - ref).max() / np.abs(ref).max()
    _say(f"  request {k} (P={r['P']}, min gap {r['gap_min']:.1e}): served vs oracle {d:.2e}")
    # device SVD vs LAPACK SVD of the self blocks: agreement at the level the
    # discrete problem is determined to (as for the device set-up test)
    assert d < 1e-5


def test_serving_admits_by_memory(dev, stream):
    """An arena that holds the largest request once: the resident requests
    never need more than the arena, and never more of them than the
    smallest ones could fit."""
    need = [dev.Problem(r["centers"], 1.0, **DISC, **SOLVER).sizes.workspace_bytes for r in stream[:6]]
    arena = max(need) + 4096
    fit = np.searchsorted(np.cumsum(sorted(-(-np.array(need) // 256) * 256)), arena, side="right")
    _say(f"serving: arena {arena / 2**20:.1f} MiB for 6 requests of {min(need) / 2**20:.1f}.."
         f"{max(need) / 2**20:.1f} MiB (at most {fit} fit together)")
    srv = dev.Server(arena_bytes=arena, max_active=8, **DISC, **SOLVER)
    ids = [srv.submit(r["centers"], r["rbm"]) for r in stream[:6]]
    srv.drain(timeout_s=120)
    st = srv.stats()
    res = [srv.poll(i, r["P"]) for i, r in zip(ids, stream[:6])]
    srv.close()
    assert all(x["status"] == 0 for x in res)
    assert st["arena_peak"] <= arena
    assert st["peak_active"] <= fit < 6


def test_serving_zero_motion_request(dev):
    srv = dev.Server(arena_bytes=1 << 30, max_active=2, **DISC, **SOLVER)
    c = np.array([[0.0, 0, 0], [2.5, 0, 0]])
    i = srv.submit(c, np.zeros((2, 6)))
    srv.drain(timeout_s=60)
    r = srv.poll(i, 2)
    srv.close()
    assert r["status"] == 0 and r["iterations"] == 0
    assert np.all(r["ft"] == 0.0)
