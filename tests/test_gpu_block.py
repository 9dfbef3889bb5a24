"""Many right-hand sides: the block product and the lock-step block GMRES
(through the C-ABI) against the FP64 oracle and against the single-vector
calls of the same library.

Each column of a block product is the single product of that column: the
pairs are the same, the geometry is computed once per run of four columns
and the per-sphere pseudo-inverse runs as a GEMM on the matrix cores, so
only the summation order differs.  Bars as for the single product: 1e-10
relative on smooth inputs, 20 times the oracle's own rounding sensitivity
on rough ones.
"""
import numpy as np
import pytest

from oracle import geometry as geo, mfs
from paper_2407_03343_amd import workloads as wl

from gpu_common import NOGUARD, _say, _t, _n, _rel, _import_oracle_factors, _transform_ext

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SMALL = dict(n_proxy=120, n_colloc_base=160, n_image=6, n_check_base=80)


@pytest.fixture(scope="module")
def small12(dev, oracle_pairsum_built):
    """Twelve spheres with two near-contact pairs (gaps 2e-3 and 0.05),
    small discretisation, oracle factors imported."""
    rng = np.random.default_rng(41)
    c = [np.array([0.0, 0.0, 0.0]), np.array([2.002, 0.0, 0.0]),
         np.array([0.0, 4.0, 0.0]), np.array([0.0, 6.05, 0.0])]
    while len(c) < 12:
        x = rng.uniform(-6, 8, 3)
        if all(np.linalg.norm(x - y) > 2.4 for y in c):
            c.append(x)
    c = np.array(c)
    g = geo.build(c, 1.0, geo.Params(**SMALL))
    pbo = mfs.Problem(g).setup()
    lib = dev.Problem(c, 1.0, gmres_tol=1e-11, **SMALL, **NOGUARD).bind()
    _import_oracle_factors(lib, pbo)
    return dict(c=c, g=g, pb=pbo, lib=lib)


@pytest.mark.parametrize("nrhs", [1, 5, 37])
def test_block_apply_vs_oracle_and_single(small12, nrhs):
    _say(f"block product, 12 spheres, nrhs={nrhs}")
    g, pbo, lib = small12["g"], small12["pb"], small12["lib"]
    n = 3 * g.T
    M = np.empty((nrhs, n))
    rbm = wl.random_rbm(g.P, nrhs, 42)
    for q in range(nrhs):     # even columns smooth (boundary data), odd rough
        M[q] = pbo.rhs(rbm[q]) if q % 2 == 0 else wl.random_vector(n, 100 + q)
    Y = _n(lib.apply_block(_t(M).view(nrhs, n))).reshape(nrhs, n)
    ts = g.target_sphere
    for q in range(nrhs):
        ref = pbo.apply(M[q])
        # per sphere, even the smooth columns pass through the pseudo-inverse
        # of the gap-2e-3 pair: the bar is the oracle's own rounding
        # sensitivity (its transform in extended precision), at least 1e-10
        bar = max(1e-10, 20 * _rel(pbo.apply(M[q], _transform_ext(pbo, M[q])), ref, ts))
        assert _rel(Y[q], ref, ts) < bar, (q, _rel(Y[q], ref, ts), bar)
        ys = _n(lib.apply(_t(M[q])))
        assert _rel(Y[q], ys, ts) < bar, (q, _rel(Y[q], ys, ts))


def test_block_apply_full_size_cluster(dev, oracle_pairsum_built):
    """100-sphere cluster at full size, 64 columns (the size the block
    benchmark uses), seeded rank-48 factors; every column against the single
    product, eight columns against the oracle on sampled rows."""
    _say("cluster of 100: block product of 64 columns")
    pk, _ = wl.workload_cluster100(0)
    g = geo.build(pk.centers, 1.0)
    lib = dev.Problem(pk.centers, 1.0).bind()
    pbo = mfs.Problem(g)
    for fid in range(lib.sizes.n_factors):
        info = lib.factor_info(fid)
        if info["sphere"] < 0:
            continue
        U, s, V = wl.random_factors(info["rows"], info["cols"], 48, seed=100 + fid)
        lib.import_factor(fid, U, s, V)
        pbo.factors[int(pbo.factor_of[info["sphere"]])] = mfs.Factor(U, s, V, float(s[0]), info["cols"])
    nrhs, n = 64, 3 * g.T
    M = torch.empty(nrhs, n, dtype=torch.float64, device="cuda")
    Mh = np.stack([wl.random_vector(n, 500 + q) for q in range(nrhs)])
    M.copy_(torch.from_numpy(Mh))
    Y = lib.apply_block(M)
    worst = 0.0
    for q in range(nrhs):
        ys = lib.apply(M[q].contiguous())
        worst = max(worst, float(torch.linalg.norm(Y[q] - ys) / torch.linalg.norm(ys)))
    _say(f"  block vs single worst column {worst:.3e}")
    assert worst < 1e-12
    Yh = _n(Y).reshape(nrhs, -1, 3)
    rows = np.random.default_rng(22).choice(g.T, 300, replace=False)
    for q in (0, 1, 31, 32, 60, 61, 62, 63):
        lam_hat = pbo.transform(Mh[q])
        ref = Mh[q].reshape(-1, 3)[rows] + pbo.apply_rows(lam_hat, rows, is_lambda=True)
        assert _rel(Yh[q][rows], ref, g.target_sphere[rows]) < 1e-10, q


def test_block_solve_matches_oracle_and_single(dev, small12):
    restart = 200
    _say(f"block resistance solve, 12 spheres, 6 systems, restart {restart}")
    g, pbo, lib = small12["g"], small12["pb"], small12["lib"]
    nrhs = 6
    rbm = wl.random_rbm(g.P, nrhs, 43)
    rbm[3] = 0.0                     # a zero right-hand side stays zero
    out = lib.solve_resistance_block(_t(rbm), restart=restart)
    assert out["status"] in (0, 3) and out["n_converged"] == nrhs
    ft = _n(out["ft"]).reshape(nrhs, g.P, 6)
    assert np.all(ft[3] == 0.0) and out["iterations"][3] == 0
    for q in (0, 1, 5):
        ref = mfs.solve_resistance(pbo, rbm[q], tol=1e-11)["ft"]
        # the oracle's own rounding sensitivity: the same solve with its
        # pseudo-inverse apply in extended precision
        b = pbo.rhs(rbm[q])
        res = mfs.gmres(lambda v: pbo.apply(v, _transform_ext(pbo, v)), b, 1e-11, 500)
        ref_ext = pbo.force_torque(_transform_ext(pbo, res.x))
        scale = np.abs(ref).max()
        bar = max(1e-10, 20 * np.abs(ref_ext - ref).max() / scale)
        d_or = np.abs(ft[q] - ref).max() / scale
        single = lib.solve_resistance(_t(rbm[q]), want_check=False)
        fs = _n(single["ft"]).reshape(-1, 6)
        d_single = np.abs(ft[q] - fs).max() / scale
        _say(f"  system {q}: block-oracle {d_or:.2e}, block-single {d_single:.2e}, bar {bar:.2e}, "
             f"iterations {out['iterations'][q]} vs {single['iterations']}")
        assert d_or < bar and d_single < bar, q
        # the same Krylov process as the single solve, whose refinement sweeps
        # on the FP64 true residual (after its rounding floor) may add more
        if single["refinements"] == 0:
            assert abs(int(out["iterations"][q]) - single["iterations"]) <= 3
        else:
            assert int(out["iterations"][q]) <= single["iterations"] + 3
    # the true residual floors near 1e-7 here (rounding amplified by the
    # truncated pseudo-inverse of the gap-2e-3 pair), as for single solves
    assert np.all(out["true_rel_residual"] < 1e-6)


def test_block_solve_restarted(dev, oracle_pairsum_built):
    """GMRES(12) with restarts: the block solver and the single-vector
    solver with the same restart length take the same path."""
    _say("block resistance solve with restarts (GMRES(12)), three spheres, 9 systems")
    prm = dict(n_proxy=60, n_colloc_base=80, n_image=4, n_check_base=50)
    c = np.array([[0.0, 0, 0], [2.05, 0.3, 0.0], [0.4, 2.3, 0.1]])
    g = geo.build(c, 1.0, geo.Params(**prm))
    pbo = mfs.Problem(g).setup()
    lib = dev.Problem(c, 1.0, gmres_tol=1e-10, gmres_restart=12, gmres_max_it=3000, **prm,
                      **NOGUARD).bind()
    _import_oracle_factors(lib, pbo)
    nrhs = 9
    rbm = wl.random_rbm(3, nrhs, 44)
    out = lib.solve_resistance_block(_t(rbm), restart=12)
    assert out["status"] in (0, 3)
    ft = _n(out["ft"]).reshape(nrhs, 3, 6)
    for q in range(nrhs):
        single = lib.solve_resistance(_t(rbm[q]), want_check=False)
        fs = _n(single["ft"]).reshape(-1, 6)
        assert abs(int(out["iterations"][q]) - single["iterations"]) <= 2, q
        assert np.abs(ft[q] - fs).max() < 1e-9 * np.abs(fs).max(), q
    ref = mfs.solve_resistance(pbo, rbm[nrhs - 1], tol=1e-12)["ft"]
    assert np.abs(ft[nrhs - 1] - ref).max() < 1e-8 * np.abs(ref).max()
    assert out["max_iterations"] > 12          # restarts did happen


def test_block_apply_mixed(dev, small12):
    """Mixed block product (FP32 far field of the contact-free proxies for
    runs of four vectors): every column within 1e-5 per sphere of the FP64
    oracle on boundary-data vectors, and within FP32 rounding of the
    single-vector mixed product."""
    _say("mixed block product, 12 spheres, 9 columns")
    g, pbo, lib = small12["g"], small12["pb"], small12["lib"]
    assert lib.sizes.n_factors > 1 and any(g.contact_free(k) for k in range(g.P))
    n, nrhs = 3 * g.T, 9
    rbm = wl.random_rbm(g.P, nrhs, 46)
    M = np.stack([pbo.rhs(rbm[q]) for q in range(nrhs)])
    Y = _n(lib.apply_block(_t(M).view(nrhs, n), precision=dev.SMFS_MIXED_FAR)).reshape(nrhs, n)
    Y64 = _n(lib.apply_block(_t(M).view(nrhs, n))).reshape(nrhs, n)
    ts = g.target_sphere
    for q in range(nrhs):
        ref = pbo.apply(M[q])
        ys = _n(lib.apply(_t(M[q]), precision=dev.SMFS_MIXED_FAR))
        d, d64, ds = _rel(Y[q], ref, ts), _rel(Y64[q], ref, ts), _rel(Y[q], ys, ts)
        bar64 = max(1e-10, 20 * _rel(pbo.apply(M[q], _transform_ext(pbo, M[q])), ref, ts))
        assert d64 < bar64, (q, d64, bar64)
        assert d < 1e-5 and ds < 1e-5, (q, d, ds)
        assert not np.array_equal(Y[q], Y64[q])        # the FP32 path did run


def test_block_solve_mixed(dev, oracle_pairsum_built):
    """Mixed block solve of six systems (FP32 far field inside the cycles,
    FP64 true residuals at every restart and up to two refinements): forces
    and torques within 1e-5 of the oracle's FP64 solves."""
    _say("mixed block resistance solve, 12 spheres, 6 systems")
    rng = np.random.default_rng(47)
    c = [np.array([0.0, 0.0, 0.0]), np.array([2.01, 0.0, 0.0])]
    while len(c) < 12:
        x = rng.uniform(-6, 8, 3)
        if all(np.linalg.norm(x - y) > 2.4 for y in c):
            c.append(x)
    c = np.array(c)
    g = geo.build(c, 1.0, geo.Params(**SMALL))
    pbo = mfs.Problem(g).setup()
    lib = dev.Problem(c, 1.0, gmres_tol=1e-9, precision=dev.SMFS_MIXED_FAR, **SMALL).bind()
    _import_oracle_factors(lib, pbo)
    nrhs = 6
    rbm = wl.random_rbm(g.P, nrhs, 48)
    out = lib.solve_resistance_block(_t(rbm), restart=200)
    ft = _n(out["ft"]).reshape(nrhs, g.P, 6)
    _say(f"  status {out['status']}, refinements {out['refinements']}, max it {out['max_iterations']}, "
         f"true residuals {np.max(out['true_rel_residual']):.2e}, fp32 pairs {out['pair_evals_f32']:.3e}")
    assert out["status"] in (0, 3) and out["pair_evals_f32"] > 0
    # a mixed block solve reports a stalled FP64 residual only after both
    # refinement restarts (every system is checked on its FP64 residual)
    assert out["status"] == 0 or out["refinements"] == 2
    assert (out["status"] == 0) == bool(np.all(out["true_rel_residual"] <= 1e-9))
    for q in range(nrhs):
        ref = mfs.solve_resistance(pbo, rbm[q], tol=1e-10)["ft"]
        d = np.abs(ft[q] - ref).max() / np.abs(ref).max()
        assert d < 1e-5, (q, d)
