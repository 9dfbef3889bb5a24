"""Products at the full sizes of the packing workloads, checked on sampled
rows against the oracle (which evaluates those rows one by one).

In the random-vector checks the self-block factors are replaced by seeded
well-conditioned rank-48 factors, so that neither side needs the SVDs and
the check isolates the product: every sphere's pseudo-inverse apply and all
off-sphere pairs.  The real-rank check takes the oracle's LAPACK factors of
the shared contact-free block and of one contact block, and seeded factors
of the same rank for the other contact blocks, so that every loop over a
factor runs its real trip count.
"""
import numpy as np
import pytest

from oracle import geometry as geo, mfs
from paper_2407_03343_amd import workloads as wl

from gpu_common import _say, _rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _random_factors(lib, pbo, seed0):
    for fid in range(lib.sizes.n_factors):
        info = lib.factor_info(fid)
        if info["sphere"] < 0:
            continue
        U, s, V = wl.random_factors(info["rows"], info["cols"], 48, seed=seed0 + fid)
        lib.import_factor(fid, U, s, V)
        pbo.factors[int(pbo.factor_of[info["sphere"]])] = mfs.Factor(U, s, V, float(s[0]), info["cols"])


def _rows(g, n, seed):
    rng = np.random.default_rng(seed)
    rows = set(rng.choice(g.T, n, replace=False).tolist())
    for k in rng.choice(g.P, 20, replace=False):      # first and last node of some spheres
        rows.add(int(g.target_offsets[k]))
        rows.add(int(g.target_offsets[k + 1] - 1))
    return np.array(sorted(rows))


def test_packing2000_products_sampled(dev, oracle_pairsum_built):
    """2000 spheres at volume fraction 0.3, 5% in near-contact pairs: FP64
    product to 1e-10 and the mixed products to 2e-4 per sphere on sampled
    rows (a random vector: the FP32 far field of 1.2 million sources with
    cancellation, measured 7.3e-5 per sphere, 3e-6 over the whole vector;
    the equivalent-source far field is held to the same bar)."""
    _say("2000-sphere packing: full-size products (FP64, mixed, mixed far), sampled rows")
    pk = wl.workload_packing2000(2000, seed=0)
    g = geo.build(pk.centers, 1.0)
    lib = dev.Problem(pk.centers, 1.0, gmres_restart=4).bind()
    assert (lib.T, lib.S) == (g.T, g.S)
    pbo = mfs.Problem(g)
    _random_factors(lib, pbo, 300)
    lib.setup_far_field()
    mu = wl.random_vector(3 * g.T, 51)
    mu_d = torch.from_numpy(mu).cuda()
    rows = _rows(g, 400, 52)
    ref = mu.reshape(-1, 3)[rows] + pbo.apply_rows(pbo.transform(mu), rows, is_lambda=True)
    for name, prec, bar in (("fp64", dev.SMFS_FP64, 1e-10), ("mixed", dev.SMFS_MIXED, 2e-4),
                            ("mixed_far", dev.SMFS_MIXED_FAR, 2e-4), ("mixed_eq", dev.SMFS_MIXED_EQ, 2e-4)):
        y = lib.apply(mu_d, precision=prec).cpu().numpy().reshape(-1, 3)
        d = _rel(y[rows], ref, g.target_sphere[rows])
        _say(f"  {name}: per-sphere rel diff {d:.3e}, whole-vector {_rel(y[rows], ref):.3e} on {rows.size} rows")
        assert d < bar, name


def test_block500_block_product_sampled(dev, oracle_pairsum_built):
    """500 spheres at volume fraction 0.35, 40% in near-contact pairs, 1000
    proxies and 1680 base nodes per sphere: block product of 12 vectors
    (three runs of four), sampled rows of three columns against the oracle
    and every column against the single-vector product."""
    _say("500-sphere block workload at N=1000, M_base=1680: block product, sampled rows")
    pk, _ = wl.workload_block500(500, seed=0)
    prm = dict(n_proxy=1000, n_colloc_base=1680)
    g = geo.build(pk.centers, 1.0, geo.Params(**prm))
    lib = dev.Problem(pk.centers, 1.0, gmres_restart=4, **prm).bind()
    assert (lib.T, lib.S) == (g.T, g.S)
    pbo = mfs.Problem(g)
    _random_factors(lib, pbo, 700)
    nrhs, n = 12, 3 * g.T
    M = np.stack([wl.random_vector(n, 600 + q) for q in range(nrhs)])
    Md = torch.from_numpy(M).cuda()
    Y = lib.apply_block(Md)
    worst = 0.0
    for q in range(nrhs):
        ys = lib.apply(Md[q].contiguous())
        worst = max(worst, float(torch.linalg.norm(Y[q] - ys) / torch.linalg.norm(ys)))
    _say(f"  block vs single worst column {worst:.3e}")
    assert worst < 1e-12
    Yh = Y.cpu().numpy().reshape(nrhs, -1, 3)
    rows = _rows(g, 200, 53)
    for q in (0, 5, 11):
        ref = M[q].reshape(-1, 3)[rows] + pbo.apply_rows(pbo.transform(M[q]), rows, is_lambda=True)
        assert _rel(Yh[q][rows], ref, g.target_sphere[rows]) < 1e-10, q


def test_packing2000_real_ranks_physical(dev, oracle_pairsum_built):
    """2000-sphere packing with factors of the real truncated ranks: the
    oracle's LAPACK SVD of the shared contact-free block (full rank 1800)
    and of one contact block, seeded factors of that contact rank for the
    others.  A physical right-hand side (whose rounding sensitivity is at
    the 1e-14 level): FP64 product to 1e-10 per sphere on sampled rows, the
    mixed products to 1e-3 per sphere (the surface-velocity bar of the mixed
    form: the FP32 far field from the rough strengths of the full-rank
    shared factor, measured 1.5e-4), the equivalent-source form to 1e-4."""
    _say("2000-sphere packing: products with factors of the real truncated ranks")
    pk = wl.workload_packing2000(2000, seed=0)
    g = geo.build(pk.centers, 1.0)
    lib = dev.Problem(pk.centers, 1.0, gmres_restart=4).bind()
    pbo = mfs.Problem(g)
    contact_rank = None
    for fid in range(lib.sizes.n_factors):
        info = lib.factor_info(fid)
        k = info["sphere"]
        if k < 0:
            continue
        if fid == 0 or contact_rank is None:
            f = mfs.truncated_svd(mfs.self_block(g, k), g.params.trunc_rel)
            if fid != 0:
                contact_rank = f.s.size
            _say(f"  LAPACK factor {fid}: {info['rows']} x {info['cols']}, rank {f.s.size}")
            U, s, V = f.U, f.s, f.V
        else:
            U, s, V = wl.random_factors(info["rows"], info["cols"], contact_rank, seed=900 + fid)
        lib.import_factor(fid, U, s, V)
        assert lib.factor_info(fid)["rank"] == s.size
        pbo.factors[int(pbo.factor_of[k])] = mfs.Factor(U, s, V, float(s[0]), info["cols"])
    assert contact_rank is not None and contact_rank > 1800
    lib.setup_far_field()
    rbm = wl.random_rbm(g.P, 1, 55)[0]
    b = pbo.rhs(rbm)
    b_d = torch.from_numpy(b).cuda()
    rows = _rows(g, 400, 56)
    ref = b.reshape(-1, 3)[rows] + pbo.apply_rows(pbo.transform(b), rows, is_lambda=True)
    for name, prec, bar in (("fp64", dev.SMFS_FP64, 1e-10), ("mixed", dev.SMFS_MIXED, 1e-3),
                            ("mixed_far", dev.SMFS_MIXED_FAR, 1e-3), ("mixed_eq", dev.SMFS_MIXED_EQ, 1e-4)):
        y = lib.apply(b_d, precision=prec).cpu().numpy().reshape(-1, 3)
        d = _rel(y[rows], ref, g.target_sphere[rows])
        _say(f"  {name}: per-sphere rel diff {d:.3e} on {rows.size} rows")
        assert d < bar, name
