"""The device SVD of the self blocks (B = Q1 R1, R1^T = Q2 R2, one-sided
Jacobi on R2^T, U = Q1 U_X, V = Q2 J) against the oracle's LAPACK SVD, through
the C-ABI: ranks, singular values, the truncated pseudo-inverse applied to a
physical vector, and the solve it leads to (Section 2.2, eq. transform; the
truncation eps_trunc of Section 5)."""
import numpy as np
import pytest

from oracle import brenner, mfs
from paper_2407_03343_amd import workloads as wl

from gpu_common import _say, _t, _n, _finished

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pair_jacobi(dev, pair001):
    _say("device Jacobi SVD: two spheres at gap 0.01 (default discretisation)")
    lib = dev.Problem(pair001["pk"].centers, 1.0, svd_method=dev.SMFS_SVD_JACOBI).bind()
    import time
    t0 = time.perf_counter()
    lib.setup()
    torch.cuda.synchronize()
    _say(f"  set-up {time.perf_counter() - t0:.2f} s, {lib.sizes.svd_sweeps} Jacobi sweeps")
    assert 0 < lib.sizes.svd_sweeps < 40
    return lib


def test_jacobi_ranks_match_lapack(dev, pair_jacobi, pair001):
    pbo = pair001["pb"]
    for fid in range(pair_jacobi.sizes.n_factors):
        info = pair_jacobi.factor_info(fid)
        if info["sphere"] < 0:
            continue
        of = pbo.factors[int(pbo.factor_of[info["sphere"]])]
        _say(f"  factor {fid}: {info['rows']} x {info['cols']}, rank {info['rank']} (LAPACK {of.s.size})")
        assert abs(info["rank"] - of.s.size) <= max(2, of.s.size // 100)


def _perturbation_sensitivity(B, b, trunc):
    """Relative change of the truncated B^+ b when B is perturbed by a random
    matrix at the rounding level (eps max|B|): how far two backward-stable
    SVDs of the same block may put B^+ b apart."""
    def pinv(M):
        U, s, Vt = np.linalg.svd(M, full_matrices=False)
        r = int(np.sum(s > trunc * s[0]))
        return Vt[:r].T @ ((U[:, :r].T @ b) / s[:r])
    E = np.random.default_rng(7).standard_normal(B.shape) * (2.2e-16 * np.abs(B).max())
    x0, x1 = pinv(B), pinv(B + E)
    return np.linalg.norm(x1 - x0) / np.linalg.norm(x0)


@pytest.fixture(scope="module")
def block0(pair001):
    """Sphere 0's self block, a physical right-hand side on it, and the
    measured perturbation sensitivity of its truncated pseudo-inverse."""
    g, pbo = pair001["g"], pair001["pb"]
    B = mfs.self_block(g, 0)
    b = pair001["out"]["b"][pbo.tslice(0)]
    sens = _perturbation_sensitivity(B, b, g.params.trunc_rel)
    f = pbo.factors[int(pbo.factor_of[0])]
    lam_ref = f.V @ ((f.U.T @ b) / f.s)
    _say(f"  B^+ b of sphere 0: sensitivity to an eps-level perturbation of B {sens:.2e}")
    return B, b, lam_ref, sens


def _lambda0(lib, pair001):
    """lambda_hat of sphere 0 (local source order) from the library's B^+."""
    g = pair001["g"]
    lam = _n(lib.transform(_t(pair001["out"]["b"]))).reshape(-1, 3)
    return lam[g.local_sources[0]].reshape(-1)


def test_jacobi_pseudo_inverse_and_solve(dev, pair_jacobi, pair001, block0):
    """B^+ b of a physical right-hand side: within 10 x the perturbation
    sensitivity of the oracle's LAPACK result, and with the same projection
    residual |B B^+ b - b| / |b| to 1e-3 relative (well conditioned); then
    the solve: forces within 1e-5 of the oracle's and Brenner's force within
    1e-3."""
    B, b, lam_ref, sens = block0
    lam = _lambda0(pair_jacobi, pair001)
    d = np.linalg.norm(lam - lam_ref) / np.linalg.norm(lam_ref)
    r_ref = np.linalg.norm(B @ lam_ref - b) / np.linalg.norm(b)
    r = np.linalg.norm(B @ lam - b) / np.linalg.norm(b)
    _say(f"  B^+ b: Jacobi vs LAPACK {d:.3e} (sensitivity {sens:.2e}); residual {r:.6e} (LAPACK {r_ref:.6e})")
    assert d < 10 * sens
    assert abs(r - r_ref) < 1e-3 * r_ref
    out = pair_jacobi.solve_resistance(_t(pair001["rbm"][0]))
    ft = _n(out["ft"]).reshape(-1, 6)
    ref = pair001["out"]["ft"]
    dF = np.abs(ft - ref).max() / np.abs(ref).max()
    Fb = brenner.brenner_force(0.01, 0.5)
    _say(f"  solve: it {out['iterations']}, status {out['status']}, F/T vs oracle {dF:.2e}, "
         f"|F| {np.linalg.norm(ft[0, :3]):.6f} (Brenner {Fb:.6f})")
    assert _finished(out) and out["true_rel_residual"] < 1e-6
    assert dF < 1e-5
    assert abs(np.linalg.norm(ft[0, :3]) - Fb) < 1e-3 * Fb


def test_jacobi_matches_rocsolver_factors(dev, pair_jacobi, pair001, block0):
    """The two device SVDs of the same blocks: equal ranks (within 1%), and
    B^+ b within 10 x the perturbation sensitivity of each other."""
    B, b, lam_ref, sens = block0
    other = dev.Problem(pair001["pk"].centers, 1.0, svd_method=dev.SMFS_SVD_ROCSOLVER).bind().setup()
    for fid in range(pair_jacobi.sizes.n_factors):
        ia, ib = pair_jacobi.factor_info(fid), other.factor_info(fid)
        if ia["sphere"] < 0:
            continue
        assert abs(ia["rank"] - ib["rank"]) <= max(2, ib["rank"] // 100)
    la, lb = _lambda0(pair_jacobi, pair001), _lambda0(other, pair001)
    d = np.linalg.norm(la - lb) / np.linalg.norm(lb)
    dr = np.linalg.norm(lb - lam_ref) / np.linalg.norm(lam_ref)
    _say(f"  B^+ b: Jacobi vs rocSOLVER {d:.3e}, rocSOLVER vs LAPACK {dr:.3e} (sensitivity {sens:.2e})")
    assert d < 10 * sens


@pytest.mark.parametrize("disc", [dict(n_proxy=60, n_colloc_base=80, n_image=4),
                                  dict(n_proxy=120, n_colloc_base=160, n_image=6),
                                  dict(n_proxy=200, n_colloc_base=260, n_image=8)],
                         ids=["cols216", "cols414", "cols672"])
def test_jacobi_small_blocks(dev, oracle_pairsum_built, disc):
    """Blocks of at most 768 columns take the one-wave pair tasks (4, 8 and 12
    rows per lane for 216, 414 and 672 columns): two spheres at gap 0.01 at
    reduced discretisations, the device Jacobi SVD against the oracle's
    LAPACK factors: ranks, B^+ b of a physical right-hand side within 10 x
    its perturbation sensitivity, the same projection residual to 1e-3, and
    the solve's forces and torques within 1e-5 of the oracle's."""
    from oracle import geometry as geo
    pk, rbms = wl.workload_two_sphere_gap001()
    rbm = rbms[0]
    g = geo.build(pk.centers, 1.0, geo.Params(**disc))
    pbo = mfs.Problem(g).setup()
    ref = mfs.solve_resistance(pbo, rbm, tol=1e-10)
    lib = dev.Problem(pk.centers, 1.0, svd_method=dev.SMFS_SVD_JACOBI, **disc).bind().setup()
    B = mfs.self_block(g, 0)
    assert B.shape[1] <= 768
    for fid in range(lib.sizes.n_factors):
        info = lib.factor_info(fid)
        if info["sphere"] < 0:
            continue
        of = pbo.factors[int(pbo.factor_of[info["sphere"]])]
        assert abs(info["rank"] - of.s.size) <= max(2, of.s.size // 100)
    b = ref["b"][pbo.tslice(0)]
    sens = _perturbation_sensitivity(B, b, g.params.trunc_rel)
    f = pbo.factors[int(pbo.factor_of[0])]
    lam_ref = f.V @ ((f.U.T @ b) / f.s)
    lam = _n(lib.transform(_t(ref["b"]))).reshape(-1, 3)[g.local_sources[0]].reshape(-1)
    d = np.linalg.norm(lam - lam_ref) / np.linalg.norm(lam_ref)
    r_ref = np.linalg.norm(B @ lam_ref - b) / np.linalg.norm(b)
    r = np.linalg.norm(B @ lam - b) / np.linalg.norm(b)
    out = lib.solve_resistance(_t(rbm))
    ft = _n(out["ft"]).reshape(-1, 6)
    dF = np.abs(ft - ref["ft"]).max() / np.abs(ref["ft"]).max()
    _say(f"  {B.shape[0]} x {B.shape[1]}: {lib.sizes.svd_sweeps} sweeps; B^+ b vs LAPACK {d:.2e} "
         f"(sensitivity {sens:.2e}); residual {r:.6e} (LAPACK {r_ref:.6e}); solve it {out['iterations']}, "
         f"F/T vs oracle {dF:.2e}")
    assert 0 < lib.sizes.svd_sweeps < 40
    assert d < 10 * sens
    assert abs(r - r_ref) < 1e-3 * r_ref
    assert _finished(out) and dF < 1e-5
