"""Pins of the FP64 oracle against facts fixed by the paper and by the
mathematics (closed forms, exact identities, asymptotic limits, brute force).
CPU only."""
import json
import math
import os

import numpy as np
import pytest

from oracle import geometry as geo, kernels, mfs, brenner
from oracle.pairsum import pairsum

from closed_forms import jeffery_axial_torque, stimson_jeffery

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")


def _sphere_points(n, rng):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# -- kernels: exact single-sphere identities ------------------------------

@pytest.mark.parametrize("a,mu", [(1.0, 1.0), (1.3, 0.7)])
def test_translating_sphere_identity(a, mu):
    """Stokeslet 6 pi mu a U plus potential dipole -pi a^3 U at the centre
    give exactly u = U on |x - c| = a (rigid translation)."""
    rng = np.random.default_rng(0)
    c = np.array([0.3, -0.2, 0.5])
    U = np.array([0.4, -1.1, 0.7])
    x = c + a * _sphere_points(200, rng)
    r = x - c
    u = kernels.stokeslet(r, mu) @ (6 * math.pi * mu * a * U) + kernels.dipole(r) @ (-math.pi * a ** 3 * U)
    assert np.abs(u - U).max() < 1e-13


@pytest.mark.parametrize("a,mu", [(1.0, 1.0), (0.8, 2.5)])
def test_rotating_sphere_identity(a, mu):
    """Rotlet 8 pi mu a^3 omega at the centre gives omega x (x - c) on the sphere."""
    rng = np.random.default_rng(1)
    c = np.array([1.0, 2.0, -1.0])
    w = np.array([0.2, 0.9, -0.5])
    x = c + a * _sphere_points(200, rng)
    u = kernels.rotlet(x - c, mu) @ (8 * math.pi * mu * a ** 3 * w)
    assert np.abs(u - np.cross(w, x - c)).max() < 1e-13


def test_kernel_symmetries():
    rng = np.random.default_rng(2)
    r = rng.standard_normal((50, 3))
    S, R, D = kernels.stokeslet(r, 1.0), kernels.rotlet(r, 1.0), kernels.dipole(r)
    assert np.abs(S - np.swapaxes(S, 1, 2)).max() < 1e-15
    assert np.abs(D - np.swapaxes(D, 1, 2)).max() < 1e-15
    assert np.abs(R + np.swapaxes(R, 1, 2)).max() < 1e-15
    # rotlet is the cross product t x r / (8 pi |r|^3)
    t = rng.standard_normal(3)
    rn = np.linalg.norm(r, axis=1)[:, None]
    assert np.allclose(R @ t, np.cross(t, r) / (8 * math.pi * rn ** 3), rtol=0, atol=1e-14)


@pytest.mark.parametrize("kind", [geo.KIND_S, geo.KIND_R, geo.KIND_D])
def test_kernel_divergence_free(kind):
    rng = np.random.default_rng(3)
    h = 1e-4
    for _ in range(10):
        x = rng.standard_normal(3) * 2
        lam = rng.standard_normal(3)
        div = 0.0
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            up = kernels.tensor(kind, (x + e)[None], 1.0)[0] @ lam
            um = kernels.tensor(kind, (x - e)[None], 1.0)[0] @ lam
            div += (up[c] - um[c]) / (2 * h)
        scale = np.abs(kernels.tensor(kind, x[None], 1.0)[0] @ lam).max() / np.linalg.norm(x)
        assert abs(div) < 1e-6 * scale


def test_kernel_far_field_decay():
    """Stokeslet decays like 1/r, rotlet and dipole like 1/r^2."""
    e = np.array([0.3, 0.4, 0.866])
    for kind, p in ((geo.KIND_S, 1), (geo.KIND_R, 2), (geo.KIND_D, 3)):
        a = np.abs(kernels.tensor(kind, (10 * e)[None], 1.0)).max()
        b = np.abs(kernels.tensor(kind, (20 * e)[None], 1.0)).max()
        assert abs(a / b - 2 ** p) < 1e-12 * 2 ** p


def test_c_pairsum_matches_dense_blocks(oracle_pairsum_built):
    rng = np.random.default_rng(4)
    nt, ns = 37, 53
    x = rng.standard_normal((nt, 3)) * 3
    y = rng.standard_normal((ns, 3)) * 0.5
    kinds = rng.integers(0, 3, ns).astype(np.int32)
    lam = rng.standard_normal((ns, 3))
    G = kernels.dense_block(x, y, kinds, 0.9)
    u = pairsum(x, y, kinds, lam, 0.9)
    ref = (G @ lam.reshape(-1)).reshape(-1, 3)
    assert np.abs(u - ref).max() < 1e-13 * np.abs(ref).max()
    # skip pairs in the same "sphere"
    tsph = rng.integers(0, 4, nt).astype(np.int32)
    ssph = rng.integers(0, 4, ns).astype(np.int32)
    u2 = pairsum(x, y, kinds, lam, 0.9, tsph, ssph, skip_same=True)
    mask = (tsph[:, None] != ssph[None, :]).astype(float)
    Gm = G.reshape(nt, 3, ns, 3) * mask[:, None, :, None]
    ref2 = (Gm.reshape(3 * nt, 3 * ns) @ lam.reshape(-1)).reshape(-1, 3)
    assert np.abs(u2 - ref2).max() < 1e-13 * np.abs(ref2).max()


# -- geometry ------------------------------------------------------------

@pytest.mark.parametrize("delta", [0.1, 0.5, 1.0])
def test_accumulation_point_is_limit_of_reflections(delta):
    """Reflecting each centre in the other sphere over and over converges
    to eq. (acc_points); its distance to the centre is eq. (Racc)."""
    c1 = np.array([0.0, 0.0, 0.0])
    c2 = np.array([2.0 + delta, 0.0, 0.0])
    x = c2.copy()                  # image of c2 in sphere 1, then alternate
    img1 = None
    for _ in range(20000):
        img1 = geo.kelvin_reflect(x, c1)
        x = geo.kelvin_reflect(img1, c2)
    a1, a2 = geo.accumulation_points(c1, c2)
    assert np.abs(img1 - a1).max() < 1e-12
    assert np.abs(x - a2).max() < 1e-12
    assert abs(np.linalg.norm(a1 - c1) - geo.r_acc(delta)) < 1e-14


@pytest.mark.parametrize("Rp", [0.5, 0.63, 0.7, 0.9])
def test_delta_star_solves_racc(Rp):
    assert abs(geo.r_acc(geo.delta_star(Rp)) - Rp) < 1e-14


def test_paper_printed_values():
    """Values printed in the paper (tests/golden/paper_values.json)."""
    gv = json.load(open(GOLDEN))
    # delta* ~ 0.129 for R_p = 0.7 (Section 3, after Figure Rg_sweep)
    assert abs(geo.delta_star(0.7) - gv["delta_star_Rp_0p7"]["value"]) < 5e-4
    # 3 M = 3 (801 + 12 n_c 3 20) with n_c = 3 printed as 3*2960 (Section 5.3)
    m = geo.m_estimate(801, [20, 20, 20])
    assert abs(m - gv["m_tetrahedron"]["value"]) <= 1
    # 4.81e6 degrees of freedom for 2000 spheres of 801 nodes (Section 4, Ex. 2)
    assert abs(3 * 801 * 2000 - gv["dof_2000"]["value"]) / gv["dof_2000"]["value"] < 2e-3
    # image count rule, eq. (image_est): 20 images suffice for delta > 1e-3
    assert geo.n_image_rule(1.01e-3) <= 20
    assert geo.n_image_rule(0.2) == 0


def test_image_nodes():
    delta, Rp, n, D = 0.01, 0.7, 20, 0.05
    t = geo.image_t(delta, Rp, n, D)
    assert abs(t[0] - geo.r_acc(delta)) < 1e-15          # first node at x_acc
    assert np.all(np.diff(t) < 0)                          # clustered toward x_acc
    assert abs(t[-1] - (Rp * (1 + D) + (geo.r_acc(delta) - Rp * (1 + D)) * math.sin(math.pi / (2 * n)))) < 1e-15
    assert abs(geo.r_acc(0.01) - 0.904875) < 1e-6


def test_geometry_counts_and_caps():
    c = np.array([[0.0, 0, 0], [2.01, 0, 0], [20.0, 0, 0]])
    g = geo.build(c, 1.0)
    assert g.M(0) == 1500 and g.Nk(0) == 660          # one-contact sphere
    assert g.M(2) == 780 and g.Nk(2) == 600           # contact-free sphere
    assert g.M(0) == geo.m_estimate(780, [20])
    # caps: points on the unit sphere, within their half-angle of the axis
    k = 0
    t0 = g.target_offsets[k]
    X = g.targets[t0:t0 + g.M(k)] - c[k]
    assert np.abs(np.linalg.norm(X, axis=1) - 1).max() < 1e-14
    e = np.array([1.0, 0, 0])
    cap1 = X[780:780 + 360]
    cap2 = X[780 + 360:]
    ang1 = np.arccos(np.clip(cap1 @ e, -1, 1))
    ang2 = np.arccos(np.clip(cap2 @ e, -1, 1))
    assert ang1.max() <= math.pi / 5 + 1e-12 and ang1.max() > 0.98 * math.pi / 5
    assert ang2.max() <= math.pi / 60 + 1e-12 and ang2.max() > 0.98 * math.pi / 60
    # weights sum to the sphere area for the base set and to the cap areas
    w = g.target_weight[t0:t0 + g.M(k)]
    assert abs(w[:780].sum() - 4 * math.pi) < 1e-12
    assert abs(w[780:1140].sum() - 2 * math.pi * (1 - math.cos(math.pi / 5))) < 1e-12
    # proxy and image sources inside the sphere, images on the line of centres
    src = g.src_pos[g.local_sources[0]] - c[0]
    assert np.linalg.norm(src, axis=1).max() < 1.0
    img = src[600:620]
    assert np.abs(img[:, 1:]).max() < 1e-15 and np.all(img[:, 0] > 0.7)
    # kinds: 620 S, 20 R, 20 D in local order
    kinds = g.src_kind[g.local_sources[0]]
    assert (kinds[:620] == 0).all() and (kinds[620:640] == 1).all() and (kinds[640:] == 2).all()


# -- Brenner series ---------------------------------------------------------

def test_brenner_far_field_limit():
    """Approaching spheres far apart: F / (6 pi v) = 1 + 3/(2d) + O(d^-2)."""
    res = []
    for delta in (50.0, 100.0, 200.0):
        d = 2 + delta
        res.append(brenner.brenner_force(delta) / (6 * math.pi) - 1 - 1.5 / d)
    # the remainder is second order: halving 1/d quarters it
    assert 3.0 < res[0] / res[1] < 5.0 and 3.0 < res[1] / res[2] < 5.0


def test_brenner_lubrication_limit():
    """F / (6 pi v) = 1/(2 delta) + (9/20) log(1/delta) + O(1)."""
    c = [brenner.brenner_force(d) / (6 * math.pi) - 0.5 / d - 0.45 * math.log(1 / d)
         for d in (1e-3, 1e-4, 1e-5)]
    assert abs(c[1] - c[2]) < 0.02 and abs(c[0] - c[1]) < 0.1
    assert abs(c[2]) < 5.0


# -- solve-level pins ---------------------------------------------------------

@pytest.fixture(scope="module")
def single_sphere(oracle_pairsum_built):
    g = geo.build(np.array([[0.5, -0.25, 2.0]]), 1.0)
    pb = mfs.Problem(g).setup()
    return g, pb


def test_single_sphere_translation_and_rotation(single_sphere):
    g, pb = single_sphere
    rbm = np.array([[0.3, -0.8, 0.5, 0.0, 0.0, 0.0]])
    out = mfs.solve_resistance(pb, rbm, tol=1e-12)
    assert out["iterations"] <= 1                     # G_hat = I for one sphere
    assert np.allclose(out["mu"], out["b"], rtol=0, atol=1e-14)
    F = out["ft"][0, :3]
    assert np.abs(F - mfs.stokes_drag(1.0, 1.0, rbm[0, :3])).max() < 1e-6 * np.linalg.norm(F)
    assert np.abs(out["ft"][0, 3:]).max() < 1e-6 * np.linalg.norm(F)
    rbm = np.array([[0.0, 0.0, 0.0, 0.2, 0.9, -0.4]])
    out = mfs.solve_resistance(pb, rbm, tol=1e-12)
    T = out["ft"][0, 3:]
    assert np.abs(T - mfs.stokes_torque(1.0, 1.0, rbm[0, 3:])).max() < 1e-6 * np.linalg.norm(T)
    assert np.abs(out["ft"][0, :3]).max() < 1e-6 * np.linalg.norm(T)


def test_pseudo_inverse_properties(single_sphere):
    g, pb = single_sphere
    f = pb.factors[0]
    B = mfs.self_block(g, 0)
    assert np.abs(f.U.T @ f.U - np.eye(f.s.size)).max() < 1e-12
    assert np.abs(f.V.T @ f.V - np.eye(f.s.size)).max() < 1e-12
    Bp_B = f.V @ ((f.U.T @ B) / f.s[:, None])
    assert np.abs(B @ Bp_B - B).max() < 1e-9 * f.sigma_max


def test_two_spheres_against_brenner(pair001):
    """Gap 0.01, separating at unit relative speed: each force equals
    Brenner's |F| with |v| = 1/2 (target accuracy 1e-3 of the paper)."""
    out = pair001["out"]
    Fb = brenner.brenner_force(0.01, 0.5)
    F1, F2 = out["ft"][0, :3], out["ft"][1, :3]
    assert abs(np.linalg.norm(F1) - Fb) < 1e-3 * Fb
    assert abs(np.linalg.norm(F2) - Fb) < 1e-3 * Fb
    # force on the fluid points along each sphere's own velocity
    assert F1[0] < 0 < F2[0]
    assert np.abs(F1 + F2).max() < 1e-4 * Fb
    eps, _ = pair001["pb"].residuals(out["lam"], pair001["rbm"][0], pair001["g"].check,
                                     pair001["g"].check_sphere)
    assert eps < 1e-3


def test_stimson_jeffery_far_field_expansion():
    """The Stimson-Jeffery series against the method of reflections for spheres far
    apart: 1 - 3/(2d) + 9/(4d^2) - 19/(8d^3) + O(d^-4), d the centre distance."""
    for d in (20.0, 40.0, 80.0):
        r = stimson_jeffery(d / 2) - (1 - 1.5 / d + 2.25 / d ** 2 - 2.375 / d ** 3)
        assert abs(r) * d ** 4 < 10.0, (d, r)


def test_two_spheres_translating_together(pair001):
    """Gap 0.01, both spheres moving with unit velocity along the line of
    centres: each force equals 6 pi mu a U times the Stimson-Jeffery factor
    (0.6457 here).  With the separating motion pinned against Brenner's
    series, this fixes both two-body resistance functions along the line
    of centres, so a sign error in the coupling between the spheres fails
    one of the two."""
    pb = pair001["pb"]
    rbm = np.zeros((2, 6))
    rbm[:, 0] = 1.0
    out = mfs.solve_resistance(pb, rbm, tol=1e-10)
    c = pair001["g"].centers
    h = 0.5 * np.linalg.norm(c[1] - c[0])
    Fsj = 6 * math.pi * stimson_jeffery(h)
    for F in out["ft"][:, :3]:
        assert abs(F[0] - Fsj) < 1e-4 * Fsj            # measured 7.8e-6
        assert np.abs(F[1:]).max() < 1e-5 * Fsj
    assert np.abs(out["ft"][:, 3:]).max() < 1e-5 * Fsj


def test_jeffery_series_limits():
    """At contact the factors tend to zeta(3) (opposite senses) and
    (3/4) zeta(3) (same sense); far apart to 1 -/+ (a/d)^3, the vorticity
    of the other sphere's rotlet at distance d."""
    z3 = 1.2020569031595942
    assert abs(jeffery_axial_torque(1 + 1e-8, False) - z3) < 1e-6
    assert abs(jeffery_axial_torque(1 + 1e-8, True) - 0.75 * z3) < 1e-6
    for d in (10.0, 20.0):
        assert abs(jeffery_axial_torque(d / 2, True) - (1 - d ** -3)) < 2 * d ** -6
        assert abs(jeffery_axial_torque(d / 2, False) - (1 + d ** -3)) < 2 * d ** -6


@pytest.mark.parametrize("d", [4.0, 8.0])
def test_separated_pair_against_series(oracle_pairsum_built, d):
    """Two contact-free spheres d radii apart (proxies only, one shared
    factor): translating together along the line of centres and spinning
    about it in the same sense, the forces and torques equal the
    Stimson-Jeffery and Jeffery series to 1e-7 (measured 5.6e-9 and 3.9e-9
    at d = 4, 5.1e-9 and 3.9e-9 at d = 8)."""
    c = np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]])
    pb = mfs.Problem(geo.build(c, 1.0)).setup()
    for off, ref in ((0, 6 * math.pi * stimson_jeffery(d / 2)), (3, 8 * math.pi * jeffery_axial_torque(d / 2, True))):
        rbm = np.zeros((2, 6))
        rbm[:, off] = 1.0
        ft = mfs.solve_resistance(pb, rbm, tol=1e-12)["ft"]
        assert np.abs(ft[:, off] - ref).max() < 1e-7 * ref
        other = np.delete(ft, off, axis=1)
        assert np.abs(other).max() < 1e-7 * ref


@pytest.mark.parametrize("same_sense", [True, False])
def test_two_spheres_spinning_about_line_of_centres(pair001, same_sense):
    """Gap 0.01, unit angular velocities about the line of centres, in the
    same or opposite senses: each torque equals 8 pi mu a^3 Omega times
    Jeffery's series (22.684 and 29.932 here; measured agreement 1e-9), the
    forces and the other torque components vanish.  This pins the rotlet
    and doublet images and the torque reduction."""
    pb = pair001["pb"]
    rbm = np.zeros((2, 6))
    rbm[0, 3], rbm[1, 3] = 1.0, (1.0 if same_sense else -1.0)
    out = mfs.solve_resistance(pb, rbm, tol=1e-10)
    c = pair001["g"].centers
    Tj = 8 * math.pi * jeffery_axial_torque(0.5 * np.linalg.norm(c[1] - c[0]), same_sense)
    ft = out["ft"]
    assert abs(ft[0, 3] - Tj) < 1e-6 * Tj
    assert abs(ft[1, 3] - rbm[1, 3] * Tj) < 1e-6 * Tj
    assert np.abs(ft[:, 4:]).max() < 1e-6 * Tj
    assert np.abs(ft[:, :3]).max() < 1e-6 * Tj


@pytest.mark.parametrize("case", ["forces", "torques_same", "torques_opposite"])
def test_mobility_pair_closed_forms(pair001, case):
    """Mobility problem for the pair at gap 0.01: equal unit forces along the
    line of centres move both spheres with U = F / (6 pi mu a lambda_SJ);
    unit torques about it, in the same or opposite senses, spin them with
    Omega = T / (8 pi mu a^3 tau_J).  Every other component vanishes.
    Measured agreement 1e-7 (forces) and 1e-9 (torques)."""
    c = pair001["g"].centers
    ax = (c[1] - c[0]) / np.linalg.norm(c[1] - c[0])
    h = 0.5 * np.linalg.norm(c[1] - c[0])
    ft = np.zeros((2, 6))
    if case == "forces":
        ft[:, :3] = ax
        off, want, bar = 0, 1 / (6 * math.pi * stimson_jeffery(h)), 1e-5
    else:
        same = case == "torques_same"
        ft[0, 3:], ft[1, 3:] = ax, (ax if same else -ax)
        off, want, bar = 3, 1 / (8 * math.pi * jeffery_axial_torque(h, same)), 1e-6
    out = mfs.solve_mobility(pair001["pb"], ft, tol=1e-10)
    rbm = out["rbm"]
    for q in range(2):
        sgn = ft[q, off:off + 3] @ ax
        assert abs(rbm[q, off:off + 3] @ ax - sgn * want) < bar * want
        expect = np.zeros(6)
        expect[off:off + 3] = sgn * want * ax
        assert np.abs(rbm[q] - expect).max() < 10 * bar * want


@pytest.mark.parametrize("flow", ["stream", "rotation"])
def test_pair_at_rest_in_background_flow(pair001, flow):
    """The pair at gap 0.01 held at rest (eq. bc with v = omega = 0) in a
    uniform stream along its line of centres, or in a rigid rotation about
    that line: the disturbance is that of the pair moving with -U, or
    spinning with -Omega in the same sense, in fluid at rest, so the forces
    are -6 pi mu a U lambda_SJ and the torques -8 pi mu a^3 Omega tau_J
    (measured agreement 7.8e-6 and 1e-9)."""
    c = pair001["g"].centers
    ax = (c[1] - c[0]) / np.linalg.norm(c[1] - c[0])
    h = 0.5 * np.linalg.norm(c[1] - c[0])
    if flow == "stream":
        u_inf, off, ref, bar = mfs.linear_flow(U=ax), 0, -6 * math.pi * stimson_jeffery(h), 1e-4
    else:
        assert np.abs(np.cross(c[0], ax)).max() < 1e-14        # the axis passes through the centres
        W = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
        u_inf, off, ref, bar = (mfs.linear_flow(L=W), 3, -8 * math.pi * jeffery_axial_torque(h, True),
                                1e-6)
    ft = mfs.solve_resistance(pair001["pb"], np.zeros((2, 6)), tol=1e-10, u_inf=u_inf)["ft"]
    for q in range(2):
        assert abs(ft[q, off:off + 3] @ ax - ref) < bar * abs(ref)
        expect = np.zeros(6)
        expect[off:off + 3] = ref * ax
        assert np.abs(ft[q] - expect).max() < 10 * bar * abs(ref)


def test_resistance_matrix_symmetric_positive(pair001):
    """Lorentz reciprocity: the 12 x 12 resistance matrix of the pair is
    symmetric and positive definite (to discretisation accuracy)."""
    pb = pair001["pb"]
    R = np.zeros((12, 12))
    for j in range(12):
        rbm = np.zeros((2, 6))
        rbm[j // 6, j % 6] = 1.0
        out = mfs.solve_resistance(pb, rbm, tol=1e-9)
        R[:, j] = out["ft"].reshape(-1)
    asym = np.abs(R - R.T).max() / np.abs(R).max()
    assert asym < 1e-4
    assert np.linalg.eigvalsh(0.5 * (R + R.T)).min() > 0


def test_gmres_matches_dense_lu(oracle_pairsum_built):
    """Brute force: G_hat formed column by column and solved by LU."""
    prm = geo.Params(n_proxy=60, n_colloc_base=80, n_image=4)
    c = np.array([[0.0, 0, 0], [2.05, 0.3, 0.0], [0.4, 2.3, 0.1]])
    g = geo.build(c, 1.0, prm)
    pb = mfs.Problem(g).setup()
    rbm = np.random.default_rng(5).standard_normal((3, 6))
    b = pb.rhs(rbm)
    A = pb.dense_Ghat()
    x_lu = np.linalg.solve(A, b)
    res = mfs.gmres(pb.apply, b, tol=1e-13, max_it=3 * g.T)
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(res.x - x_lu) / np.linalg.norm(x_lu) < max(1e-8, kappa * 1e-12)
    # diagonal blocks of G_hat are the identity
    for k in range(g.P):
        s = pb.tslice(k)
        assert np.abs(A[s, s] - np.eye(s.stop - s.start)).max() < 1e-14


def test_translation_and_permutation_invariance(pair001):
    """Shifting and reordering the spheres changes only rounding.  The
    truncated pseudo-inverses (eps_trunc = 5e-12) make the discrete solution
    sensitive to rounding-level changes of the node coordinates: about 1e-6
    relative in F at gap 0.01, so the bound is 1e-5."""
    pk, rbm = pair001["pk"], pair001["rbm"]
    ft0 = pair001["out"]["ft"]
    shift = np.array([3.25, -1.5, 0.75])
    c = pk.centers[::-1] + shift
    g = geo.build(c, 1.0)
    pb = mfs.Problem(g).setup()
    out = mfs.solve_resistance(pb, rbm[0][::-1], tol=1e-10)
    assert np.abs(out["ft"][::-1] - ft0).max() < 1e-5 * np.abs(ft0).max()


# -- mobility (augmented system; the paper points to it as separate work) -----

def test_mobility_single_sphere_is_stokes(single_sphere):
    """Force F and torque T on one sphere give v = F/(6 pi mu a) and
    omega = T/(8 pi mu a^3)."""
    g, pb = single_sphere
    ft = np.array([[1.0, -2.0, 0.5, 0.3, 0.0, -0.7]])
    out = mfs.solve_mobility(pb, ft, tol=1e-12)
    assert np.abs(out["rbm"][0, :3] - ft[0, :3] / (6 * math.pi)).max() < 1e-6 * np.abs(ft[0, :3]).max()
    assert np.abs(out["rbm"][0, 3:] - ft[0, 3:] / (8 * math.pi)).max() < 1e-6 * np.abs(ft[0, 3:]).max()


def test_mobility_round_trip(oracle_pairsum_built):
    """A resistance solve gives F/T from V; the mobility solve with those
    F/T returns V (the same discrete operator, exact up to the tolerance)."""
    prm = geo.Params(n_proxy=60, n_colloc_base=80, n_image=4)
    c = np.array([[0.0, 0, 0], [2.05, 0.3, 0.0], [0.4, 2.3, 0.1]])
    g = geo.build(c, 1.0, prm)
    pb = mfs.Problem(g).setup()
    rbm = np.random.default_rng(5).standard_normal((3, 6))
    r = mfs.solve_resistance(pb, rbm, tol=1e-12)
    m = mfs.solve_mobility(pb, r["ft"], tol=1e-12)
    assert np.abs(m["rbm"] - rbm).max() < 1e-8 * np.abs(rbm).max()
    assert np.abs(m["ft"] - r["ft"]).max() < 1e-8 * np.abs(r["ft"]).max()


def test_mobility_two_spheres_far_apart(oracle_pairsum_built):
    """Two unit spheres 8 radii apart, a force on the first only (mu = 1).
    Far-field hydrodynamics fixes the answer to high order in a/r: the
    second sphere moves with the Rotne-Prager-Yamakawa coupling
    (1/(8 pi r)) [(1 + 2a^2/(3r^2)) I + (1 - 2a^2/r^2) rr] F and turns with
    half the vorticity of the Stokeslet, (F x r)/(8 pi r^3); the first moves
    with F/(6 pi a), its component along the line of centres reduced by
    the first reflection, 1 - (15/4)(a/r)^4 (the method of reflections;
    transverse corrections are O((a/r)^6)).  A sign or factor slip in the
    coupling of the augmented system would show at O(1)."""
    d = 8.0
    g = geo.build(np.array([[0.0, 0.0, 0.0], [d, 0.0, 0.0]]), 1.0)
    pb = mfs.Problem(g).setup()
    F = np.array([1.0, 0.5, -0.3])
    ft = np.zeros((2, 6))
    ft[0, :3] = F
    V = mfs.solve_mobility(pb, ft, tol=1e-12)["rbm"]
    r = np.array([d, 0.0, 0.0])
    rh = r / d
    M12 = ((1 + 2 / (3 * d * d)) * np.eye(3) + (1 - 2 / (d * d)) * np.outer(rh, rh)) / (8 * math.pi * d)
    v2, w2 = M12 @ F, np.cross(F, r) / (8 * math.pi * d ** 3)
    v1 = np.array([F[0] * (1 - 15 / (4 * d ** 4)), F[1], F[2]]) / (6 * math.pi)
    scale1 = np.abs(F).max() / (6 * math.pi)
    assert np.abs(V[0, :3] - v1).max() < 1e-4 * scale1          # measured 2.2e-5
    assert np.abs(V[1, :3] - v2).max() < 2e-4 * np.abs(v2).max()  # measured 4.8e-5
    assert np.abs(V[1, 3:] - w2).max() < 1e-5 * np.abs(w2).max()  # measured 3.5e-8
    assert np.abs(V[0, 3:]).max() < 1e-6                        # measured 3.2e-8


# -- background flow (eq. bc with u_inf; the paper's fixed clusters in a
# uniform and in a shear flow) -------------------------------------------------

def _rel_err(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def test_fixed_sphere_in_uniform_flow(single_sphere):
    """A sphere held fixed in a uniform stream U feels the Stokes drag: the
    force it exerts on the fluid is -6 pi mu a U, and no torque."""
    g, pb = single_sphere
    U = np.array([5.0, -1.0, 2.0])
    out = mfs.solve_resistance(pb, np.zeros((1, 6)), tol=1e-12, u_inf=mfs.linear_flow(U=U))
    F, T = out["ft"][0, :3], out["ft"][0, 3:]
    assert _rel_err(F, -mfs.stokes_drag(1.0, 1.0, U)) < 1e-6
    assert np.abs(T).max() < 1e-6 * np.abs(F).max()


def test_fixed_sphere_in_rotational_flow(single_sphere):
    """u_inf = w x x about the origin, sphere centred at c != 0: relative to
    the sphere the fluid translates with w x c and rotates with w, so
    F = -6 pi mu a (w x c) and T = -8 pi mu a^3 w (absolute coordinates, and
    the sign of the gradient's antisymmetric part, both pinned)."""
    g, pb = single_sphere
    w = np.array([0.3, -0.7, 1.1])
    L = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])   # L x = w x x
    c = g.centers[0]
    out = mfs.solve_resistance(pb, np.zeros((1, 6)), tol=1e-12, u_inf=mfs.linear_flow(L=L))
    assert _rel_err(out["ft"][0, :3], -mfs.stokes_drag(1.0, 1.0, np.cross(w, c))) < 1e-6
    assert _rel_err(out["ft"][0, 3:], -mfs.stokes_torque(1.0, 1.0, w)) < 1e-6


def test_fixed_sphere_in_strain(single_sphere):
    """A pure strain E (symmetric, trace-free) about the origin: the sphere
    at c sees the uniform part E c (force -6 pi mu a E c) and a strain that
    exerts no torque on a sphere."""
    g, pb = single_sphere
    E = np.array([[0.4, 1.2, -0.3], [1.2, -0.9, 0.5], [-0.3, 0.5, 0.5]])
    c = g.centers[0]
    out = mfs.solve_resistance(pb, np.zeros((1, 6)), tol=1e-12, u_inf=mfs.linear_flow(L=E))
    F = out["ft"][0, :3]
    assert _rel_err(F, -mfs.stokes_drag(1.0, 1.0, E @ c)) < 1e-6
    assert np.abs(out["ft"][0, 3:]).max() < 1e-6 * np.abs(F).max()


def test_free_sphere_follows_linear_flow(single_sphere):
    """Force- and torque-free sphere in u_inf = U + L x: it moves with the
    local flow at its centre, v = U + L c, and spins with half the vorticity,
    omega_i = eps_ijk L_kj / 2 (Faxen's laws; exact for a linear flow)."""
    g, pb = single_sphere
    U = np.array([0.5, 1.5, -0.2])
    L = np.array([[0.2, 1.0, -0.4], [0.3, -0.5, 0.8], [0.6, -0.1, 0.3]])
    c = g.centers[0]
    out = mfs.solve_mobility(pb, np.zeros((1, 6)), tol=1e-12, u_inf=mfs.linear_flow(U, L))
    v_ref = U + L @ c
    om_ref = 0.5 * np.array([L[2, 1] - L[1, 2], L[0, 2] - L[2, 0], L[1, 0] - L[0, 1]])
    assert _rel_err(out["rbm"][0, :3], v_ref) < 1e-6
    assert _rel_err(out["rbm"][0, 3:], om_ref) < 1e-6


# -- residuals (eqs. residual_x, residual) and the floor rule ---------------

def _point_source_problem(c, kinds, a=1.0, mu=1.0):
    """An oracle Problem whose only sources sit at the sphere centre (one
    per entry of kinds): the exact single-sphere solutions are sums of
    such centre singularities, so the residual routine can be checked on
    fields that satisfy the boundary data exactly."""
    from types import SimpleNamespace
    g = SimpleNamespace(src_pos=np.repeat(np.asarray(c, float)[None, :], len(kinds), 0),
                        src_kind=np.asarray(kinds, np.int32), centers=np.asarray(c, float)[None, :],
                        params=SimpleNamespace(mu=mu), radius=a)
    pb = mfs.Problem.__new__(mfs.Problem)
    pb.g = g
    return pb


def test_residuals_vanish_for_exact_single_sphere_fields():
    """Translation: Stokeslet 6 pi mu a U plus dipole -pi a^3 U at the centre;
    rotation: rotlet 8 pi mu a^3 omega; both reproduce the rigid motion on
    the sphere exactly, so eps_res and the absolute form are rounding only."""
    rng = np.random.default_rng(11)
    for a, mu in ((1.0, 1.0), (1.4, 0.6)):
        c = np.array([0.4, -1.0, 2.0])
        pts = c + a * _sphere_points(300, rng)
        sph = np.zeros(len(pts), int)
        U, w = np.array([0.3, -0.9, 0.4]), np.array([-0.5, 0.2, 0.8])
        pb = _point_source_problem(c, [geo.KIND_S, geo.KIND_D, geo.KIND_R], a, mu)
        lam = np.array([6 * math.pi * mu * a * U, -math.pi * a ** 3 * U, 8 * math.pi * mu * a ** 3 * w])
        rbm = np.concatenate([U, w])[None, :]
        eps, absr = pb.residuals(lam, rbm, pts, sph)
        assert eps < 1e-14 and absr < 1e-14


def test_residuals_planted_mismatch_and_floor():
    """A field of pure rotation omega = w e_z about the centre against
    boundary data with an extra translation dU (perpendicular to the field at
    the equator point).  Equator point: |u - u_bc| = |dU|, |u_bc| =
    sqrt(w^2 a^2 + |dU|^2).  Pole point: u_bc = dU, a relative residual of 1,
    which the floor rule (read: leave out points with |u_bc| <= 1e-3 max
    |u_bc|) drops when |dU| is below 1e-3 of the largest boundary speed and
    keeps when above.  Euclidean norms per point: dU has two nonzero
    components, so a max-norm would give other values."""
    a, w = 1.0, 2.0
    c = np.array([1.0, 0.0, -0.5])
    pts = c + np.array([[a, 0.0, 0.0], [0.0, 0.0, a]])      # equator (on x), pole (on z)
    sph = np.zeros(2, int)
    pb = _point_source_problem(c, [geo.KIND_R], a)
    lam = np.array([[0.0, 0.0, 8 * math.pi * a ** 3 * w]])  # rotation about z
    # omega x r at the equator point is along +y; dU along x and z is perpendicular to it
    for s, expect_eps in ((5e-4, None), (4e-3, 1.0)):
        dU = s * w * a * np.array([0.6, 0.0, 0.8])
        rbm = np.concatenate([dU, [0.0, 0.0, w]])[None, :]
        eps, absr = pb.residuals(lam, rbm, pts, sph)
        d = np.linalg.norm(dU)
        eq = d / math.sqrt((w * a) ** 2 + d * d)
        assert abs(absr - eq) < 1e-14                     # max |u - u_bc| / max |u_bc|
        if expect_eps is None:                            # pole below the floor: left out
            assert abs(eps - eq) < 1e-14
        else:                                             # pole above the floor: ratio 1
            assert abs(eps - 1.0) < 1e-14


# -- the adaptive image count, eq. (image_est) -------------------------------

@pytest.mark.parametrize("delta,n", [(1e-3, 21), (1e-2, 12), (0.1, 3), (0.1499, 2), (0.15, 0), (0.5, 0),
                                     (2e-3, 18), (5e-2, 6)])
def test_image_rule_values(delta, n):
    """Hand-evaluated: -8.72 log10(delta) - 6.15 is 20.01 at 1e-3 (21 after
    the ceiling), 11.29 at 1e-2, 2.57 at 0.1, 1.04 at 0.1499, 17.39 at 2e-3,
    5.20 at 5e-2; zero at and above 0.15."""
    assert geo.n_image_rule(delta) == n


def test_image_rule_ceiling_boundary():
    """Where the fitted line crosses an integer the count steps up just past
    it: the value 5 is reached at log10(delta) = -11.15 / 8.72."""
    d5 = 10.0 ** (-11.15 / 8.72)
    assert geo.n_image_rule(d5 * (1 + 1e-9)) == 5
    assert geo.n_image_rule(d5 * (1 - 1e-9)) == 6


# -- GMRES: the true residual it reports ------------------------------------

def test_gmres_reports_true_residual():
    """On a well-conditioned dense system the reported true residual is
    ||b - A x|| / ||b|| of the returned x, it agrees with the recursive
    estimate far above the rounding floor, and n steps solve an n x n
    system to rounding."""
    rng = np.random.default_rng(5)
    n = 40
    A = np.eye(n) + 0.3 * rng.standard_normal((n, n)) / math.sqrt(n)
    b = rng.standard_normal(n)
    res = mfs.gmres(lambda v: A @ v, b, 1e-6, 200)
    direct = np.linalg.norm(b - A @ res.x) / np.linalg.norm(b)
    assert res.true_rel_residual == pytest.approx(direct, rel=1e-10)
    assert res.rel_residual <= 1e-6
    assert abs(res.true_rel_residual - res.rel_residual) < 1e-9
    full = mfs.gmres(lambda v: A @ v, b, 0.0, n)
    assert full.iterations == n and full.true_rel_residual < 1e-13


# -- GMRES: the iteration count against the gap (Section 5.3) ---------------

def test_gmres_count_grows_like_inverse_sqrt_gap(oracle_pairsum_built):
    """Section 5.3 (Figure iters): for four spheres on a tetrahedron, each
    pair delta apart, the GMRES count to tolerance 1e-6 grows about like
    delta^(-1/2).  Here, at a reduced discretisation (120 proxies, 160 base
    nodes, 6 image nodes) and random rigid motions, the count must grow by a
    factor in [2, 5] per decade of delta (delta^(-1/2) gives 3.16; measured
    41, 129, 400 iterations, factors 3.15 and 3.10).  A growth like 1/delta
    (a factor 10) or no lubrication-driven growth at all fails."""
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float)
    rbm = np.random.default_rng(3).standard_normal((4, 6))
    prm = geo.Params(n_proxy=120, n_colloc_base=160, n_image=6)
    its = []
    for delta in (1e-1, 1e-2, 1e-3):
        c = v * (2 + delta) / np.linalg.norm(v[0] - v[1])
        pb = mfs.Problem(geo.build(c, 1.0, prm)).setup()
        out = mfs.solve_resistance(pb, rbm, tol=1e-6)
        assert out["true_rel_residual"] < 1e-5
        its.append(out["iterations"])
    for a, b in zip(its, its[1:]):
        assert 2.0 <= b / a <= 5.0, its
