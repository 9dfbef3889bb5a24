"""Pins of the oracle's equivalent-source far field (oracle/farfield.py)
against what does not depend on it: the closed-form Stokes flow past a
translating sphere, the exact direct sum, and the degenerate case with no
far pairs.  CPU only."""
import numpy as np
import pytest

from oracle import farfield as ff, geometry as geo, mfs
from oracle.pairsum import pairsum


def _translating_flow(x, c, U, a=1.0):
    """Exterior flow of a sphere translating at U in fluid at rest (Stokes):
    u = (3a/4)(U/r + (U.e) e / r) + (a^3/4)(U/r^3 - 3 (U.e) e / r^3)."""
    r = x - c
    rn = np.linalg.norm(r, axis=1)[:, None]
    e = r / rn
    Ue = (e @ U)[:, None]
    return 0.75 * a * (U / rn + Ue * e / rn) + 0.25 * a ** 3 * (U / rn ** 3 - 3.0 * Ue * e / rn ** 3)


def test_translating_sphere_far_field_closed_form(oracle_pairsum_built):
    """One translating sphere (G_hat = I, so mu = b): the field of its
    equivalent Stokeslets at 2.5 to 6 radii equals the closed-form flow to
    the MFS error (measured 3.5e-8) and the field of its proxies to 1e-7
    (measured 8.8e-9)."""
    c = np.array([0.3, -0.2, 0.1])
    g = geo.build(c[None], 1.0)
    pb = mfs.Problem(g).setup()
    U = np.array([0.3, -1.0, 0.5])
    lam = pb.transform(pb.rhs(np.concatenate([U, np.zeros(3)])[None]))
    ep = ff.EqParams()
    E = ff.eq_map(g, ep)
    assert E.shape == (3 * ep.n_eq, 3 * g.params.n_proxy)
    rng = np.random.default_rng(0)
    d = rng.standard_normal((300, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    x = c + d * rng.uniform(ep.r_check, 6.0, 300)[:, None]
    ue = ff.equivalent_field(g, ep, E, lam[g.local_sources[0]], c, x)
    up = pairsum(x, g.src_pos, g.src_kind, lam, g.params.mu)
    us = _translating_flow(x, c, U)
    assert np.abs(ue - us).max() < 1e-6 * np.abs(us).max()
    assert np.abs(ue - up).max() < 1e-7 * np.abs(up).max()


@pytest.fixture(scope="module")
def lattice():
    """12 spheres on a 2 x 3 x 2 lattice of spacing 3.2 (far and near pairs
    at the default separation 3.5) plus one sphere 0.01 below the first
    (a contact pair: image lines, never far)."""
    cs = np.array([[i * 3.2, j * 3.2, k * 3.2] for i in range(2) for j in range(3) for k in range(2)]
                  + [[0.0, 0.0, -2.01]])
    g = geo.build(cs, 1.0)
    return g, mfs.Problem(g).setup()


def test_far_pairs_classified(lattice):
    g, _ = lattice
    ep = ff.EqParams()
    far = [(k, ks) for k in range(g.P) for ks in range(g.P) if ff.is_far(g, ep, k, ks)]
    assert far and len(far) < g.P * (g.P - 1)
    for k, ks in far:
        assert k != ks and g.contact_free(ks)
        assert np.linalg.norm(g.centers[k] - g.centers[ks]) >= ep.sep
    assert not any(ff.is_far(g, ep, k, 0) or ff.is_far(g, ep, k, 12) for k in range(g.P))


def test_apply_eq_close_to_exact_product(lattice, oracle_pairsum_built):
    """G_hat mu with equivalent far fields against the exact product:
    off-diagonal part within 1e-8 for a physical vector (measured 4.7e-10)
    and 1e-4 for a random one (measured 4.9e-6), relative 2-norm."""
    g, pb = lattice
    ep = ff.EqParams()
    E = ff.eq_map(g, ep)
    rng = np.random.default_rng(1)
    for mu, bar in ((pb.rhs(rng.standard_normal((g.P, 6))), 1e-8), (rng.standard_normal(3 * g.T), 1e-4)):
        y = pb.apply(mu)
        ye = ff.apply_eq(pb, mu, ep, E)
        assert np.linalg.norm(ye - y) / np.linalg.norm(y - mu) < bar


def test_apply_eq_without_far_pairs_is_exact(lattice, oracle_pairsum_built):
    g, pb = lattice
    mu = np.random.default_rng(2).standard_normal(3 * g.T)
    assert np.array_equal(ff.apply_eq(pb, mu, ff.EqParams(sep=100.0)), pb.apply(mu))
