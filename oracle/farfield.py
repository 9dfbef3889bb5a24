"""Equivalent-source far field of the contact-free spheres (test
infrastructure), FP64.

The paper evaluates the all-to-all sum of eq. (uAll) (Section 2.2) with a
fast multipole method and names direct summation as the alternative.  The
library's accelerated form keeps the direct sum for every pair that needs
it and, for a target sphere k and a contact-free source sphere k' that are
well separated, replaces the field of the N proxy Stokeslets of k' by that
of n_e equivalent Stokeslets: a one-level form of the kernel-independent
multipole idea (equivalent sources whose field is fitted to the true one on
a check surface).  Every contact-free sphere has the same proxy layout
relative to its centre, so one map serves them all.

This module defines that approximation plainly (no blocking, dense
matrices), from these steps:

  equivalent points  y_e = c + r_e a u_j, u_j the n_e-point Fibonacci spiral
                     (the spiral of the proxies);
  check points       x_c = c + r_c a u'_j, the 2 n_e-point spiral;
  map                E = K(x_c, y_e)^+ K(x_c, y_p), the pseudo-inverse
                     keeping singular values above rcond sigma_1, y_p the
                     proxies: q = E lambda_hat_p are the equivalent
                     strengths of proxy strengths lambda_hat_p;
  far pairs          target sphere k, contact-free source sphere k' != k,
                     |c_k - c_k'| >= sep a: the field of q at y_e;
  every other pair   exact, as in the plain product (identity self blocks).

K is the Stokeslet tensor of eq. (stokeslet).  Nothing here comes from the
library; the parameters are the library's defaults (n_e = 200, r_e = 1,
r_c = 2.5, sep = 3.5, rcond = 1e-12).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import kernels
from .geometry import fibonacci_sphere, KIND_S
from .pairsum import pairsum


@dataclass
class EqParams:
    n_eq: int = 200          # equivalent Stokeslets per sphere
    r_eq: float = 1.0        # their radius, in sphere radii
    r_check: float = 2.5     # check-surface radius, in sphere radii
    sep: float = 3.5         # centre separation (in radii) from which a pair is far
    rcond: float = 1e-12     # pseudo-inverse cutoff, relative to sigma_1


def equivalent_points(ep: EqParams, a: float) -> np.ndarray:
    return fibonacci_sphere(ep.n_eq) * (ep.r_eq * a)


def check_points(ep: EqParams, a: float) -> np.ndarray:
    return fibonacci_sphere(2 * ep.n_eq) * (ep.r_check * a)


def free_proxies(g) -> np.ndarray:
    """Proxy positions of a contact-free sphere relative to its centre (the
    same for all of them)."""
    k = next(k for k in range(g.P) if g.contact_free(k))
    idx = np.asarray(g.local_sources[k])
    assert np.all(g.src_kind[idx] == KIND_S)
    return g.src_pos[idx] - g.centers[k]


def eq_map(g, ep: EqParams) -> np.ndarray:
    """E (3 n_e x 3 N): proxy strengths -> equivalent strengths, node-major."""
    a = g.radius
    ye, xc, yp = equivalent_points(ep, a), check_points(ep, a), free_proxies(g)
    mu = g.params.mu
    Kce = kernels.dense_block(xc, ye, np.full(len(ye), KIND_S), mu)
    Kcs = kernels.dense_block(xc, yp, np.full(len(yp), KIND_S), mu)
    return np.linalg.pinv(Kce, rcond=ep.rcond) @ Kcs


def is_far(g, ep: EqParams, k: int, ks: int) -> bool:
    """Source sphere ks reaches target sphere k through its equivalent
    sources."""
    if ks == k or not g.contact_free(ks):
        return False
    d = g.centers[k] - g.centers[ks]
    return float(d @ d) >= (ep.sep * g.radius) ** 2


def equivalent_field(g, ep: EqParams, E: np.ndarray, lam_p: np.ndarray, centre, x) -> np.ndarray:
    """Velocity at points x (n x 3) of the equivalent sources of one
    contact-free sphere centred at `centre` with proxy strengths lam_p
    (N x 3)."""
    q = E @ lam_p.reshape(-1)
    ye = equivalent_points(ep, g.radius) + centre
    K = kernels.dense_block(x, ye, np.full(len(ye), KIND_S), g.params.mu)
    return (K @ q).reshape(-1, 3)


def apply_eq(pb, mu: np.ndarray, ep: EqParams, E: np.ndarray | None = None) -> np.ndarray:
    """G_hat mu with the far pairs through equivalent sources (eq. uAll,
    Section 2.2, with the approximation above)."""
    g = pb.g
    if E is None:
        E = eq_map(g, ep)
    lam = pb.transform(mu)
    u = np.zeros((g.T, 3))
    for k in range(g.P):
        t = slice(int(g.target_offsets[k]), int(g.target_offsets[k + 1]))
        far = [ks for ks in range(g.P) if is_far(g, ep, k, ks)]
        keep = np.ones(g.S, bool)
        keep[g.src_sphere == k] = False
        for ks in far:
            keep[g.src_sphere == ks] = False
        x = g.targets[t]
        if keep.any():
            u[t] = pairsum(x, g.src_pos[keep], g.src_kind[keep], lam[keep], g.params.mu)
        for ks in far:
            u[t] += equivalent_field(g, ep, E, lam[g.local_sources[ks]], g.centers[ks], x)
    sw = np.sqrt(g.target_weight) if g.params.left_weights else np.ones(g.T)
    return mu + (sw[:, None] * u).reshape(-1)
