"""Seeded synthetic inputs for the Stokes-sphere resistance workloads.

This module only draws random numbers and places spheres: it holds none of
the solver's arithmetic (no kernels, no node sets, no factors).  Both the
FP64 CPU oracle and the HIP library are fed from here, so every test and
benchmark sees the same centres, radii and rigid-body velocities.

Workloads (all unit spheres, viscosity 1):

* ``two_sphere``     -- two spheres on the x axis with a given gap; the
                        squeeze/separation problem of the paper's two-sphere
                        studies (Section 3, eq. Brenner).
* ``cluster``        -- cluster-growth random sequential addition in a cube
                        sized for a target volume fraction: every new sphere
                        is placed at a log-uniform gap from a random existing
                        sphere in a random direction and rejected when it
                        leaves the cube or comes closer than ``gap_min`` to
                        any other sphere.  Stands in for the paper's random
                        clusters (Sections 4 and 5.2), whose geometries are
                        not published.
* ``serving_stream`` -- a Poisson stream of independent resistance requests:
                        sphere counts uniform in [P_lo, P_hi], volume
                        fractions uniform in [phi_lo, phi_hi], minimum gaps
                        log-uniform in [gap_lo, gap_hi] (cluster growth with
                        gaps log-uniform between the drawn minimum and one
                        radius, in a cube of side at least 6 radii, enlarged
                        by 10% steps when the growth gets stuck), rigid
                        motions N(0, 1).
* ``random_rbm``     -- rigid-body velocities (v, omega) drawn from N(0, 1).
* ``workload_block500`` -- the many-right-hand-side workload: hard-sphere
                        fluid at volume fraction 0.35 with 40% of the spheres
                        pulled into pairs at gaps log-uniform in
                        [1e-3, 5e-2], 64 sets of rigid motions.
* ``random_factors`` -- arbitrary dense factors (U, sigma, V) of given
                        shapes, used only to exercise the matrix-vector
                        product at full size with inputs that need no SVD.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Packing:
    centers: np.ndarray          # (P, 3) float64
    radius: float                # common sphere radius
    box: float                   # cube side (0 when unbounded)
    anchor_gaps: np.ndarray = field(default_factory=lambda: np.zeros(0))

    @property
    def P(self) -> int:
        return int(self.centers.shape[0])

    def min_gaps(self) -> np.ndarray:
        """Nearest-neighbour surface gap of every sphere (in radii)."""
        c = self.centers
        if c.shape[0] < 2:
            return np.full(c.shape[0], np.inf)
        d = np.sqrt(((c[:, None, :] - c[None, :, :]) ** 2).sum(-1))
        np.fill_diagonal(d, np.inf)
        return d.min(1) / self.radius - 2.0


def two_sphere(gap: float, radius: float = 1.0) -> Packing:
    """Two spheres centred at -/+ (radius + gap*radius/2) on the x axis."""
    h = radius * (1.0 + 0.5 * gap)
    c = np.array([[-h, 0.0, 0.0], [h, 0.0, 0.0]], dtype=np.float64)
    return Packing(centers=c, radius=radius, box=0.0,
                   anchor_gaps=np.array([gap]))


def separating_pair_rbm(speed: float = 1.0) -> np.ndarray:
    """Rigid-body data (1, 2, 6) for the two_sphere pair moving apart along
    the line of centres at relative speed ``speed`` (each at speed/2)."""
    rbm = np.zeros((1, 2, 6))
    rbm[0, 0, 0] = -0.5 * speed
    rbm[0, 1, 0] = +0.5 * speed
    return rbm


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def cluster(P: int, phi: float, gap_lo: float, gap_hi: float, seed: int,
            gap_min: float = 1e-3, radius: float = 1.0,
            max_tries: int = 2_000_000, min_box: float = 0.0,
            far: tuple | None = None) -> Packing:
    """Cluster-growth packing of ``P`` spheres (see module docstring); the
    cube side is at least ``min_box`` radii (a few spheres at a high volume
    fraction do not fit a cube of the nominal size).  With ``far = (frac,
    lo, hi)`` a new sphere's gap to its anchor is drawn log-uniform in
    [lo, hi] with probability ``frac`` instead of [gap_lo, gap_hi]."""
    rng = np.random.default_rng(seed)
    a = radius
    L = max((P * 4.0 * math.pi / 3.0 / phi) ** (1.0 / 3.0), min_box) * a
    centers = np.empty((P, 3))
    centers[0] = 0.5 * L
    gaps = [0.0]
    n = 1
    tries = 0
    lg_lo, lg_hi = math.log10(gap_lo), math.log10(gap_hi)
    while n < P:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("cluster packing did not converge")
        anchor = int(rng.integers(n))
        if far is not None and rng.uniform() < far[0]:
            g = 10.0 ** rng.uniform(math.log10(far[1]), math.log10(far[2]))
        else:
            g = 10.0 ** rng.uniform(lg_lo, lg_hi)
        d = _unit_vectors(rng, 1)[0]
        c = centers[anchor] + (2.0 + g) * a * d
        if np.any(c < a) or np.any(c > L - a):
            continue
        dist = np.sqrt(((centers[:n] - c) ** 2).sum(1))
        if np.min(dist) / a - 2.0 < min(gap_min, g) * (1.0 - 1e-12):
            continue
        centers[n] = c
        gaps.append(g)
        n += 1
    return Packing(centers=centers, radius=a, box=L,
                   anchor_gaps=np.asarray(gaps))


def fluid_with_pairs(P: int, phi: float, gap_min: float, pair_frac: float, pair_lo: float,
                     pair_hi: float, seed: int, sweeps: int = 40, radius: float = 1.0,
                     pair_gap_min: float = 0.1) -> Packing:
    """Random packing of ``P`` spheres in a cube at volume fraction ``phi``:
    a hard-sphere Monte Carlo fluid (random displacements from a cubic
    lattice start) in which every surface gap stays at least ``gap_min``;
    then a fraction ``pair_frac`` of the spheres is pulled together in
    nearest-neighbour pairs, each pair moved symmetrically along its line of
    centres to a gap log-uniform in [pair_lo, pair_hi], keeping a gap of at
    least ``pair_gap_min`` to every other sphere."""
    rng = np.random.default_rng(seed)
    a = radius
    L = (P * 4.0 * math.pi / 3.0 / phi) ** (1.0 / 3.0) * a
    n_side = int(math.ceil(P ** (1.0 / 3.0)))
    s = (L - 2.0 * a) / max(1, n_side - 1)
    if s < (2.0 + gap_min) * a:
        raise ValueError("volume fraction too high for the lattice start")
    idx = np.array([(i, j, k) for i in range(n_side) for j in range(n_side)
                    for k in range(n_side)])
    idx = idx[rng.permutation(len(idx))[:P]]
    c = a + idx * s
    dmin = (2.0 + gap_min) * a
    step = 0.5 * (s - dmin) + 0.1 * a
    for _ in range(sweeps):
        for i in rng.permutation(P):
            trial = c[i] + rng.uniform(-step, step, 3)
            if np.any(trial < a) or np.any(trial > L - a):
                continue
            d2 = ((c - trial) ** 2).sum(1)
            d2[i] = np.inf
            if d2.min() >= dmin * dmin:
                c[i] = trial
    # pull nearest-neighbour pairs together
    n_pairs = int(round(pair_frac * P / 2.0))
    used = np.zeros(P, bool)
    lg_lo, lg_hi = math.log10(pair_lo), math.log10(pair_hi)
    made, tries = 0, 0
    while made < n_pairs and tries < 100 * P:
        tries += 1
        i = int(rng.integers(P))
        if used[i]:
            continue
        d = np.sqrt(((c - c[i]) ** 2).sum(1))
        d[i] = np.inf
        d[used] = np.inf
        j = int(np.argmin(d))
        if not np.isfinite(d[j]):
            continue
        g = 10.0 ** rng.uniform(lg_lo, lg_hi)
        e = (c[j] - c[i]) / d[j]
        mid = 0.5 * (c[i] + c[j])
        ci, cj = mid - (1.0 + 0.5 * g) * a * e, mid + (1.0 + 0.5 * g) * a * e
        ok = True
        for cn, self_, other in ((ci, i, j), (cj, j, i)):
            dd = np.sqrt(((c - cn) ** 2).sum(1)) / a - 2.0
            dd[[self_, other]] = np.inf
            if dd.min() < pair_gap_min:
                ok = False
        if not ok:
            continue
        c[i], c[j] = ci, cj
        used[i] = used[j] = True
        made += 1
    return Packing(centers=c, radius=a, box=L)


def random_ft(P: int, nrhs: int, seed: int) -> np.ndarray:
    """Forces and torques, shape (nrhs, P, 6), every component N(0, 1)."""
    return np.random.default_rng(seed).standard_normal((nrhs, P, 6))


def random_rbm(P: int, nrhs: int, seed: int) -> np.ndarray:
    """Rigid-body velocities, shape (nrhs, P, 6) = (v_x, v_y, v_z, w_x, w_y,
    w_z), every component N(0, 1)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nrhs, P, 6))


def random_factors(rows: int, cols: int, rank: int, seed: int,
                   sigma_lo: float = 0.1):
    """Dense factors U (rows x rank), sigma (rank), V (cols x rank), all
    column-major-agnostic numpy arrays in float64.  Entries of U and V are
    N(0, 1) scaled by 1/sqrt(rows) and 1/sqrt(cols); sigma is log-uniform
    in [sigma_lo, 1] and sorted descending."""
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((rows, rank)) / math.sqrt(rows)
    V = rng.standard_normal((cols, rank)) / math.sqrt(cols)
    s = np.sort(10.0 ** rng.uniform(math.log10(sigma_lo), 0.0, rank))[::-1]
    return U, s.copy(), V


def random_vector(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(n)


# Named workloads -----------------------------------------------------------

def workload_two_sphere_gap001():
    """Two unit spheres, gap 0.01 radius, separating at unit relative speed."""
    return two_sphere(0.01), separating_pair_rbm(1.0)


def workload_packing2000(P: int = 2000, seed: int = 0):
    """Unit spheres at volume fraction 0.3: a hard-sphere fluid with every
    gap at least 0.2 (the image cutoff), with 5% of the spheres pulled into
    near-contact pairs at gaps log-uniform in [1e-3, 1e-2].  ``P`` < 2000
    gives a cut of the same recipe."""
    return fluid_with_pairs(P, 0.3, 0.2, 0.05, 1e-3, 1e-2, seed=seed)


def workload_cluster100(seed: int = 0):
    """100 unit spheres, cube at volume fraction 0.2, gaps log-uniform in
    [1e-3, 1e-1]; N(0,1) rigid-body velocities."""
    pk = cluster(100, 0.2, 1e-3, 1e-1, seed=seed)
    return pk, random_rbm(pk.P, 1, seed + 1000)


def serving_stream(n: int = 512, rate: float = 200.0, P_lo: int = 2, P_hi: int = 200,
                   phi_lo: float = 0.1, phi_hi: float = 0.3, gap_lo: float = 1e-3,
                   gap_hi: float = 1e-1, seed: int = 0):
    """``n`` requests with exponential inter-arrival times of mean 1/rate
    (seconds from the first arrival); each a dict with keys t, P, phi,
    gap_min, centers (P x 3), rbm (P x 6)."""
    rng = np.random.default_rng(seed)
    t = np.concatenate([[0.0], np.cumsum(rng.exponential(1.0 / rate, n - 1))])
    out = []
    for i in range(n):
        P = int(rng.integers(P_lo, P_hi + 1))
        phi = float(rng.uniform(phi_lo, phi_hi))
        g = float(10.0 ** rng.uniform(math.log10(gap_lo), math.log10(gap_hi)))
        cseed = int(rng.integers(1 << 31))
        box = max((P * 4.0 * math.pi / 3.0 / phi) ** (1.0 / 3.0), 6.0)
        while True:   # a cluster that gets stuck in its cube retries in a 10% larger one
            try:
                pk = cluster(P, phi, g, 1.0, seed=cseed, gap_min=g, min_box=box, max_tries=20000)
                break
            except RuntimeError:
                box *= 1.1
        out.append(dict(t=float(t[i]), P=P, phi=phi, gap_min=g, centers=pk.centers,
                        phi_actual=P * 4.0 * math.pi / 3.0 / pk.box ** 3,
                        rbm=rng.standard_normal((P, 6))))
    return out


def workload_block500(P: int = 500, seed: int = 0):
    """Unit spheres at volume fraction 0.35: a hard-sphere fluid with every
    gap at least 0.05, then 40% of the spheres pulled into nearest-neighbour
    pairs at gaps log-uniform in [1e-3, 5e-2]; 64 sets of rigid-body
    velocities N(0, 1).  ``P`` < 500 gives a cut of the same recipe."""
    pk = fluid_with_pairs(P, 0.35, 0.05, 0.4, 1e-3, 5e-2, seed=seed, pair_gap_min=0.05)
    return pk, random_rbm(pk.P, 64, seed + 2000)
