"""Oracle one-body preconditioned MFS solve (test infrastructure), FP64.

Steps, in the paper's order (Section 2.2, with Section 2.3 / 5.1 additions):
  setup      B_k = W_k G^(kk) (left weights, Remark left-precond), thin SVD
             B_k = U S V^T, keep sigma_i > trunc_rel * sigma_1 (Section 5,
             eps_trunc = 5e-12).  Contact-free spheres have identical node
             sets relative to their centres and share one factor.
  rhs        b_k = W_k (v_k + omega_k x (x - c_k) - u_inf(x)), eq. (bc).
  transform  lambda_hat_k = V (S^+ (U^T mu_k)), eq. (transform).
  all-to-all u_All = G lambda_hat, eq. (uAll); with direct summation the
             self blocks are skipped and replaced by the identity, so
             (G_hat mu)_k = mu_k + W_k sum_{k' != k} G^(kk') lambda_hat_k'.
  GMRES      on G_hat mu = b, x0 = 0, classical Gram-Schmidt applied twice,
             Givens rotations; stops when the recursive (Givens) estimate
             of ||b - G_hat mu|| / ||b|| is <= tol, and reports the true
             relative residual ||b - G_hat mu|| / ||b|| of the iterate it
             returns beside the estimate (restart length, start vector,
             orthogonalisation and stopping rule are not stated in the
             paper; this is the reading used here).
  post       lambda = B^+ mu (same transform), force and torque
             (Remark: extracting net forces and torques), surface velocity
             and the pointwise relative residual, eqs. (residual_x),
             (residual), (force_err).
The dense brute force ``dense_Ghat`` forms G_hat column by column from the
same transform and blocks; it is used to pin GMRES on small problems.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from . import kernels
from .geometry import Geometry, KIND_S, KIND_R
from .pairsum import pairsum


@dataclass
class Factor:
    U: np.ndarray       # (3M, r)
    s: np.ndarray       # (r,)
    V: np.ndarray       # (3N, r)
    sigma_max: float
    full_rank: int


def row_scale(g: Geometry, k: int) -> np.ndarray:
    """sqrt(w_i) repeated over the three components of node i of sphere k."""
    t0, t1 = g.target_offsets[k], g.target_offsets[k + 1]
    w = g.target_weight[t0:t1] if g.params.left_weights else np.ones(t1 - t0)
    return np.repeat(np.sqrt(w), 3)


def self_block(g: Geometry, k: int) -> np.ndarray:
    """B_k = W_k G^(kk)."""
    t0, t1 = g.target_offsets[k], g.target_offsets[k + 1]
    src = g.local_sources[k]
    G = kernels.dense_block(g.targets[t0:t1], g.src_pos[src], g.src_kind[src], g.params.mu)
    return row_scale(g, k)[:, None] * G


def truncated_svd(B: np.ndarray, trunc_rel: float) -> Factor:
    U, s, Vt = sla.svd(B, full_matrices=False, lapack_driver="gesvd")
    keep = s > trunc_rel * s[0]
    return Factor(U=U[:, keep].copy(), s=s[keep].copy(), V=Vt[keep].T.copy(),
                  sigma_max=float(s[0]), full_rank=int(s.size))


class Problem:
    """Discretised resistance problem with its per-sphere factors."""

    def __init__(self, g: Geometry, factors: dict | None = None):
        self.g = g
        self.factor_of = np.zeros(g.P, np.int64)   # factor id per sphere
        # factor id 0 = shared contact-free factor (if any contact-free
        # sphere exists), then one per contact sphere in sphere order.
        nid = 1
        for k in range(g.P):
            if g.contact_free(k):
                self.factor_of[k] = 0
            else:
                self.factor_of[k] = nid
                nid += 1
        self.n_factors = nid
        self.factors = factors if factors is not None else {}

    def representative(self, fid: int) -> int:
        return int(np.nonzero(self.factor_of == fid)[0][0])

    def factor_ids(self):
        return sorted(set(int(f) for f in self.factor_of))

    def setup(self):
        for fid in self.factor_ids():
            if fid not in self.factors:
                k = self.representative(fid)
                self.factors[fid] = truncated_svd(self_block(self.g, k), self.g.params.trunc_rel)
        return self

    # -- the operator ------------------------------------------------------

    def tslice(self, k):
        g = self.g
        return slice(3 * int(g.target_offsets[k]), 3 * int(g.target_offsets[k + 1]))

    def transform(self, mu: np.ndarray) -> np.ndarray:
        """lambda (S x 3, packed by kind) from mu (3T), eq. (transform) per sphere."""
        g = self.g
        lam = np.zeros((g.S, 3))
        for k in range(g.P):
            f = self.factors[int(self.factor_of[k])]
            lk = f.V @ ((f.U.T @ mu[self.tslice(k)]) / f.s)
            lam[g.local_sources[k]] = lk.reshape(-1, 3)
        return lam

    def apply(self, mu: np.ndarray, lam_hat: np.ndarray | None = None) -> np.ndarray:
        """(G_hat mu): identity self blocks plus weighted off-diagonal sums."""
        g = self.g
        if lam_hat is None:
            lam_hat = self.transform(mu)
        u = pairsum(g.targets, g.src_pos, g.src_kind, lam_hat, g.params.mu,
                    tsph=g.target_sphere, ssph=g.src_sphere, skip_same=True)
        sw = np.sqrt(g.target_weight) if g.params.left_weights else np.ones(g.T)
        return mu + (sw[:, None] * u).reshape(-1)

    def apply_rows(self, mu_or_lam, rows: np.ndarray, is_lambda=False) -> np.ndarray:
        """Selected target rows of (G_hat mu), returned (len(rows), 3)."""
        g = self.g
        lam_hat = mu_or_lam if is_lambda else self.transform(mu_or_lam)
        u = pairsum(g.targets[rows], g.src_pos, g.src_kind, lam_hat, g.params.mu,
                    tsph=g.target_sphere[rows], ssph=g.src_sphere, skip_same=True)
        sw = np.sqrt(g.target_weight[rows]) if g.params.left_weights else np.ones(len(rows))
        return sw[:, None] * u

    # -- right-hand side ---------------------------------------------------

    def boundary_velocity(self, rbm: np.ndarray, pts: np.ndarray, sph: np.ndarray,
                          u_inf=None) -> np.ndarray:
        """u_bc at points on sphere sph, eq. (bc); rbm is (P, 6)."""
        c = self.g.centers[sph]
        v, w = rbm[sph, :3], rbm[sph, 3:]
        u = v + np.cross(w, pts - c)
        if u_inf is not None:
            u = u - u_inf(pts)
        return u

    def rhs(self, rbm: np.ndarray, u_inf=None) -> np.ndarray:
        g = self.g
        ubc = self.boundary_velocity(rbm, g.targets, g.target_sphere, u_inf)
        sw = np.sqrt(g.target_weight) if g.params.left_weights else np.ones(g.T)
        return (sw[:, None] * ubc).reshape(-1)

    # -- post-processing ---------------------------------------------------

    def force_torque(self, lam: np.ndarray) -> np.ndarray:
        """(P, 6): F = sum of Stokeslet strengths, T = sum of rotlet strengths
        + sum (y - c) x f over Stokeslets."""
        g = self.g
        out = np.zeros((g.P, 6))
        for k in range(g.P):
            idx = g.local_sources[k]
            kinds = g.src_kind[idx]
            s = idx[kinds == KIND_S]
            r = idx[kinds == KIND_R]
            f = lam[s]
            out[k, :3] = f.sum(0)
            out[k, 3:] = np.cross(g.src_pos[s] - g.centers[k], f).sum(0) + lam[r].sum(0)
        return out

    def velocity(self, lam: np.ndarray, pts: np.ndarray) -> np.ndarray:
        g = self.g
        return pairsum(pts, g.src_pos, g.src_kind, lam, g.params.mu)

    def residuals(self, lam, rbm, pts, sph, u_inf=None, floor=1e-3):
        """Pointwise relative residual, eq. (residual_x); points where
        |u_bc| is below floor * max|u_bc| are left out (the ratio is
        undefined where u_bc vanishes).  Returns (max eps_res, max abs err /
        max |u_bc|)."""
        u = self.velocity(lam, pts)
        ubc = self.boundary_velocity(rbm, pts, sph, u_inf)
        err = np.linalg.norm(u - ubc, axis=1)
        nb = np.linalg.norm(ubc, axis=1)
        m = nb > floor * nb.max()
        return float((err[m] / nb[m]).max()), float(err.max() / nb.max())

    # -- dense brute force ---------------------------------------------------

    def dense_Ghat(self) -> np.ndarray:
        n = 3 * self.g.T
        A = np.zeros((n, n))
        e = np.zeros(n)
        for j in range(n):
            e[j] = 1.0
            A[:, j] = self.apply(e)
            e[j] = 0.0
        return A


@dataclass
class GmresResult:
    x: np.ndarray
    iterations: int
    rel_residual: float        # recursive estimate at exit
    history: list
    true_rel_residual: float = float("nan")   # ||b - A x|| / ||b|| of the returned x


def gmres(apply, b: np.ndarray, tol: float, max_it: int, restart: int | None = None,
          fixed_iterations: int | None = None) -> GmresResult:
    """GMRES(m) with x0 = 0, classical Gram-Schmidt applied twice and Givens
    rotations; stops when the recursive residual estimate is <= tol (or at
    max_it), and reports the true relative residual of the returned x.
    ``fixed_iterations`` forces exactly that many Arnoldi steps (for
    step-by-step comparisons)."""
    n = b.size
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n)
    if bnorm == 0.0:
        return GmresResult(x, 0, 0.0, [0.0], 0.0)
    m = restart or max_it
    total = 0
    hist = [1.0]
    r = b.copy()
    while True:
        beta = float(np.linalg.norm(r))
        Q = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        Q[0] = r / beta
        j_done = 0
        converged = False
        for j in range(m):
            w = apply(Q[j])
            h = Q[: j + 1] @ w
            w = w - Q[: j + 1].T @ h
            h2 = Q[: j + 1] @ w
            w = w - Q[: j + 1].T @ h2
            h = h + h2
            hn = float(np.linalg.norm(w))
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            if hn > 0.0:
                Q[j + 1] = w / hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = math.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_done = j + 1
            res = abs(g[j + 1]) / bnorm
            hist.append(res)
            if fixed_iterations is not None:
                if total >= fixed_iterations:
                    converged = True
                    break
            elif res <= tol or total >= max_it or hn == 0.0:
                converged = True
                break
        y = sla.solve_triangular(H[:j_done, :j_done], g[:j_done])
        x = x + Q[:j_done].T @ y
        r = b - apply(x)
        if converged:
            return GmresResult(x, total, hist[-1], hist, float(np.linalg.norm(r)) / bnorm)


def solve_resistance(pb: Problem, rbm: np.ndarray, tol=1e-10, max_it=500,
                     restart=None, u_inf=None, fixed_iterations=None):
    """Full oracle solve: returns dict with mu, lambda, F/T (P x 6), GMRES info."""
    b = pb.rhs(rbm, u_inf)
    res = gmres(pb.apply, b, tol, max_it, restart, fixed_iterations)
    lam = pb.transform(res.x)
    return dict(mu=res.x, lam=lam, ft=pb.force_torque(lam), iterations=res.iterations,
                rel_residual=res.rel_residual, true_rel_residual=res.true_rel_residual, b=b,
                history=res.history)


def mobility_scales(pb: Problem):
    """Row scales of the force and torque equations: 1/(6 pi mu a) and
    1/(8 pi mu a^3), so that they read in velocity units."""
    g = pb.g
    return (1.0 / (6.0 * math.pi * g.params.mu * g.radius),
            1.0 / (8.0 * math.pi * g.params.mu * g.radius ** 3))


def mobility_apply(pb: Problem, x: np.ndarray) -> np.ndarray:
    """Augmented operator of the mobility problem (not in the paper; the
    reading used here).  Unknowns (mu, V) with V the rigid motions (v, omega)
    of every sphere.  Rows: the resistance rows G_hat mu - W Psi V, where
    Psi V = v + omega x (x - c) at the collocation nodes, and the force and
    torque of lambda = B^+ mu (Remark on extracting forces and torques),
    scaled by mobility_scales."""
    g = pb.g
    n = 3 * g.T
    mu, V = x[:n], x[n:].reshape(g.P, 6)
    lam = pb.transform(mu)
    top = pb.apply(mu, lam) - pb.rhs(V)
    sF, sT = mobility_scales(pb)
    ft = pb.force_torque(lam)
    ft[:, :3] *= sF
    ft[:, 3:] *= sT
    return np.concatenate([top, ft.reshape(-1)])


def linear_flow(U=None, L=None):
    """u_inf(x) = U + L x for points x (n, 3), L[i][j] = d u_inf_i / d x_j:
    the background flows of the paper's fixed-cluster examples (uniform and
    shear) are of this form; a trace-free L makes it a Stokes solution."""
    U = np.zeros(3) if U is None else np.asarray(U, np.float64)
    L = np.zeros((3, 3)) if L is None else np.asarray(L, np.float64)
    return lambda x: U[None, :] + np.asarray(x) @ L.T


def solve_mobility(pb: Problem, ft: np.ndarray, tol=1e-10, max_it=1000, u_inf=None):
    """Forces and torques (P, 6) in, rigid motions out.  In a background
    flow u_inf the velocity rows of the right-hand side are the boundary
    data of spheres at rest, -W u_inf (eq. bc with v = omega = 0, the
    unknown motion being on the left)."""
    g = pb.g
    n = 3 * g.T
    sF, sT = mobility_scales(pb)
    rhs_ft = np.array(ft, dtype=np.float64).copy()
    rhs_ft[:, :3] *= sF
    rhs_ft[:, 3:] *= sT
    top = np.zeros(n) if u_inf is None else pb.rhs(np.zeros((g.P, 6)), u_inf)
    b = np.concatenate([top, rhs_ft.reshape(-1)])
    res = gmres(lambda v: mobility_apply(pb, v), b, tol, max_it)
    mu, V = res.x[:n], res.x[n:].reshape(g.P, 6)
    lam = pb.transform(mu)
    return dict(mu=mu, rbm=V, lam=lam, ft=pb.force_torque(lam), iterations=res.iterations,
                rel_residual=res.rel_residual, true_rel_residual=res.true_rel_residual)


def stokes_drag(mu, a, U):
    """Force on the fluid by a sphere translating at U in unbounded fluid."""
    return 6.0 * math.pi * mu * a * np.asarray(U)


def stokes_torque(mu, a, omega):
    return 8.0 * math.pi * mu * a ** 3 * np.asarray(omega)
