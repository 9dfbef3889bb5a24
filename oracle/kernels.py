"""Oracle fundamental solutions and dense target-from-source blocks (test infrastructure).

Tensors, with r = x - y (Section 2.1 eq. stokeslet; Section 2.3):
  Stokeslet          S(r) = (I + r r^T / |r|^2) / (8 pi mu |r|)
  rotlet             R(r) t = (t x r) / (8 pi mu |r|^3), i.e. the matrix
                     [[0, r3, -r2], [-r3, 0, r1], [r2, -r1, 0]] / (8 pi mu |r|^3)
  potential dipole   D(r) = (-I / |r|^3 + 3 r r^T / |r|^5) / (4 pi)   (no mu)

Pinned by exact single-sphere identities (translating sphere: Stokeslet of
strength 6 pi mu a U plus dipole of strength -pi a^3 U at the centre give
u = U on the surface; rotating sphere: rotlet 8 pi mu a^3 omega gives
omega x (x - c)), symmetry / antisymmetry and zero divergence.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import KIND_S, KIND_R, KIND_D


def stokeslet(r: np.ndarray, mu: float) -> np.ndarray:
    """(..., 3) -> (..., 3, 3)."""
    rn = np.linalg.norm(r, axis=-1)[..., None, None]
    I = np.eye(3)
    rr = r[..., :, None] * r[..., None, :]
    return (I + rr / rn ** 2) / (8.0 * math.pi * mu * rn)


def rotlet(r: np.ndarray, mu: float) -> np.ndarray:
    rn = np.linalg.norm(r, axis=-1)[..., None, None]
    z = np.zeros(r.shape[:-1])
    r1, r2, r3 = r[..., 0], r[..., 1], r[..., 2]
    m = np.stack([np.stack([z, r3, -r2], -1),
                  np.stack([-r3, z, r1], -1),
                  np.stack([r2, -r1, z], -1)], -2)
    return m / (8.0 * math.pi * mu * rn ** 3)


def dipole(r: np.ndarray) -> np.ndarray:
    rn = np.linalg.norm(r, axis=-1)[..., None, None]
    I = np.eye(3)
    rr = r[..., :, None] * r[..., None, :]
    return (-I / rn ** 3 + 3.0 * rr / rn ** 5) / (4.0 * math.pi)


def tensor(kind: int, r: np.ndarray, mu: float) -> np.ndarray:
    if kind == KIND_S:
        return stokeslet(r, mu)
    if kind == KIND_R:
        return rotlet(r, mu)
    if kind == KIND_D:
        return dipole(r)
    raise ValueError(kind)


def dense_block(x: np.ndarray, y: np.ndarray, kinds: np.ndarray, mu: float) -> np.ndarray:
    """Target-from-source matrix (3 M x 3 N), node-major rows and columns:
    block (i, j) is K_j(x_i - y_j) (Section 2.3, the blocks G^(kk'))."""
    M, N = x.shape[0], y.shape[0]
    G = np.zeros((M, 3, N, 3))
    r = x[:, None, :] - y[None, :, :]
    for kind in (KIND_S, KIND_R, KIND_D):
        sel = np.nonzero(kinds == kind)[0]
        if sel.size:
            G[:, :, sel, :] = np.transpose(tensor(kind, r[:, sel, :], mu), (0, 2, 1, 3))
    return G.reshape(3 * M, 3 * N)
