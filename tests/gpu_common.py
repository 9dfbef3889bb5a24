"""Helpers shared by the GPU test modules (host-side marshalling and the
oracle's extended-precision rounding reference)."""
import sys

import numpy as np
import torch

TAG = "gpu"


def _say(msg):
    print(f"[{TAG}] {msg}", flush=True)
    sys.stdout.flush()


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float64).reshape(-1)).cuda()


def _n(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# Solver settings that keep a solve on the oracle's iteration path: the
# true-residual guard off, so GMRES stops on its recursive estimate as the
# oracle's GMRES does.
NOGUARD = dict(gmres_check_every=0)


def _finished(out):
    """A solve that ended on its tolerance or on the true-residual floor
    (not on the iteration limit); the status must be honest: OK only when
    the FP64 true residual met the tolerance."""
    return out["status"] in (0, 3)


def _rel(a, b, groups=None):
    """Element-wise relative difference: max |a - b| / max |b| over the whole
    array; with groups (one label per row of a and b viewed as
    (len(groups), -1) arrays, e.g. the sphere of every node), the largest
    such ratio over the groups, each taken against its own largest entry,
    so that an error confined to a few rows of one sphere is not diluted by
    the rest."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if groups is None:
        return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))
    lab, inv = np.unique(np.asarray(groups), return_inverse=True)
    n = len(inv)
    d = np.abs(a.reshape(n, -1) - b.reshape(n, -1)).max(1)
    m = np.abs(b.reshape(n, -1)).max(1)
    dk, mk = np.zeros(lab.size), np.zeros(lab.size)
    np.maximum.at(dk, inv, d)
    np.maximum.at(mk, inv, m)
    return float((dk / np.maximum(mk, 1e-300)).max())


def _import_oracle_factors(lib, pbo):
    for fid in range(lib.sizes.n_factors):
        info = lib.factor_info(fid)
        if info["sphere"] < 0:
            continue
        of = pbo.factors[int(pbo.factor_of[info["sphere"]])]
        assert of.U.shape[0] == info["rows"] and of.V.shape[0] == info["cols"]
        lib.import_factor(fid, of.U, of.s, of.V)


def _transform_ext(pbo, vec):
    """Oracle transform in extended precision (rounding reference)."""
    g = pbo.g
    lam = np.zeros((g.S, 3))
    for k in range(g.P):
        f = pbo.factors[int(pbo.factor_of[k])]
        mk = vec[pbo.tslice(k)].astype(np.longdouble)
        t = (f.U.astype(np.longdouble).T @ mk) / f.s.astype(np.longdouble)
        lam[g.local_sources[k]] = (f.V.astype(np.longdouble) @ t).astype(np.float64).reshape(-1, 3)
    return lam
