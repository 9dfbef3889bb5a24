"""Thin ctypes binding of libsmfs (the C-ABI in include/smfs.h).

Only argument marshalling lives here: every numerical step runs in the HIP
library.  PyTorch provides device memory (the caller-owned workspace and the
vectors) and the current HIP stream.  If libsmfs.so is missing this module
raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SMFS_LIB", os.path.join(HERE, "libsmfs.so"))

SMFS_OK = 0
SMFS_NOT_CONVERGED = 1
SMFS_GAP_BELOW_VALIDATED = 2
SMFS_STAGNATED = 3
SMFS_E_AGAIN = -8
SOLVE_WARNINGS = (SMFS_OK, SMFS_NOT_CONVERGED, SMFS_STAGNATED)
SMFS_FP64, SMFS_MIXED, SMFS_MIXED_FAR, SMFS_MIXED_EQ = 0, 1, 2, 3
SMFS_SVD_JACOBI, SMFS_SVD_ROCSOLVER = 0, 1
KIND_S, KIND_R, KIND_D = 1, 2, 4

EXPORTED = [
    "smfs_params_default", "smfs_problem_create", "smfs_problem_destroy", "smfs_problem_sizes",
    "smfs_export_nodes", "smfs_sphere_factor", "smfs_factor_info", "smfs_bind", "smfs_setup",
    "smfs_setup_workspace_bytes", "smfs_far_field_workspace_bytes", "smfs_setup_far_field",
    "smfs_import_factor", "smfs_apply", "smfs_transform", "smfs_rhs", "smfs_set_background",
    "smfs_force_torque",
    "smfs_eval_velocity", "smfs_solve_resistance", "smfs_solve_mobility", "smfs_set_solver",
    "smfs_pairs_per_apply", "smfs_block_workspace_bytes", "smfs_apply_block",
    "smfs_apply_block_noalloc", "smfs_noalloc_scratch_bytes",
    "smfs_solve_resistance_block", "smfs_server_create", "smfs_server_destroy",
    "smfs_server_clock", "smfs_server_submit", "smfs_server_step", "smfs_server_poll",
    "smfs_server_config_default", "smfs_server_memory_bytes",
    "smfs_server_release", "smfs_server_stats_read",
    "smfs_profile",
    "smfs_profile_read", "smfs_last_error",
]


class smfs_params(C.Structure):
    _fields_ = [
        ("n_proxy", C.c_int32), ("proxy_radius", C.c_double), ("n_colloc_base", C.c_int32),
        ("n_image", C.c_int32), ("image_kinds", C.c_uint32), ("image_offset", C.c_double),
        ("image_gap_cutoff", C.c_double), ("near_gap_cutoff", C.c_double),
        ("cap_alpha", C.c_int32 * 2), ("cap_beta", C.c_double * 2), ("left_weights", C.c_int32),
        ("trunc_rel", C.c_double), ("mu", C.c_double), ("n_check_base", C.c_int32),
        ("precision", C.c_int32), ("gmres_tol", C.c_double), ("gmres_max_it", C.c_int32),
        ("gmres_restart", C.c_int32), ("gmres_check_every", C.c_int32), ("svd_method", C.c_int32),
        ("eq_points", C.c_int32), ("eq_radius", C.c_double), ("eq_check_radius", C.c_double),
        ("eq_separation", C.c_double), ("eq_rcond", C.c_double), ("progress", C.c_int32),
    ]


class smfs_sizes(C.Structure):
    _fields_ = [
        ("P", C.c_int32), ("n_factors", C.c_int32), ("n_contacts", C.c_int32),
        ("min_gap_flag", C.c_int32), ("T", C.c_int64), ("S", C.c_int64),
        ("n_kind", C.c_int64 * 3), ("n_check", C.c_int64), ("workspace_bytes", C.c_size_t),
        ("factor_bytes", C.c_size_t), ("svd_sweeps", C.c_int32),
        ("eq_far_pairs", C.c_int64), ("eq_exact_pairs", C.c_int64), ("eq_near_spheres", C.c_int64),
    ]


class smfs_out(C.Structure):
    _fields_ = [
        ("mu", C.c_void_p), ("lambda_", C.c_void_p), ("ft", C.c_void_p), ("u_check", C.c_void_p),
        ("rbm", C.c_void_p),
        ("iterations", C.c_int32), ("rel_residual", C.c_double),
        ("true_rel_residual", C.c_double), ("lambda_inf", C.c_double),
        ("eps_res_max", C.c_double), ("abs_res_max", C.c_double), ("t_rhs_ms", C.c_double),
        ("t_gmres_ms", C.c_double), ("t_post_ms", C.c_double), ("pair_evals", C.c_int64),
        ("pair_evals_f32", C.c_int64), ("refinements", C.c_int32),
        ("true_checks", C.c_int32), ("floor_iteration", C.c_int32), ("floor_rel_residual", C.c_double),
    ]


class smfs_kernel_stats(C.Structure):
    _fields_ = [
        ("direct_launches", C.c_int64), ("direct_ms", C.c_double), ("direct_flops", C.c_double),
        ("pinv_launches", C.c_int64), ("pinv_ms", C.c_double), ("pinv_bytes", C.c_double),
        ("far32_launches", C.c_int64), ("far32_ms", C.c_double), ("far32_flops", C.c_double),
        ("mixed64_launches", C.c_int64), ("mixed64_ms", C.c_double), ("mixed64_flops", C.c_double),
        ("bdirect_launches", C.c_int64), ("bdirect_ms", C.c_double), ("bdirect_flops", C.c_double),
        ("bpinv_launches", C.c_int64), ("bpinv_ms", C.c_double), ("bpinv_flops", C.c_double),
        ("bnrhs", C.c_int32),
        ("eq_launches", C.c_int64), ("eq_far_ms", C.c_double), ("eq_far_flops", C.c_double),
        ("eq_near_ms", C.c_double), ("eq_near_flops", C.c_double), ("eq_strength_ms", C.c_double),
    ]


class smfs_request_result(C.Structure):
    _fields_ = [
        ("status", C.c_int32), ("P", C.c_int32), ("iterations", C.c_int32), ("restarts", C.c_int32),
        ("rel_residual", C.c_double), ("true_rel_residual", C.c_double),
        ("t_arrival", C.c_double), ("t_admitted", C.c_double), ("t_started", C.c_double),
        ("t_done", C.c_double), ("pair_evals", C.c_int64), ("pair_evals_f32", C.c_int64),
        ("refinements", C.c_int32), ("error", C.c_char * 160),
    ]


class smfs_server_config(C.Structure):
    _fields_ = [
        ("radius", C.c_double), ("max_active", C.c_int32), ("setup_workers", C.c_int32),
        ("max_queued", C.c_int32), ("precision", C.c_int32), ("worker_scratch_bytes", C.c_size_t),
        ("iters_per_step", C.c_int32), ("setup_batch", C.c_int32),
    ]


class smfs_server_stats(C.Structure):
    _fields_ = [
        ("steps", C.c_int64), ("request_iterations", C.c_int64), ("completed", C.c_int64),
        ("failed", C.c_int64), ("arena_bytes", C.c_size_t), ("arena_peak", C.c_size_t),
        ("peak_active", C.c_int32), ("step_ms", C.c_double), ("tick_ms", C.c_double),
        ("setup_ms", C.c_double),
        ("setup_batches", C.c_int64), ("iterations", C.c_int64),
    ]


class smfs_block_out(C.Structure):
    _fields_ = [
        ("ft", C.c_void_p), ("mu", C.c_void_p), ("iterations", C.c_void_p),
        ("true_rel_residual", C.c_void_p), ("max_iterations", C.c_int32),
        ("n_converged", C.c_int32), ("t_gmres_ms", C.c_double), ("t_post_ms", C.c_double),
        ("pair_evals", C.c_int64), ("pair_evals_f32", C.c_int64), ("refinements", C.c_int32),
    ]


_lib = None


def lib():
    """Load libsmfs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2407_03343_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "smfs_params_default": ([P(smfs_params)], C.c_int),
        "smfs_problem_create": ([P(smfs_params), i32, vp, vp, P(vp)], C.c_int),
        "smfs_problem_destroy": ([vp], None),
        "smfs_problem_sizes": ([vp, P(smfs_sizes)], C.c_int),
        "smfs_export_nodes": ([vp] + [vp] * 8, C.c_int),
        "smfs_sphere_factor": ([vp, i32, P(i32)], C.c_int),
        "smfs_factor_info": ([vp, i32, P(i32), P(i32), P(i32), P(i32)], C.c_int),
        "smfs_bind": ([vp, vp, C.c_size_t, vp], C.c_int),
        "smfs_setup_workspace_bytes": ([vp, P(C.c_size_t)], C.c_int),
        "smfs_setup": ([vp, vp, C.c_size_t, vp], C.c_int),
        "smfs_far_field_workspace_bytes": ([vp, P(C.c_size_t)], C.c_int),
        "smfs_setup_far_field": ([vp, vp, C.c_size_t, vp], C.c_int),
        "smfs_import_factor": ([vp, i32, i32, vp, vp, vp, vp], C.c_int),
        "smfs_apply": ([vp, vp, vp, i32, vp], C.c_int),
        "smfs_transform": ([vp, vp, vp, vp], C.c_int),
        "smfs_rhs": ([vp, vp, vp, vp], C.c_int),
        "smfs_set_background": ([vp, vp, vp], C.c_int),
        "smfs_force_torque": ([vp, vp, vp, vp], C.c_int),
        "smfs_eval_velocity": ([vp, vp, i64, vp, vp, vp], C.c_int),
        "smfs_solve_resistance": ([vp, vp, P(smfs_out), vp], C.c_int),
        "smfs_solve_mobility": ([vp, vp, P(smfs_out), vp], C.c_int),
        "smfs_pairs_per_apply": ([vp], i64),
        "smfs_block_workspace_bytes": ([vp, i32, i32, P(C.c_size_t)], C.c_int),
        "smfs_server_config_default": ([P(smfs_server_config)], C.c_int),
        "smfs_server_memory_bytes": ([P(smfs_params), P(smfs_server_config), P(C.c_size_t)], C.c_int),
        "smfs_server_create": ([P(smfs_params), P(smfs_server_config), vp, C.c_size_t, P(vp)], C.c_int),
        "smfs_server_destroy": ([vp], None),
        "smfs_server_clock": ([], dbl),
        "smfs_server_submit": ([vp, i32, vp, vp, dbl, P(i64)], C.c_int),
        "smfs_server_step": ([vp, P(i32), P(i32)], C.c_int),
        "smfs_server_poll": ([vp, i64, P(smfs_request_result), vp], C.c_int),
        "smfs_server_release": ([vp, i64], C.c_int),
        "smfs_server_stats_read": ([vp, P(smfs_server_stats)], C.c_int),
        "smfs_apply_block": ([vp, i32, vp, vp, i64, i32, vp, C.c_size_t, vp], C.c_int),
        "smfs_apply_block_noalloc": ([vp, i32, vp, vp, i64, vp], C.c_int),
        "smfs_noalloc_scratch_bytes": ([], C.c_size_t),
        "smfs_solve_resistance_block": ([vp, i32, vp, i32, vp, C.c_size_t, P(smfs_block_out), vp],
                                        C.c_int),
        "smfs_set_solver": ([vp, i32, dbl, i32], C.c_int),
        "smfs_profile": ([vp, i32], C.c_int),
        "smfs_profile_read": ([vp, P(smfs_kernel_stats)], C.c_int),
        "smfs_last_error": ([], C.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


class SmfsError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().smfs_last_error().decode()
        super().__init__(f"{where} failed with code {code}: {msg}")
        self.code = code


def _check(rc, where, ok=(SMFS_OK,)):
    if rc not in ok:
        raise SmfsError(rc, where)
    return rc


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def params_default(**over) -> smfs_params:
    p = smfs_params()
    _check(lib().smfs_params_default(C.byref(p)), "smfs_params_default")
    for k, v in over.items():
        if k in ("cap_alpha", "cap_beta"):
            arr = getattr(p, k)
            arr[0], arr[1] = v
        else:
            setattr(p, k, v)
    return p


class Problem:
    """One discretised resistance problem (host geometry + device state)."""

    def __init__(self, centers, radius=1.0, params: smfs_params | None = None, **over):
        self.params = params if params is not None else params_default(**over)
        c = np.ascontiguousarray(centers, np.float64).reshape(-1, 3)
        self.P = c.shape[0]
        r = np.full(self.P, float(radius))
        h = C.c_void_p()
        rc = lib().smfs_problem_create(C.byref(self.params), self.P, _np_ptr(c), _np_ptr(r), C.byref(h))
        _check(rc, "smfs_problem_create", ok=(SMFS_OK, SMFS_GAP_BELOW_VALIDATED))
        self.gap_warning = rc == SMFS_GAP_BELOW_VALIDATED
        self.h = h
        self.sizes = smfs_sizes()
        _check(lib().smfs_problem_sizes(self.h, C.byref(self.sizes)), "smfs_problem_sizes")
        self.T, self.S, self.n_check = self.sizes.T, self.sizes.S, self.sizes.n_check
        self.ws = None

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().smfs_problem_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # -- host introspection ---------------------------------------------------
    def export_nodes(self):
        T, S, Cn = self.T, self.S, self.n_check
        out = dict(targets=np.zeros((T, 3)), target_sphere=np.zeros(T, np.int32),
                   target_weight=np.zeros(T), sources=np.zeros((S, 3)),
                   source_kind=np.zeros(S, np.int32), source_sphere=np.zeros(S, np.int32),
                   check=np.zeros((Cn, 3)), check_sphere=np.zeros(Cn, np.int32))
        _check(lib().smfs_export_nodes(self.h, *[_np_ptr(out[k]) for k in (
            "targets", "target_sphere", "target_weight", "sources", "source_kind",
            "source_sphere", "check", "check_sphere")]), "smfs_export_nodes")
        return out

    def sphere_factor(self, k):
        f = C.c_int32()
        _check(lib().smfs_sphere_factor(self.h, k, C.byref(f)), "smfs_sphere_factor")
        return f.value

    def factor_info(self, fid):
        r, c, k, s = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().smfs_factor_info(self.h, fid, C.byref(r), C.byref(c), C.byref(k), C.byref(s)),
               "smfs_factor_info")
        return dict(rows=r.value, cols=c.value, rank=k.value, sphere=s.value)

    @property
    def pairs_per_apply(self):
        return int(lib().smfs_pairs_per_apply(self.h))

    def set_solver(self, precision=None, tol=None, max_it=None):
        p = self.params
        precision = p.precision if precision is None else precision
        tol = p.gmres_tol if tol is None else tol
        max_it = p.gmres_max_it if max_it is None else max_it
        _check(lib().smfs_set_solver(self.h, precision, tol, max_it), "smfs_set_solver")
        p.precision, p.gmres_tol, p.gmres_max_it = precision, tol, max_it

    def set_background(self, U=None, L=None):
        """Background flow u_inf(x) = U + L x of the boundary data (eq. bc);
        L[i][j] = d u_inf_i / d x_j.  No arguments: quiescent fluid."""
        u = None if U is None else np.ascontiguousarray(U, np.float64).reshape(3)
        g = None if L is None else np.ascontiguousarray(L, np.float64).reshape(9)
        _check(lib().smfs_set_background(self.h, None if u is None else _np_ptr(u),
                                         None if g is None else _np_ptr(g)), "smfs_set_background")

    def profile(self, enable: bool):
        _check(lib().smfs_profile(self.h, 1 if enable else 0), "smfs_profile")

    def profile_read(self) -> dict:
        st = smfs_kernel_stats()
        _check(lib().smfs_profile_read(self.h, C.byref(st)), "smfs_profile_read")
        return {k: getattr(st, k) for k, _ in smfs_kernel_stats._fields_}

    # -- device ----------------------------------------------------------------
    def bind(self, device="cuda"):
        import torch
        nbytes = int(self.sizes.workspace_bytes)
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        aligned = (base + 255) // 256 * 256
        _check(lib().smfs_bind(self.h, C.c_void_p(aligned), nbytes, _stream()), "smfs_bind")
        return self

    def setup_workspace_bytes(self):
        n = C.c_size_t(0)
        _check(lib().smfs_setup_workspace_bytes(self.h, C.byref(n)), "smfs_setup_workspace_bytes")
        return int(n.value)

    def setup(self):
        """Assemble and factor the self blocks; the device scratch of the
        SVDs is a torch allocation released afterwards."""
        import torch
        n = self.setup_workspace_bytes()
        buf = torch.empty(n + 256, dtype=torch.uint8, device="cuda")
        base = (buf.data_ptr() + 255) // 256 * 256
        _check(lib().smfs_setup(self.h, C.c_void_p(base), n, _stream()), "smfs_setup")
        del buf
        _check(lib().smfs_problem_sizes(self.h, C.byref(self.sizes)), "smfs_problem_sizes")
        return self

    def setup_far_field(self):
        """Fit the equivalent sources of the contact-free spheres (needed by
        SMFS_MIXED_EQ products; smfs_setup runs it too)."""
        import torch
        n = C.c_size_t(0)
        _check(lib().smfs_far_field_workspace_bytes(self.h, C.byref(n)), "smfs_far_field_workspace_bytes")
        buf = torch.empty(int(n.value) + 256, dtype=torch.uint8, device="cuda")
        base = (buf.data_ptr() + 255) // 256 * 256
        _check(lib().smfs_setup_far_field(self.h, C.c_void_p(base), int(n.value), _stream()),
               "smfs_setup_far_field")
        del buf
        return self

    def import_factor(self, fid, U, sigma, V):
        U = np.asfortranarray(U, np.float64)          # rows x rank, column-major
        V = np.ascontiguousarray(V, np.float64)       # cols x rank, row-major
        s = np.ascontiguousarray(sigma, np.float64)
        info = self.factor_info(fid)
        r = s.size
        if U.shape != (info["rows"], r) or V.shape != (info["cols"], r) or not 0 < r <= info["cols"]:
            raise ValueError(f"factor {fid}: expected U {info['rows']}x{r} and V {info['cols']}x{r}")
        _check(lib().smfs_import_factor(self.h, fid, s.size, _np_ptr(U), _np_ptr(s), _np_ptr(V),
                                        _stream()), "smfs_import_factor")

    def _dvec(self, n, like=None):
        import torch
        return torch.empty(n, dtype=torch.float64, device="cuda")

    @staticmethod
    def _need(t, n, what):
        import torch
        if (not torch.is_tensor(t) or t.dtype != torch.float64 or not t.is_cuda
                or not t.is_contiguous() or t.numel() != n):
            raise ValueError(f"{what}: expected a contiguous float64 device tensor of {n} values")

    def apply(self, mu, precision=SMFS_FP64, out=None):
        self._need(mu, 3 * self.T, "mu")
        y = out if out is not None else self._dvec(3 * self.T)
        self._need(y, 3 * self.T, "y")
        _check(lib().smfs_apply(self.h, _ptr(mu), _ptr(y), precision, _stream()), "smfs_apply")
        return y

    def transform(self, mu, out=None):
        self._need(mu, 3 * self.T, "mu")
        lam = out if out is not None else self._dvec(3 * self.S)
        self._need(lam, 3 * self.S, "lambda")
        _check(lib().smfs_transform(self.h, _ptr(mu), _ptr(lam), _stream()), "smfs_transform")
        return lam

    def rhs(self, rbm):
        self._need(rbm, 6 * self.P, "rbm")
        b = self._dvec(3 * self.T)
        _check(lib().smfs_rhs(self.h, _ptr(rbm), _ptr(b), _stream()), "smfs_rhs")
        return b

    def force_torque(self, lam):
        self._need(lam, 3 * self.S, "lambda")
        ft = self._dvec(6 * self.P)
        _check(lib().smfs_force_torque(self.h, _ptr(lam), _ptr(ft), _stream()), "smfs_force_torque")
        return ft

    def eval_velocity(self, lam, x):
        n = x.numel() // 3
        self._need(lam, 3 * self.S, "lambda")
        self._need(x, 3 * n, "points")
        u = self._dvec(3 * n)
        _check(lib().smfs_eval_velocity(self.h, _ptr(lam), n, _ptr(x), _ptr(u), _stream()),
               "smfs_eval_velocity")
        return u

    @staticmethod
    def _outputs(o, rc):
        """Host statistics of a solve; status is SMFS_OK (true residual met
        the tolerance), SMFS_STAGNATED or SMFS_NOT_CONVERGED."""
        return dict(status=rc, converged=rc == SMFS_OK, stagnated=rc == SMFS_STAGNATED,
                    iterations=o.iterations, rel_residual=o.rel_residual,
                    true_rel_residual=o.true_rel_residual, lambda_inf=o.lambda_inf,
                    eps_res_max=o.eps_res_max, abs_res_max=o.abs_res_max,
                    t_rhs_ms=o.t_rhs_ms, t_gmres_ms=o.t_gmres_ms, t_post_ms=o.t_post_ms,
                    pair_evals=o.pair_evals, pair_evals_f32=o.pair_evals_f32,
                    refinements=o.refinements, true_checks=o.true_checks,
                    floor_iteration=o.floor_iteration, floor_rel_residual=o.floor_rel_residual)

    def solve_mobility(self, ft, want_check=True):
        """Forces/torques (P x 6, device) in; rigid motions out."""
        self._need(ft, 6 * self.P, "ft")
        mu, lam = self._dvec(3 * self.T), self._dvec(3 * self.S)
        ft_out, rbm = self._dvec(6 * self.P), self._dvec(6 * self.P)
        uc = self._dvec(3 * self.n_check) if (want_check and self.n_check) else None
        o = smfs_out()
        o.mu, o.lambda_, o.ft, o.rbm = mu.data_ptr(), lam.data_ptr(), ft_out.data_ptr(), rbm.data_ptr()
        o.u_check = uc.data_ptr() if uc is not None else None
        rc = lib().smfs_solve_mobility(self.h, _ptr(ft), C.byref(o), _stream())
        _check(rc, "smfs_solve_mobility", ok=SOLVE_WARNINGS)
        d = self._outputs(o, rc)
        d.update(mu=mu, lam=lam, ft=ft_out, rbm=rbm, u_check=uc)
        return d

    def solve_resistance(self, rbm, want_check=True):
        self._need(rbm, 6 * self.P, "rbm")
        mu = self._dvec(3 * self.T)
        lam = self._dvec(3 * self.S)
        ft = self._dvec(6 * self.P)
        uc = self._dvec(3 * self.n_check) if (want_check and self.n_check) else None
        o = smfs_out()
        o.mu, o.lambda_, o.ft = mu.data_ptr(), lam.data_ptr(), ft.data_ptr()
        o.u_check = uc.data_ptr() if uc is not None else None
        rc = lib().smfs_solve_resistance(self.h, _ptr(rbm), C.byref(o), _stream())
        _check(rc, "smfs_solve_resistance", ok=SOLVE_WARNINGS)
        d = self._outputs(o, rc)
        d.update(mu=mu, lam=lam, ft=ft, u_check=uc)
        return d

    # -- many right-hand sides ---------------------------------------------
    def block_workspace_bytes(self, nrhs, restart=0):
        n = C.c_size_t(0)
        _check(lib().smfs_block_workspace_bytes(self.h, nrhs, restart, C.byref(n)),
               "smfs_block_workspace_bytes")
        return int(n.value)

    def block_workspace(self, nrhs, restart=0):
        """A device buffer for the block calls (kept on the object and reused
        while large enough)."""
        import torch
        need = self.block_workspace_bytes(nrhs, restart)
        old = getattr(self, "_bws", None)
        if old is None or old.numel() - 256 < need:
            self._bws = None
            self._bws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
        base = self._bws.data_ptr()
        return (base + 255) // 256 * 256, self._bws.numel() - ((base + 255) // 256 * 256 - base)

    def apply_block(self, mu, out=None, precision=SMFS_FP64):
        """mu: (nrhs, 3T) contiguous float64 device tensor; returns G_hat mu_q per row."""
        import torch
        if mu.dim() != 2 or mu.shape[1] != 3 * self.T:
            raise ValueError("mu: expected shape (nrhs, 3T)")
        nrhs = mu.shape[0]
        self._need(mu, nrhs * 3 * self.T, "mu")
        y = out if out is not None else torch.empty_like(mu)
        self._need(y, nrhs * 3 * self.T, "y")
        ws, nb = self.block_workspace(nrhs, 0)
        _check(lib().smfs_apply_block(self.h, nrhs, _ptr(mu), _ptr(y), 3 * self.T, precision,
                                      C.c_void_p(ws), nb, _stream()), "smfs_apply_block")
        return y

    def solve_resistance_block(self, rbm, restart=100):
        """rbm: nrhs x P x 6 values (device, contiguous); returns ft (nrhs, P, 6), mu (nrhs, 3T),
        per-system iterations and true relative residuals."""
        import torch
        nrhs = rbm.numel() // (6 * self.P)
        if nrhs < 1:
            raise ValueError("rbm: expected (nrhs, P, 6) values")
        self._need(rbm, nrhs * 6 * self.P, "rbm")
        ft = torch.empty(nrhs, self.P, 6, dtype=torch.float64, device="cuda")
        mu = torch.empty(nrhs, 3 * self.T, dtype=torch.float64, device="cuda")
        its = np.zeros(nrhs, np.int32)
        tr = np.zeros(nrhs, np.float64)
        ws, nb = self.block_workspace(nrhs, restart)
        o = smfs_block_out()
        o.ft, o.mu = ft.data_ptr(), mu.data_ptr()
        o.iterations, o.true_rel_residual = its.ctypes.data, tr.ctypes.data
        rc = lib().smfs_solve_resistance_block(self.h, nrhs, _ptr(rbm), restart, C.c_void_p(ws), nb,
                                               C.byref(o), _stream())
        _check(rc, "smfs_solve_resistance_block", ok=SOLVE_WARNINGS)
        return dict(ft=ft, mu=mu, iterations=its, true_rel_residual=tr, status=rc, converged=rc == SMFS_OK,
                    max_iterations=o.max_iterations, n_converged=o.n_converged,
                    t_gmres_ms=o.t_gmres_ms, t_post_ms=o.t_post_ms, pair_evals=o.pair_evals,
                    pair_evals_f32=o.pair_evals_f32, refinements=o.refinements)


class Server:
    """Continuous-batching server of independent resistance solves (see
    smfs_server_* in include/smfs.h).  All requests share one discretisation
    (keyword overrides of smfs_params) and the sphere radius."""

    def __init__(self, radius=1.0, arena_bytes=8 << 30, max_active=64, setup_workers=1, max_queued=0,
                 server_precision=SMFS_FP64, worker_scratch_bytes=0, iters_per_step=0, setup_batch=0,
                 **over):
        """The server's device memory (its fixed part plus an arena of
        arena_bytes) is one torch allocation held by this object.
        iters_per_step: GMRES iterations per step() (0: the library's 8);
        setup_batch: most requests a set-up worker factorises together (0:
        64); the other arguments are the fields of smfs_server_config."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("smfs.Server needs a HIP device")
        torch.cuda.init()
        self.params = params_default(**over)
        cfg = smfs_server_config()
        _check(lib().smfs_server_config_default(C.byref(cfg)), "smfs_server_config_default")
        cfg.radius, cfg.max_active, cfg.setup_workers = float(radius), max_active, setup_workers
        cfg.max_queued, cfg.precision = max_queued, server_precision
        if worker_scratch_bytes:
            cfg.worker_scratch_bytes = worker_scratch_bytes
        if iters_per_step:
            cfg.iters_per_step = iters_per_step
        if setup_batch:
            cfg.setup_batch = setup_batch
        self.config = cfg
        fixed = C.c_size_t(0)
        _check(lib().smfs_server_memory_bytes(C.byref(self.params), C.byref(cfg), C.byref(fixed)),
               "smfs_server_memory_bytes")
        total = int(fixed.value) + int(arena_bytes)
        self.mem = torch.empty(total + 256, dtype=torch.uint8, device="cuda")
        base = (self.mem.data_ptr() + 255) // 256 * 256
        h = C.c_void_p()
        _check(lib().smfs_server_create(C.byref(self.params), C.byref(cfg), C.c_void_p(base), total,
                                        C.byref(h)), "smfs_server_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().smfs_server_destroy(self.h)
            self.h = None
        self.mem = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def clock():
        return lib().smfs_server_clock()

    def submit(self, centers, rbm, t_arrival=-1.0):
        c = np.ascontiguousarray(centers, np.float64).reshape(-1, 3)
        r = np.ascontiguousarray(rbm, np.float64).reshape(-1, 6)
        if r.shape[0] != c.shape[0]:
            raise ValueError("rbm must have one row of 6 per sphere")
        rid = C.c_int64()
        _check(lib().smfs_server_submit(self.h, c.shape[0], _np_ptr(c), _np_ptr(r), float(t_arrival),
                                        C.byref(rid)), "smfs_server_submit")
        return int(rid.value)

    def try_submit(self, centers, rbm, t_arrival=-1.0):
        """As submit, but None (nothing queued) when the queue is full."""
        try:
            return self.submit(centers, rbm, t_arrival)
        except SmfsError as e:
            if e.code == SMFS_E_AGAIN:
                return None
            raise

    def step(self):
        a, w = C.c_int32(), C.c_int32()
        _check(lib().smfs_server_step(self.h, C.byref(a), C.byref(w)), "smfs_server_step")
        return int(a.value), int(w.value)

    def poll(self, rid, P):
        """None while the request runs; else a dict with forces/torques (P x 6)."""
        res = smfs_request_result()
        ft = np.zeros((P, 6))
        rc = lib().smfs_server_poll(self.h, rid, C.byref(res), _np_ptr(ft))
        if rc == 1:
            return None
        _check(rc, "smfs_server_poll")
        d = {k: getattr(res, k) for k, _ in smfs_request_result._fields_}
        d["error"] = res.error.decode(errors="replace")
        d["ft"] = ft
        return d

    def release(self, rid):
        _check(lib().smfs_server_release(self.h, rid), "smfs_server_release")

    def stats(self):
        st = smfs_server_stats()
        _check(lib().smfs_server_stats_read(self.h, C.byref(st)), "smfs_server_stats_read")
        return {k: getattr(st, k) for k, _ in smfs_server_stats._fields_}

    def drain(self, timeout_s=600.0):
        """Step until nothing is resident or waiting."""
        import time
        t0 = time.perf_counter()
        while True:
            a, w = self.step()
            if a == 0 and w == 0:
                return
            if a == 0:
                time.sleep(0.0005)
            if time.perf_counter() - t0 > timeout_s:
                raise TimeoutError("server did not drain")
