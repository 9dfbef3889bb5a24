"""Host-side checks of libsmfs (no GPU needed): exported symbols, node sets
against the oracle's independent geometry, error paths."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import geometry as geo
from paper_2407_03343_amd import smfs, workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "smfs.h")).read()
    declared = set(re.findall(r"\b(smfs_[a-z_0-9]+)\s*\(", hdr))
    assert declared, "no declarations found"
    L = smfs.lib()
    for name in sorted(declared):
        assert hasattr(L, name), name
    assert declared == set(smfs.EXPORTED)


def _compare_nodes(pb, g):
    n = pb.export_nodes()
    assert n["targets"].shape == g.targets.shape
    assert n["sources"].shape == g.src_pos.shape
    assert np.abs(n["targets"] - g.targets).max() < 1e-13
    assert np.abs(n["target_weight"] - g.target_weight).max() < 1e-15
    assert np.abs(n["sources"] - g.src_pos).max() < 1e-13
    assert np.abs(n["check"] - g.check).max() < 1e-13
    assert (n["source_kind"] == g.src_kind).all()
    assert (n["source_sphere"] == g.src_sphere).all()
    assert (n["target_sphere"] == g.target_sphere).all()
    assert (n["check_sphere"] == g.check_sphere).all()


def test_nodes_match_oracle_two_spheres():
    pk, _ = wl.workload_two_sphere_gap001()
    pb = smfs.Problem(pk.centers, 1.0)
    _compare_nodes(pb, geo.build(pk.centers, 1.0))
    assert pb.T == 3000 and pb.S == 1320


@pytest.mark.parametrize("kinds,mask", [("S", smfs.KIND_S), ("SR", smfs.KIND_S | smfs.KIND_R),
                                        ("SRD", 7)])
def test_nodes_match_oracle_cluster(kinds, mask):
    pk = wl.cluster(12, 0.1, 1e-3, 1e-1, seed=3)
    prm = geo.Params(kinds=kinds, n_image=-1)
    pb = smfs.Problem(pk.centers, 1.0, image_kinds=mask, n_image=-1)
    g = geo.build(pk.centers, 1.0, prm)
    _compare_nodes(pb, g)
    pairs = sum(g.M(k) * (g.S - g.Nk(k)) for k in range(g.P))
    assert pb.pairs_per_apply == pairs


def test_nodes_match_oracle_full_cluster():
    pk, _ = wl.workload_cluster100(0)
    pb = smfs.Problem(pk.centers, 1.0)
    _compare_nodes(pb, geo.build(pk.centers, 1.0))


def test_overlap_and_unequal_radii_rejected():
    L = smfs.lib()
    p = smfs.params_default()
    h = C.c_void_p()
    c = np.array([[0.0, 0, 0], [1.5, 0, 0]])
    r = np.ones(2)
    rc = L.smfs_problem_create(C.byref(p), 2, c.ctypes.data_as(C.c_void_p),
                               r.ctypes.data_as(C.c_void_p), C.byref(h))
    assert rc == -2
    c = np.array([[0.0, 0, 0], [5.0, 0, 0]])
    r = np.array([1.0, 1.1])
    rc = L.smfs_problem_create(C.byref(p), 2, c.ctypes.data_as(C.c_void_p),
                               r.ctypes.data_as(C.c_void_p), C.byref(h))
    assert rc == -3
    c = np.array([[0.0, 0, 0], [np.nan, 0, 0]])
    r = np.ones(2)
    rc = L.smfs_problem_create(C.byref(p), 2, c.ctypes.data_as(C.c_void_p),
                               r.ctypes.data_as(C.c_void_p), C.byref(h))
    assert rc == -1
    # an FP64 class wider than the image cutoff is not supported
    p2 = smfs.params_default(near_gap_cutoff=0.3)
    c = np.array([[0.0, 0, 0], [5.0, 0, 0]])
    rc = L.smfs_problem_create(C.byref(p2), 2, c.ctypes.data_as(C.c_void_p),
                               r.ctypes.data_as(C.c_void_p), C.byref(h))
    assert rc == -3 and "near_gap_cutoff" in L.smfs_last_error().decode()


def test_small_gap_warning_and_state_errors():
    pb = smfs.Problem(np.array([[0.0, 0, 0], [2.0005, 0, 0]]), 1.0)
    assert pb.gap_warning
    L = smfs.lib()
    # workspace too small: rejected before any device access
    rc = L.smfs_bind(pb.h, C.c_void_p(256), 1024, None)
    assert rc == -4
    # apply before bind/setup
    rc = L.smfs_apply(pb.h, C.c_void_p(256), C.c_void_p(512), 0, None)
    assert rc == -7
    assert "not bound" in L.smfs_last_error().decode()


def test_contact_free_spheres_share_one_factor():
    c = np.array([[0.0, 0, 0], [5.0, 0, 0], [0, 5.0, 0], [2.01, 0, 0]])
    pb = smfs.Problem(c, 1.0)
    fids = [pb.sphere_factor(k) for k in range(4)]
    assert fids[1] == fids[2] == 0
    assert fids[0] != 0 and fids[3] != 0 and fids[0] != fids[3]
    info = pb.factor_info(0)
    assert info["rows"] == 3 * 780 and info["cols"] == 3 * 600


def test_set_background_validation():
    """Background flow (eq. bc): a linear flow must be trace-free and
    finite; both arguments absent restore the quiescent fluid."""
    pb = smfs.Problem(np.array([[0.0, 0, 0], [2.5, 0, 0]]), 1.0)
    shear = np.array([[0.0, 5.0, 0], [0, 0, 0], [0, 0, 0]])
    pb.set_background(U=[5.0, 0, 0])
    pb.set_background(L=shear)
    pb.set_background(U=[1.0, -2.0, 0.5], L=shear)
    pb.set_background()
    with pytest.raises(smfs.SmfsError):
        pb.set_background(L=np.diag([1.0, 1.0, 0.0]))          # divergence 2
    with pytest.raises(smfs.SmfsError):
        pb.set_background(U=[np.nan, 0.0, 0.0])
    L = smfs.lib()
    assert L.smfs_set_background(None, None, None) != 0


def test_server_memory_query():
    """The server's fixed device memory (host-side sizing): the shared
    factor, per-slot buffers and each worker's scratch; bad settings and
    unsupported precisions are refused."""
    p = smfs.params_default(n_proxy=60, n_colloc_base=80, n_image=4, n_check_base=0)
    cfg = smfs.smfs_server_config()
    assert smfs.lib().smfs_server_config_default(C.byref(cfg)) == 0
    assert cfg.max_active == 64 and cfg.setup_workers == 1 and cfg.worker_scratch_bytes == 4 << 30
    assert cfg.iters_per_step == 8 and cfg.setup_batch == 64
    n = C.c_size_t(0)
    assert smfs.lib().smfs_server_memory_bytes(C.byref(p), C.byref(cfg), C.byref(n)) == 0
    one = n.value
    assert one > cfg.worker_scratch_bytes
    cfg.setup_workers = 3
    assert smfs.lib().smfs_server_memory_bytes(C.byref(p), C.byref(cfg), C.byref(n)) == 0
    assert n.value - one == 2 * (4 << 30)
    cfg.precision = smfs.SMFS_MIXED
    assert smfs.lib().smfs_server_memory_bytes(C.byref(p), C.byref(cfg), C.byref(n)) == -3
    cfg.precision = smfs.SMFS_MIXED_FAR
    assert smfs.lib().smfs_server_memory_bytes(C.byref(p), C.byref(cfg), C.byref(n)) == 0
    cfg.iters_per_step = 2000
    assert smfs.lib().smfs_server_memory_bytes(C.byref(p), C.byref(cfg), C.byref(n)) == -1
    cfg.iters_per_step = 8
    cfg.setup_batch = 65
    assert smfs.lib().smfs_server_memory_bytes(C.byref(p), C.byref(cfg), C.byref(n)) == -1
    cfg.setup_batch = 0
    cfg.max_active = 0
    assert smfs.lib().smfs_server_memory_bytes(C.byref(p), C.byref(cfg), C.byref(n)) == -1


def test_far_field_near_lists_and_pair_counts():
    """The library's near lists of the equivalent-source far field (host
    tables, no GPU) against the oracle's classification of far pairs on a
    lattice with near and far pairs and one contact pair."""
    from oracle import farfield as ff, geometry as geo
    cs = np.array([[i * 3.2, j * 3.2, k * 3.2] for i in range(2) for j in range(3) for k in range(2)]
                  + [[0.0, 0.0, -2.01]])
    g = geo.build(cs, 1.0)
    ep = ff.EqParams()
    pb = smfs.Problem(cs, 1.0)
    s = pb.sizes
    near = far = 0
    for k in range(g.P):
        for ks in range(g.P):
            if ks == k or not g.contact_free(ks):
                continue
            if ff.is_far(g, ep, k, ks):
                far += g.M(k) * ep.n_eq
            else:
                near += 1
    assert s.eq_near_spheres == near
    assert s.eq_far_pairs == far
    # exact pairs: every pair but the far proxies
    far_proxy = far // ep.n_eq * g.params.n_proxy
    assert s.eq_exact_pairs == pb.pairs_per_apply - far_proxy
    # the form is off without contact-free spheres or with eq_points = 0
    assert smfs.Problem(cs, 1.0, eq_points=0).sizes.eq_far_pairs == 0
    with pytest.raises(smfs.SmfsError):
        smfs.Problem(cs, 1.0, eq_separation=3.0)     # below eq_check_radius + 1


def test_out_of_reach_slot_adds_exactly_zero():
    """The FP32 equivalent-source sum moves a slot that must skip a source
    sphere to 1e20 instead of masking it.  In IEEE single precision the
    squared distance then overflows to +inf, 1/sqrt(inf) is +0, the
    projection r.f stays finite for strengths below 1e18, and the pair
    (f + r (r.f) / r^2) / r adds exactly zero to the accumulator."""
    f32 = np.float32
    rng = np.random.default_rng(3)
    with np.errstate(over="ignore"):
        for _ in range(200):
            s = rng.uniform(-1.0, 1.0, 3).astype(f32)           # equivalent point (radius 1)
            f = (rng.standard_normal(3) * 10.0 ** rng.uniform(-3, 17)).astype(f32)
            acc = rng.standard_normal(3).astype(f32)
            r = (np.full(3, 1e20, f32) - s).astype(f32)
            r2 = f32(r[0] * r[0] + r[1] * r[1] + r[2] * r[2])
            assert np.isinf(r2)
            ri = f32(1.0) / np.sqrt(r2)
            assert ri == 0.0
            rf = f32(r[0] * f[0] + r[1] * f[1] + r[2] * f[2])
            assert np.isfinite(rf)
            t = f32(rf * f32(ri * ri))
            new = (acc + (f + r * t) * ri).astype(f32)
            assert np.array_equal(new, acc)


def test_binding_fails_loudly_without_the_library(tmp_path):
    """No CPU fallback: with the shared library absent the binding raises on
    first use (run in a child process so the loaded library of this one is
    not disturbed)."""
    import subprocess
    import sys
    code = ("from paper_2407_03343_amd import smfs\n"
            "try:\n    smfs.lib()\nexcept RuntimeError as e:\n    print('raised:', e)\n")
    env = dict(os.environ, SMFS_LIB=str(tmp_path / "absent" / "libsmfs.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=120,
                       cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))), env=env)
    assert r.returncode == 0 and "raised:" in r.stdout and "missing" in r.stdout


def _imports(path):
    """Module names a Python file imports, with the function they sit in
    (None at module level)."""
    import ast
    tree = ast.parse(open(path).read())
    out = []

    def visit(node, fn):
        for ch in ast.iter_child_nodes(node):
            f = ch.name if isinstance(ch, (ast.FunctionDef, ast.AsyncFunctionDef)) else fn
            if isinstance(ch, ast.Import):
                out.extend((a.name, fn) for a in ch.names)
            elif isinstance(ch, ast.ImportFrom):
                out.append(("." * ch.level + (ch.module or ""), fn))
            visit(ch, f)
    visit(tree, None)
    return out


def test_oracle_and_product_share_no_code():
    """The oracle and the library are independent: no product file imports
    or includes anything under oracle/, the oracle imports nothing from the
    package, the input generators hold no import of either side's
    arithmetic, and the benchmark touches the oracle only inside its CPU
    baseline."""
    import glob
    pkg = os.path.join(ROOT, "paper_2407_03343_amd")
    for f in glob.glob(os.path.join(pkg, "*.py")):
        for mod, _ in _imports(f):
            assert not mod.startswith("oracle"), (f, mod)
    for f in glob.glob(os.path.join(pkg, "csrc", "*")):
        for line in open(f, errors="replace"):
            if line.lstrip().startswith("#include"):
                assert "oracle" not in line, (f, line)
    for f in glob.glob(os.path.join(ROOT, "oracle", "*.py")):
        for mod, _ in _imports(f):
            assert "paper_2407_03343_amd" not in mod, (f, mod)
    for mod, _ in _imports(os.path.join(pkg, "workloads.py")):
        assert mod.split(".")[0] in ("__future__", "math", "dataclasses", "numpy"), mod
    for mod, fn in _imports(os.path.join(ROOT, "bench.py")):
        if mod.startswith("oracle"):
            assert fn == "cpu_baseline", (mod, fn)


def test_header_cites_the_paper_for_every_operation():
    """Each entry point that computes a step of the method carries a
    citation of the passage it follows in its own comment; the serving calls
    under their section's comment; the allocation-free variant names the
    callers it is for.  Housekeeping calls (defaults, sizes, workspace
    queries, profiling, errors) need none."""
    src = open(os.path.join(ROOT, "include", "smfs.h")).read()
    cite = re.compile(r"Section|eq\.|Remark|Appendix|Table|Figure|Example")
    own, section = {}, {}
    last, sec = "", ""
    for m in re.finditer(r"/\*.*?\*/|^[A-Za-z][^;{}]*?\b(smfs_\w+)\s*\([^;]*?\);", src, re.S | re.M):
        t = m.group(0)
        if t.startswith("/*"):
            last = t
            if t.startswith("/* ----"):
                sec = t
        else:
            own[m.group(1)], section[m.group(1)] = last, sec
    operations = ["smfs_problem_create", "smfs_export_nodes", "smfs_sphere_factor", "smfs_setup",
                  "smfs_setup_far_field", "smfs_import_factor", "smfs_apply", "smfs_transform", "smfs_rhs",
                  "smfs_set_background", "smfs_force_torque", "smfs_eval_velocity", "smfs_solve_resistance",
                  "smfs_solve_mobility", "smfs_apply_block", "smfs_solve_resistance_block"]
    for name in operations:
        assert cite.search(own[name]), name
    for name in ("smfs_server_create", "smfs_server_submit", "smfs_server_step", "smfs_server_poll"):
        assert cite.search(section[name]), name
    assert "cannot allocate" in own["smfs_apply_block_noalloc"]
