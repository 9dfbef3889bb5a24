#!/usr/bin/env python
"""Benchmark of the one-body preconditioned MFS product on one MI355X.

Headline workload: 2000 unit spheres in a cube at volume fraction 0.3 (a
hard-sphere fluid with every gap at least 0.2), 5% of them pulled into
near-contact pairs at gaps log-uniform in [1e-3, 1e-2]; 600 proxy
Stokeslets on R_p = 0.7, 780 base collocation nodes, 20 image nodes (S, R,
D) per contact with gap < 0.2, two caps of 360 nodes per contact.  The
self-block set-up (geometry, device assembly, truncated SVD of every
distinct self block) runs before the timed region and is reported apart.

A step is one product y = G_hat mu with the one-body preconditioned
operator (Section 2.2, eq. resistance) in FP64: the pseudo-inverse of every
sphere's self block applied to its slice of mu (eq. transform), the sum of
every off-sphere Stokeslet, rotlet and dipole pair (eq. uAll) and the
identity self blocks.  This product is what every GMRES iteration of a
solve repeats.  `value` = pair evaluations of the timed products / wall
time.  The same products in the mixed forms are timed beside it, with
their error against FP64: SMFS_MIXED (FP32 sources of the contact-free
spheres) and SMFS_MIXED_EQ (the far field of the contact-free spheres
through FP64-fitted equivalent Stokeslets summed in FP32).

Sections of the default run, each inside the wall budget (--budget-s):
 * cpu_baseline: the oracle's C direct sum on a bounded sample of the same
   workload;
 * solve: solve time to 1e-3 relative surface velocity (and 1e-5 in
   forces/torques), FP64 against SMFS_MIXED_EQ (the other mixed forms on
   request), p50/p99 over repeated solves, on a 200-sphere cut of the same
   recipe;
 * two_sphere: the two-sphere case at gap 0.01, p50/p99 of complete solves.
Flags add the block product, the block solve, the serving stream and the
set-up comparison; their results go to stderr and, with --sections-out, to
a JSON file.  stdout carries exactly one JSON line.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_VALU_TFLOPS = 78.6      # MI355X, FP64 vector
PEAK_FP64_MFMA_TFLOPS = 78.6      # MI355X, FP64 dense matrix
PEAK_FP32_VALU_TFLOPS = 157.3     # MI355X, FP32 vector
PEAK_HBM_GBS = 8000.0
# HBM bytes per launch of the FP64 direct sum on the headline workload, from
# rocprofv3 FETCH_SIZE (x2, the factor a plain 1 GiB elementwise product
# reads back) plus WRITE_SIZE (x1), KiB per dispatch, as recorded in the
# counter summary of this kernel and workload under profiles/; None until
# counters of the current kernel on this workload are taken.
DIRECT_TRAFFIC_BYTES = (2 * 6230207.7 + 422606.2) * 1024

# SMFS_FP64, SMFS_MIXED_EQ, SMFS_MIXED, SMFS_MIXED_FAR
FORMS = (("fp64", 0), ("mixed_eq", 3), ("mixed", 1), ("mixed_far", 2))


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class Budget:
    """Wall-clock budget of the whole run: a section starts only when its
    estimated cost still fits."""

    def __init__(self, seconds):
        self.t0 = time.perf_counter()
        self.seconds = seconds

    def left(self):
        return self.seconds - (time.perf_counter() - self.t0)

    def fits(self, need_s):
        return self.left() > need_s


def host_info():
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        import psutil
        phys = psutil.cpu_count(logical=False)
    except Exception:
        phys = None
    return dict(cpu=model, logical_cpus=os.cpu_count(), physical_cores=phys,
                hostname=platform.node())


# ---------------------------------------------------------------------------
# Headline: FP64 products on the 2000-sphere packing, mixed beside them


def offdiag_err(y, y_ref, mu):
    """Max-norm error of the off-diagonal part (y - mu) relative to the
    largest entry of the reference's off-diagonal part (mu is copied
    exactly and would dilute the comparison)."""
    a = y - mu
    b = y_ref - mu
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def timed_products(pb, torch, mu, y, precision, warmup, steps):
    for _ in range(warmup):
        pb.apply(mu, precision=precision, out=y)
    torch.cuda.synchronize()
    pb.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pb.apply(mu, precision=precision, out=y)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    pb.profile(False)
    return elapsed, pb.profile_read()


def headline(args, torch, smfs, wl, budget):
    pk = wl.workload_packing2000(args.spheres, seed=args.seed)
    gaps = pk.min_gaps()
    log(f"workload: {pk.P} spheres, box {pk.box:.2f}, {int((gaps < 0.2).sum())} in near contact, "
        f"min gap {gaps.min():.2e}")
    svd = smfs.SMFS_SVD_JACOBI if args.svd == "jacobi" else smfs.SMFS_SVD_ROCSOLVER
    pb = smfs.Problem(pk.centers, pk.radius, gmres_restart=1, svd_method=svd)
    log(f"T={pb.T} S={pb.S} factors={pb.sizes.n_factors} workspace="
        f"{pb.sizes.workspace_bytes / 2**30:.2f} GiB pairs/apply={pb.pairs_per_apply:.4e}")
    pb.bind()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pb.setup()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    ranks = sorted({pb.factor_info(f)["rank"] for f in range(pb.sizes.n_factors)
                    if pb.factor_info(f)["sphere"] >= 0})
    log(f"setup (device assembly + truncated SVD of {pb.sizes.n_factors} distinct self blocks): "
        f"{setup_s:.1f} s ({args.svd}, {pb.sizes.svd_sweeps} Jacobi sweeps), ranks {ranks[0]}..{ranks[-1]}")

    rbm = torch.from_numpy(wl.random_rbm(pb.P, 1, 1000 + args.seed)[0].reshape(-1)).cuda()
    b = pb.rhs(rbm)                                      # a physical vector (first Krylov vector)
    mu = torch.from_numpy(wl.random_vector(3 * pb.T, 3 + args.seed)).cuda()   # rough, like later ones
    y = torch.empty_like(mu)

    elapsed, st = timed_products(pb, torch, mu, y, smfs.SMFS_FP64, args.warmup, args.steps)
    pairs = pb.pairs_per_apply * args.steps
    direct_avg_s = st["direct_ms"] / max(1, st["direct_launches"]) * 1e-3
    pinv_avg_s = st["pinv_ms"] / max(1, st["pinv_launches"]) * 1e-3
    achieved = st["direct_flops"] / direct_avg_s / 1e12
    log(f"FP64 product: {elapsed / args.steps * 1e3:.1f} ms per step, direct sum "
        f"{direct_avg_s * 1e3:.1f} ms ({achieved:.1f} TFLOP/s), pseudo-inverse {pinv_avg_s * 1e3:.2f} ms")

    if args.no_mixed:
        return pk, pb, headline_result(args, pk, pb, elapsed, st, setup_s, ranks, None)
    # mixed form: the same products, then its error against FP64
    m_el, m_st = timed_products(pb, torch, mu, y, smfs.SMFS_MIXED, min(args.warmup, 2), args.steps)
    errs = {}
    for name, vec in (("physical", b), ("random", mu)):
        y64 = pb.apply(vec, precision=smfs.SMFS_FP64).cpu().numpy()
        v = vec.cpu().numpy()
        errs[name] = {f: offdiag_err(pb.apply(vec, precision=p).cpu().numpy(), y64, v)
                      for f, p in FORMS[1:]}
    log(f"mixed product: {m_el / args.steps * 1e3:.1f} ms per step ({elapsed / m_el:.2f}x FP64); "
        f"error vs FP64 (off-diagonal, max-norm): physical {errs['physical']}, random {errs['random']}")
    e_el, e_st = timed_products(pb, torch, mu, y, smfs.SMFS_MIXED_EQ, min(args.warmup, 2), args.steps)
    s = pb.sizes
    log(f"equivalent-source product: {e_el / args.steps * 1e3:.1f} ms per step ({elapsed / e_el:.2f}x FP64), "
        f"far FP32 {e_st['eq_far_ms'] / max(1, e_st['eq_launches']):.1f} ms, near FP64 "
        f"{e_st['eq_near_ms'] / max(1, e_st['eq_launches']):.1f} ms, contact sources FP64 "
        f"{e_st['mixed64_ms'] / max(1, e_st['mixed64_launches']):.1f} ms, strengths "
        f"{e_st['eq_strength_ms'] / max(1, e_st['eq_launches']):.2f} ms")
    mixed = {
        "precision": "SMFS_MIXED: FP32 pseudo-inverse and far field for the contact-free spheres",
        "ms_per_step": m_el / args.steps * 1e3,
        "pair_evals_per_s": pb.pairs_per_apply * args.steps / m_el,
        "speedup_over_fp64": elapsed / m_el,
        "kernels": mixed_kernel_rates(m_st),
        "offdiag_rel_err_vs_fp64": errs,
        "equivalent_sources": {
            "precision": "SMFS_MIXED_EQ: far field of contact-free spheres through 200 equivalent "
                         "Stokeslets fitted in FP64, summed in FP32; pairs closer than 3.5 radii "
                         "between centres and every contact-sphere source exact in FP64",
            "ms_per_step": e_el / args.steps * 1e3,
            "speedup_over_fp64": elapsed / e_el,
            "equivalent_pairs": int(s.eq_far_pairs),
            "exact_pairs": int(s.eq_exact_pairs),
            "near_list_entries": int(s.eq_near_spheres),
            "kernels": mixed_kernel_rates(e_st),
            "strength_ms": e_st["eq_strength_ms"] / max(1, e_st["eq_launches"]),
        },
    }
    return pk, pb, headline_result(args, pk, pb, elapsed, st, setup_s, ranks, mixed)


def headline_result(args, pk, pb, elapsed, st, setup_s, ranks, mixed):
    pairs = pb.pairs_per_apply * args.steps
    direct_avg_s = st["direct_ms"] / max(1, st["direct_launches"]) * 1e-3
    pinv_avg_s = st["pinv_ms"] / max(1, st["pinv_launches"]) * 1e-3
    achieved = st["direct_flops"] / direct_avg_s / 1e12
    result = {
        "metric": "Stokeslet pair-evals/s (one-body preconditioned product G_hat mu, FP64, "
                  "2000-sphere packing); solve time at 1e-3 relative surface velocity, mixed vs FP64, "
                  "p50/p99",
        "value": pairs / elapsed,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded packing and rigid motions; random-vector products)",
        "config": {
            "workload": f"{pk.P} unit spheres, cube at volume fraction 0.3 (hard-sphere fluid, gaps >= 0.2), "
                        "5% in near-contact pairs at gaps log-uniform [1e-3, 1e-2]; N=600 proxy Stokeslets "
                        "on R_p=0.7, 780 base nodes, 20 S+R+D image nodes per contact (gap < 0.2), caps "
                        "2x360; truncated-SVD factors (5e-12) set up before the timed region; one FP64 "
                        "product with G_hat per step",
            "spheres": pk.P, "collocation_nodes": pb.T, "sources": pb.S,
            "distinct_self_blocks": pb.sizes.n_factors, "pairs_per_apply": pb.pairs_per_apply,
            "precision": "fp64",
        },
        "setup_s": setup_s,
        "setup_svd": args.svd,
        "setup_jacobi_sweeps": int(pb.sizes.svd_sweeps),
        "factor_ranks": [int(ranks[0]), int(ranks[-1])],
        "roofline": {
            "kernel": "k_direct_f64 (direct sum of every off-sphere pair)",
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_VALU_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_VALU_TFLOPS,
            "traffic": DIRECT_TRAFFIC_BYTES,
            "traffic_unit": "bytes per launch",
            "avg_launch_ms": direct_avg_s * 1e3,
            "launches": st["direct_launches"],
            "flops_per_launch": st["direct_flops"],
            "work_per_unit": "28 / 25 / 30 flops per Stokeslet / rotlet / dipole pair",
        },
        "pinv_apply": {
            "kernel": "k_pinv_u + k_pinv_v (contact spheres) + k_pinv_shared_u/v (FP64 MFMA, shared factor)",
            "bound": "hbm",
            "achieved": st["pinv_bytes"] / pinv_avg_s / 1e9 if pinv_avg_s > 0 else None,
            "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "avg_launch_ms": pinv_avg_s * 1e3, "bytes_per_launch": st["pinv_bytes"],
        },
    }
    if mixed is not None:
        result["mixed"] = mixed
    return result


def mixed_kernel_rates(st):
    """Per-kernel rates over the profiled products of one form: the FP32 far
    field against the FP32 vector peak, the FP64 direct sum (all of the sum
    in the FP64 form, the near part in the mixed forms) against the FP64
    vector peak."""
    out = {}
    for key, label, peak in (("far32", "k_far_f32", PEAK_FP32_VALU_TFLOPS),
                             ("mixed64", "k_direct_f64 (near part)", PEAK_FP64_VALU_TFLOPS),
                             ("direct", "k_direct_f64", PEAK_FP64_VALU_TFLOPS),
                             ("eq_far", "k_far_eq_f32 (equivalent sources)", PEAK_FP32_VALU_TFLOPS),
                             ("eq_near", "k_near_f64 (near contact-free proxies)", PEAK_FP64_VALU_TFLOPS)):
        n = st.get("eq_launches", 0) if key.startswith("eq_") else st[f"{key}_launches"]
        if not n:
            continue
        ms = st[f"{key}_ms"] / n
        tf = st[f"{key}_flops"] / (ms * 1e-3) / 1e12
        out[key] = dict(kernel=label, launches=n, avg_launch_ms=ms,
                        flops_per_launch=st[f"{key}_flops"], achieved=tf, peak=peak,
                        unit="TFLOP/s", frac=tf / peak)
    return out


# ---------------------------------------------------------------------------
# CPU baseline: the oracle's direct sum on a bounded sample


def cpu_baseline(pk, seconds: float):
    """The FP64 oracle's direct sum (its dominant step) over every stride-th
    collocation node of the same workload against all sources, same-sphere
    pairs skipped; the stride is chosen from a short probe so that the timed
    sample takes about `seconds`."""
    from oracle import geometry as geo
    from oracle.pairsum import pairsum, build
    build(force=False)
    t0 = time.perf_counter()
    g = geo.build(pk.centers, pk.radius)
    geo_s = time.perf_counter() - t0
    own = np.bincount(g.src_sphere, minlength=g.P)
    lam = np.random.default_rng(7).standard_normal((g.S, 3))

    def run(stride):
        rows = np.arange(0, g.T, stride)
        t = time.perf_counter()
        pairsum(g.targets[rows], g.src_pos, g.src_kind, lam, 1.0, g.target_sphere[rows], g.src_sphere, True)
        dt = time.perf_counter() - t
        return rows, dt, float(np.sum(g.S - own[g.target_sphere[rows]]))

    rows, dt, pairs = run(max(1, g.T // 256))             # probe
    rate = pairs / dt
    stride = max(1, int(g.T * g.S / (rate * seconds)))
    rows, dt, pairs = run(stride)
    threads = int(os.environ.get("OMP_NUM_THREADS") or (os.cpu_count() or 1))
    return dict(value=pairs / dt, unit="pair-evals/s", cores=threads, kind="oracle",
                host=host_info(),
                sample=(f"oracle C direct sum (FP64, OpenMP, {threads} threads), {rows.size} of {g.T} "
                        f"collocation nodes (every {stride}) x {g.S} sources of the same workload, "
                        f"same-sphere pairs skipped: {pairs:.3g} pairs in {dt:.1f} s "
                        f"(oracle geometry built in {geo_s:.1f} s, not timed)"))


# ---------------------------------------------------------------------------
# Solve time at 1e-3 surface velocity, FP64 against the mixed forms


def solve_section(args, torch, smfs, wl, budget):
    """Resistance solves on a cut of the headline recipe: the reference is
    the FP64 solve at tolerance 1e-10 (ending on its true-residual floor);
    for every form, the GMRES tolerances of a ladder are tried from the
    loosest until the check-point velocities are within 1e-3 of the
    reference (relative to the largest) and the forces and torques within
    1e-5; that tolerance is then solved `solve_reps` times for p50/p99."""
    pk = wl.workload_packing2000(args.solve_spheres, seed=args.seed)
    pb = smfs.Problem(pk.centers, pk.radius, gmres_restart=args.solve_restart,
                      gmres_max_it=args.solve_restart)
    pb.bind()
    t0 = time.perf_counter()
    pb.setup()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    rbm = torch.from_numpy(wl.random_rbm(pb.P, 1, 77)[0].reshape(-1)).cuda()
    pb.set_solver(smfs.SMFS_FP64, 1e-10)
    t1 = time.perf_counter()
    ref = pb.solve_resistance(rbm)
    torch.cuda.synchronize()
    ref_s = time.perf_counter() - t1
    u_ref, ft_ref = ref["u_check"].cpu().numpy(), ref["ft"].cpu().numpy()
    log(f"solve section: {pb.P} spheres, T={pb.T}, S={pb.S}, setup {setup_s:.1f} s; reference "
        f"{ref['iterations']} it (status {ref['status']}, true {ref['true_rel_residual']:.2e}, floor at "
        f"{ref['floor_iteration']}), {ref_s:.1f} s")
    out = {"workload": f"{pb.P}-sphere cut of the headline recipe (volume fraction 0.3, 5% in pairs)",
           "spheres": pb.P, "collocation_nodes": pb.T, "sources": pb.S,
           "pairs_per_apply": pb.pairs_per_apply, "setup_s": setup_s,
           "gates": {"u_check_rel": 1e-3, "force_torque_rel": 1e-5},
           "reference": dict(tol=1e-10, iterations=ref["iterations"], status=ref["status"],
                             true_rel_residual=ref["true_rel_residual"],
                             floor_iteration=ref["floor_iteration"], solve_s=ref_s,
                             eps_res_max=ref["eps_res_max"]),
           "forms": {}}
    last_s = ref_s
    # first the tolerance ladder of every form, then the repeated solves at
    # the chosen tolerances, so that every form gets its ladder
    chosen_of = {}
    for name, prec in FORMS:
        if name not in args.solve_forms:
            continue
        rows, chosen = [], None
        for tol in args.solve_tols:
            if not budget.fits(2.5 * last_s + args.reserve_s):
                log(f"  {name}: wall budget reached, ladder stopped")
                break
            pb.set_solver(prec, tol)
            t1 = time.perf_counter()
            o = pb.solve_resistance(rbm)
            torch.cuda.synchronize()
            last_s = time.perf_counter() - t1
            du = float(np.abs(o["u_check"].cpu().numpy() - u_ref).max() / np.abs(u_ref).max())
            dft = float(np.abs(o["ft"].cpu().numpy() - ft_ref).max() / np.abs(ft_ref).max())
            r = dict(tol=tol, iterations=o["iterations"], refinements=o["refinements"], status=o["status"],
                     solve_ms=last_s * 1e3, u_rel_err=du, ft_rel_err=dft,
                     true_rel_residual=o["true_rel_residual"], pair_evals=o["pair_evals"],
                     pair_evals_f32=o["pair_evals_f32"])
            rows.append(r)
            log(f"  {name} tol {tol:.0e}: it {o['iterations']} (+{o['refinements']}), {last_s * 1e3:.0f} ms, "
                f"u err {du:.2e}, F/T err {dft:.2e}, status {o['status']}")
            if du <= 1e-3 and dft <= 1e-5:
                chosen = r
                break
        out["forms"][name] = {"ladder": rows, "at_gates": None}
        if chosen is not None:
            chosen_of[name] = (prec, chosen)
    for name, (prec, chosen) in chosen_of.items():
        ts = [chosen["solve_ms"]]
        pb.set_solver(prec, chosen["tol"])
        for _ in range(args.solve_reps - 1):
            if not budget.fits(1.5 * chosen["solve_ms"] * 1e-3 + args.reserve_s):
                break
            t1 = time.perf_counter()
            pb.solve_resistance(rbm)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t1) * 1e3)
        out["forms"][name]["at_gates"] = dict(
            chosen, solves=len(ts), solve_ms_p50=float(np.percentile(ts, 50)),
            solve_ms_p99=float(np.percentile(ts, 99)),
            pair_evals_per_s=chosen["pair_evals"] / (np.percentile(ts, 50) * 1e-3))
        log(f"  {name} at the gates (tol {chosen['tol']:.0e}): p50 {np.percentile(ts, 50):.0f} ms, "
            f"p99 {np.percentile(ts, 99):.0f} ms over {len(ts)} solves")
    f64 = out["forms"].get("fp64", {}).get("at_gates")
    for name, _ in FORMS[1:]:
        mx = out["forms"].get(name, {}).get("at_gates")
        out[f"speedup_{name}_over_fp64"] = (f64["solve_ms_p50"] / mx["solve_ms_p50"]) if (f64 and mx) else None
    return out


def two_sphere(args, torch, smfs, wl, budget):
    """The paper's two-sphere case (Section 5, the comparison with Brenner's
    series): unit spheres at gap 0.01 moving apart at unit relative speed,
    FP64, GMRES to 1e-10 (ending on the true-residual floor).  Set-up once
    (timed), then repeated complete solves (right-hand side, GMRES,
    back-transform, forces and torques, check-point velocities) for
    p50/p99."""
    pk, rbm = wl.workload_two_sphere_gap001()
    pb = smfs.Problem(pk.centers, pk.radius)
    pb.bind()
    t0 = time.perf_counter()
    pb.setup()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    r = torch.from_numpy(rbm[0].reshape(-1)).cuda()
    o = pb.solve_resistance(r)                     # warm-up
    torch.cuda.synchronize()
    ts, pairs = [], 0
    for _ in range(args.two_sphere_reps):
        if not budget.fits(args.reserve_s):
            break
        t1 = time.perf_counter()
        o = pb.solve_resistance(r)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t1) * 1e3)
        pairs += o["pair_evals"]
    ft = o["ft"].cpu().numpy().reshape(-1, 6)
    out = dict(spheres=2, gap=0.01, collocation_nodes=pb.T, sources=pb.S, setup_s=setup_s,
               reps=len(ts), solve_ms_p50=float(np.percentile(ts, 50)),
               solve_ms_p99=float(np.percentile(ts, 99)), iterations=o["iterations"],
               status=o["status"], floor_iteration=o["floor_iteration"],
               true_rel_residual=o["true_rel_residual"], eps_res_max=o["eps_res_max"],
               force_sphere0=[float(x) for x in ft[0, :3]],
               pair_evals_per_s=pairs / (sum(ts) * 1e-3))
    log(f"two spheres, gap 0.01: setup {setup_s:.2f} s, solve p50 {out['solve_ms_p50']:.2f} ms "
        f"p99 {out['solve_ms_p99']:.2f} ms, it {o['iterations']} (floor at {o['floor_iteration']}), "
        f"|F| {np.linalg.norm(ft[0, :3]):.6f}")
    return out


# ---------------------------------------------------------------------------
# Optional sections (flags)


def block_vs_single(pb, torch, nrhs: int, reps: int, seed: int = 7):
    """Block product of nrhs vectors against nrhs single products on the
    same problem and factors: per-kernel event timing of both forms."""
    n = 3 * pb.T
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    M = torch.randn(nrhs, n, dtype=torch.float64, device="cuda", generator=g)
    Y = torch.empty_like(M)
    pb.apply_block(M, out=Y)                       # warm-up (workspace, code load)
    for q in range(nrhs):
        pb.apply(M[q], out=Y[q])
    torch.cuda.synchronize()
    pb.profile(True)
    t0 = time.perf_counter()
    for _ in range(reps):
        pb.apply_block(M, out=Y)
    torch.cuda.synchronize()
    t_block = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        for q in range(nrhs):
            pb.apply(M[q], out=Y[q])
    torch.cuda.synchronize()
    t_single = (time.perf_counter() - t0) / reps
    pb.profile(False)
    st = pb.profile_read()
    bd_s = st["bdirect_ms"] / max(1, st["bdirect_launches"]) * 1e-3
    bp_s = st["bpinv_ms"] / max(1, st["bpinv_launches"]) * 1e-3
    d_s = st["direct_ms"] / max(1, st["direct_launches"]) * 1e-3
    p_s = st["pinv_ms"] / max(1, st["pinv_launches"]) * 1e-3
    pair_rhs = pb.pairs_per_apply * nrhs
    return {
        "nrhs": nrhs,
        "block_apply_ms": t_block * 1e3,
        "single_applies_ms": t_single * 1e3,
        "speedup_block_over_single": t_single / t_block,
        "block_pair_rhs_evals_per_s": pair_rhs / t_block,
        "single_pair_evals_per_s": pair_rhs / t_single,
        "block_direct": {"kernel": "k_direct_block", "bound": "alu", "avg_launch_ms": bd_s * 1e3,
                         "flops_per_launch": st["bdirect_flops"],
                         "achieved": st["bdirect_flops"] / bd_s / 1e12 if bd_s > 0 else None,
                         "peak": PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s"},
        "block_pinv": {"kernel": "k_pinv_block_u + k_pinv_block_v (FP64 MFMA, LDS-staged)", "bound": "mfma",
                       "avg_launch_ms": bp_s * 1e3, "flops_per_launch": st["bpinv_flops"],
                       "achieved": st["bpinv_flops"] / bp_s / 1e12 if bp_s > 0 else None,
                       "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                       # the factors read once (the bytes of one single-vector apply)
                       "factor_bytes": st["pinv_bytes"],
                       "factor_gbs": st["pinv_bytes"] / bp_s / 1e9 if bp_s > 0 else None},
        "single_direct_avg_ms": d_s * 1e3,
        "single_pinv_avg_ms": p_s * 1e3,
    }


def block_section(args, torch, smfs, wl):
    """Block product of --block vectors against single products on a cut of
    the many-right-hand-side workload (volume fraction 0.35, 40% of the
    spheres in pairs, N = 1000 proxies and 1680 base nodes)."""
    pk, _ = wl.workload_block500(args.block_product_spheres, seed=args.seed)
    pb = smfs.Problem(pk.centers, pk.radius, n_proxy=1000, n_colloc_base=1680, gmres_restart=1)
    pb.bind()
    t0 = time.perf_counter()
    pb.setup()
    torch.cuda.synchronize()
    out = block_vs_single(pb, torch, args.block, 2)
    out.update(spheres=pb.P, collocation_nodes=pb.T, sources=pb.S, setup_s=time.perf_counter() - t0)
    return out


def block_solve(args, torch, smfs, wl):
    """Many-right-hand-side solve against the same systems solved one after
    another in FP64: a cut of the volume-fraction-0.35 workload (40% of the
    spheres in near-contact pairs; 1000 proxies and 1680 base nodes), 64
    rigid motions, GMRES(m) with the same restart length and tolerance; the
    block solve in --block-precision (mixed: FP32 far field in the cycles,
    FP64 restarts).  The sequential time is measured on a sample of the
    systems and scaled to all of them."""
    pk, rbm = wl.workload_block500(args.block_spheres, seed=args.seed)
    nrhs, m = rbm.shape[0], args.block_restart
    prec = {"mixed_far": smfs.SMFS_MIXED_FAR, "mixed_eq": smfs.SMFS_MIXED_EQ}.get(args.block_precision,
                                                                              smfs.SMFS_FP64)
    pb = smfs.Problem(pk.centers, pk.radius, n_proxy=1000, n_colloc_base=1680, gmres_restart=m,
                      gmres_max_it=args.block_max_it, gmres_tol=args.block_tol, gmres_check_every=0,
                      precision=prec)
    pb.bind()
    t0 = time.perf_counter()
    pb.setup()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"block solve: {pb.P} spheres, T={pb.T}, S={pb.S}, {nrhs} right-hand sides, setup {setup_s:.1f} s")
    R = torch.from_numpy(np.ascontiguousarray(rbm)).cuda()
    pb.solve_resistance_block(R[:4], restart=m)          # warm-up (code, workspace)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    blk = pb.solve_resistance_block(R, restart=m)
    torch.cuda.synchronize()
    t_block = time.perf_counter() - t1
    ft_blk = blk["ft"].cpu().numpy()
    k = min(nrhs, args.block_sequential)
    its, dft = [], 0.0
    pb.set_solver(smfs.SMFS_FP64, args.block_tol)
    t2 = time.perf_counter()
    for q in range(k):
        o = pb.solve_resistance(R[q].reshape(-1).contiguous(), want_check=False)
        its.append(o["iterations"])
        f = o["ft"].cpu().numpy().reshape(-1, 6)
        dft = max(dft, float(np.abs(f - ft_blk[q]).max() / np.abs(f).max()))
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t2) / k * nrhs
    log(f"  block solve: {t_block:.1f} s ({args.block_precision}, status {int(blk['status'])}, max it "
        f"{int(blk['max_iterations'])}, +{int(blk['refinements'])} refinements, largest true residual "
        f"{float(np.max(blk['true_rel_residual'])):.2e}) against {t_seq:.1f} s for "
        f"{nrhs} FP64 solves one after another (from {k}); F/T agree to {dft:.1e}")
    return {
        "spheres": pb.P, "collocation_nodes": pb.T, "sources": pb.S, "nrhs": nrhs, "restart": m,
        "tol": args.block_tol, "setup_s": setup_s, "block_precision": args.block_precision,
        "block_status": int(blk["status"]), "block_refinements": int(blk["refinements"]),
        "block_pair_evals_f32": int(blk["pair_evals_f32"]),
        "block_solve_s": t_block, "block_iterations_max": int(blk["max_iterations"]),
        "block_converged": int(blk["n_converged"]),
        "max_true_rel_residual": float(np.max(blk["true_rel_residual"])),
        "sequential_sample": k, "sequential_iterations": its,
        "sequential_solve_s_for_all": t_seq,
        "speedup_block_over_sequential": t_seq / t_block,
        "block_vs_sequential_ft_rel_diff": dft,
        "block_pair_rhs_evals_per_s": blk["pair_evals"] / t_block,
    }


def _gen_request(args):
    from paper_2407_03343_amd import workloads as wl
    i, seed, kw = args
    return wl.serving_stream(n=1, seed=seed * 100003 + i, **kw)[0]


def full_solve(args, torch, smfs, wl):
    """The headline packing solved as a mobility problem (random forces and
    torques in, rigid motions out), FP64 against SMFS_MIXED_EQ on the same
    seed, GMRES to --full-tol; the solver prints a progress line every 50
    iterations."""
    pk = wl.workload_packing2000(args.full_solve, seed=args.seed)
    out = {"spheres": pk.P, "tol": args.full_tol, "forms": {}}
    ft = torch.from_numpy(wl.random_ft(pk.P, 1, 5 + args.seed)[0].reshape(-1)).cuda()
    rbm = {}
    for name, prec in (("mixed_eq", smfs.SMFS_MIXED_EQ), ("fp64", smfs.SMFS_FP64)):
        if name not in args.full_forms:
            continue
        pb = smfs.Problem(pk.centers, pk.radius, gmres_restart=args.full_restart, gmres_max_it=args.full_restart,
                          gmres_tol=args.full_tol, precision=prec, progress=50)
        pb.bind()
        t0 = time.perf_counter()
        pb.setup()
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        log(f"full solve ({name}): {pb.P} spheres, T={pb.T}, S={pb.S}, setup {setup_s:.1f} s")
        t1 = time.perf_counter()
        o = pb.solve_mobility(ft, want_check=False)
        torch.cuda.synchronize()
        solve_s = time.perf_counter() - t1
        rbm[name] = o["rbm"].cpu().numpy()
        out["forms"][name] = dict(setup_s=setup_s, solve_s=solve_s, iterations=o["iterations"],
                                  refinements=o["refinements"], status=o["status"],
                                  true_rel_residual=o["true_rel_residual"], pair_evals=o["pair_evals"],
                                  pair_evals_f32=o["pair_evals_f32"])
        log(f"  {name}: {o['iterations']} it (+{o['refinements']}), status {o['status']}, true "
            f"{o['true_rel_residual']:.2e}, {solve_s:.1f} s")
        del pb
        torch.cuda.empty_cache()
    for name, r in rbm.items():
        out["forms"][name]["rbm_first_sphere"] = [float(v) for v in r[:6]]
        if args.full_save:
            np.save(f"{args.full_save}_{name}.npy", r)
    if "fp64" in rbm and "mixed_eq" in rbm:
        d = float(np.abs(rbm["mixed_eq"] - rbm["fp64"]).max() / np.abs(rbm["fp64"]).max())
        out["rbm_rel_diff_eq_vs_fp64"] = d
        out["speedup_eq_over_fp64"] = out["forms"]["fp64"]["solve_s"] / out["forms"]["mixed_eq"]["solve_s"]
        log(f"  rigid motions: SMFS_MIXED_EQ vs FP64 {d:.2e}; speed-up {out['speedup_eq_over_fp64']:.2f}x")
    return out


def serving_requests(args):
    """The request stream (generated in worker processes before the GPU is
    touched): packings and rigid motions, and Poisson arrival offsets."""
    import multiprocessing as mp
    n = args.serve_requests
    rng = np.random.default_rng(args.seed + 77)
    arrivals = np.concatenate([[0.0], np.cumsum(rng.exponential(1.0 / args.serve_rate, n - 1))])
    log(f"serving: generating {n} requests ...")
    pool = mp.get_context("spawn").Pool(min(16, os.cpu_count() or 4))
    try:
        reqs = pool.map(_gen_request, [(i, args.seed, dict(rate=args.serve_rate)) for i in range(n)])
        pool.close()
    except BaseException:
        pool.terminate()
        raise
    finally:
        pool.join()
    return reqs, arrivals


def serving(args, torch, smfs, reqs, arrivals):
    """Poisson stream of independent resistance solves through the
    continuous-batching server; p50/p99 latency from arrival to result and
    solves/s, beside the same requests solved one after another with the
    single-problem path (a sample of them, timed end to end)."""
    n = len(reqs)
    disc = dict(n_proxy=args.serve_proxy, n_colloc_base=args.serve_colloc, n_image=args.serve_image,
                n_check_base=0,
                svd_method=smfs.SMFS_SVD_JACOBI if args.serve_svd == "jacobi" else smfs.SMFS_SVD_ROCSOLVER)
    solver = dict(gmres_tol=args.serve_tol, gmres_restart=100, gmres_max_it=3000)
    prec = smfs.SMFS_MIXED_FAR if args.serve_precision == "mixed_far" else smfs.SMFS_FP64
    srv = smfs.Server(arena_bytes=args.serve_arena << 30, max_active=args.serve_slots,
                      setup_workers=args.serve_workers, server_precision=prec,
                      iters_per_step=args.serve_iters, setup_batch=args.serve_setup_batch, **disc, **solver)
    t0 = srv.clock() + 0.02
    ids, i, last_log = [], 0, time.perf_counter()
    while True:
        now = srv.clock()
        while i < n and t0 + arrivals[i] <= now:
            ids.append(srv.submit(reqs[i]["centers"], reqs[i]["rbm"], t0 + arrivals[i]))
            i += 1
        a, w = srv.step()
        st = srv.stats()
        if st["completed"] + st["failed"] == n:
            break
        if a == 0:
            time.sleep(0.0002)
        if time.perf_counter() - last_log > 20:
            last_log = time.perf_counter()
            log(f"  serving: submitted {i}, done {st['completed']}, resident {a}, waiting {w}")
    res = [srv.poll(rid, r["P"]) for rid, r in zip(ids, reqs)]
    st = srv.stats()
    srv.close()
    errors = sorted({r["error"] for r in res if r["status"] < 0})
    for e in errors:
        log(f"  serving: failed requests report: {e}")
    lat = np.array([r["t_done"] - r["t_arrival"] for r in res]) * 1e3
    span = max(r["t_done"] for r in res) - t0
    pairs = sum(r["pair_evals"] for r in res)
    its = np.array([r["iterations"] for r in res])
    out = {
        "requests": n, "rate_per_s": args.serve_rate, "setup_workers": args.serve_workers,
        "precision": args.serve_precision, "svd": args.serve_svd, "setup_batch": args.serve_setup_batch,
        "pair_evals_f32": int(sum(r["pair_evals_f32"] for r in res)),
        "refinements_max": int(max(r["refinements"] for r in res)),
        "stagnated": int(sum(1 for r in res if r["status"] == 3)),
        "discretisation": disc, "tol": args.serve_tol, "slots": args.serve_slots,
        "latency_ms_p50": float(np.percentile(lat, 50)),
        "latency_ms_p99": float(np.percentile(lat, 99)),
        "solves_per_s": n / span,
        "pair_evals_per_s": pairs / span,
        "makespan_s": span,
        "iterations_p50": float(np.percentile(its, 50)),
        "failed": int(st["failed"]), "errors": errors,
        "not_converged": int(sum(1 for r in res if r["status"] == 1)),
        "max_true_rel_residual": float(max(r["true_rel_residual"] for r in res)),
        "peak_active": st["peak_active"], "steps": st["steps"],
        "iterations_per_step": st["iterations"] / max(1, st["steps"]),
        "mean_resident_per_iteration": st["request_iterations"] / max(1, st["iterations"]),
        "setup_ms_total": st["setup_ms"], "step_ms_total": st["step_ms"], "tick_ms_total": st["tick_ms"],
        "setup_batches": st["setup_batches"],
        "arena_peak_gib": st["arena_peak"] / 2**30,
    }
    # the same requests one after another through the single-problem path
    k = min(n, args.serve_sequential)
    if k == 0:
        return out
    t1 = time.perf_counter()
    for r in reqs[:k]:
        pb = smfs.Problem(r["centers"], 1.0, gmres_check_every=0, **disc, **solver).bind().setup()
        pb.solve_resistance(torch.from_numpy(r["rbm"].reshape(-1)).cuda(), want_check=False)
        torch.cuda.synchronize()
        del pb
    seq_s = time.perf_counter() - t1
    out["sequential_sample"] = k
    out["sequential_solves_per_s"] = k / seq_s
    out["speedup_served_over_sequential"] = out["solves_per_s"] / out["sequential_solves_per_s"]
    return out


def apply_only(args, torch, smfs, wl):
    """Profiling aid: N products with G_hat on the headline workload with
    seeded rank-48 factors in place of the SVD set-up (the direct sum, the
    kernel counted here, does not depend on the factors), then one plain
    1 GiB fill and one elementwise product (the counter calibration
    kernels).  Prints one JSON line of event timings."""
    pk = wl.workload_packing2000(args.spheres, seed=args.seed)
    pb = smfs.Problem(pk.centers, pk.radius, gmres_restart=1).bind()
    for fid in range(pb.sizes.n_factors):
        info = pb.factor_info(fid)
        if info["sphere"] < 0:
            continue
        U, s, V = wl.random_factors(info["rows"], info["cols"], 48, seed=100 + fid)
        pb.import_factor(fid, U, s, V)
    prec = smfs.SMFS_MIXED_EQ if args.apply_precision == "mixed_eq" else smfs.SMFS_FP64
    if prec == smfs.SMFS_MIXED_EQ:
        pb.setup_far_field()
    mu = torch.from_numpy(wl.random_vector(3 * pb.T, 3)).cuda()
    y = torch.empty_like(mu)
    pb.profile(True)
    for _ in range(args.apply_only):
        pb.apply(mu, precision=prec, out=y)
    torch.cuda.synchronize()
    pb.profile(False)
    st = pb.profile_read()
    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    z = torch.empty_like(x)
    x.fill_(1.0)                  # calibration: writes exactly 1 GiB
    torch.mul(x, 2.0, out=z)      # calibration: reads 1 GiB, writes 1 GiB
    torch.cuda.synchronize()
    del x, z
    n_eq = max(1, st["eq_launches"])
    print(json.dumps({"apply_only": args.apply_only, "spheres": pb.P, "precision": args.apply_precision,
                      "eq_far_avg_ms": st["eq_far_ms"] / n_eq, "eq_near_avg_ms": st["eq_near_ms"] / n_eq,
                      "eq_far_flops": st["eq_far_flops"], "eq_near_flops": st["eq_near_flops"],
                      "contact_fp64_avg_ms": st["mixed64_ms"] / max(1, st["mixed64_launches"]),
                      "direct_avg_ms": st["direct_ms"] / max(1, st["direct_launches"]),
                      "pinv_avg_ms": st["pinv_ms"] / max(1, st["pinv_launches"]),
                      "direct_flops": st["direct_flops"], "pinv_bytes": st["pinv_bytes"],
                      "copy_bytes": 1 << 30}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed FP64 products")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--spheres", type=int, default=2000, help="spheres of the headline packing")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="wall-clock budget of the whole run; default sections are skipped when "
                         "their estimated cost no longer fits")
    ap.add_argument("--reserve-s", type=float, default=20.0, help="seconds kept in reserve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed products beside the headline")
    ap.add_argument("--svd", choices=["rocsolver", "jacobi"], default="rocsolver",
                    help="SVD of the self blocks at set-up")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="length of the oracle's timed sample")
    ap.add_argument("--solve-forms", nargs="+", default=["fp64", "mixed_eq"],
                    choices=[f for f, _ in FORMS],
                    help="forms of the solve section (SMFS_MIXED and SMFS_MIXED_FAR stop on their "
                         "true-residual floor above the gates on this workload)")
    ap.add_argument("--solve-spheres", type=int, default=200,
                    help="spheres of the solve-time comparison (a cut of the headline recipe; 0: skip)")
    ap.add_argument("--solve-tols", type=float, nargs="+", default=[1e-6, 1e-7, 1e-8],
                    help="GMRES tolerance ladder, loosest first, the same for every form")
    ap.add_argument("--solve-reps", type=int, default=3, help="solves at the chosen tolerance (p50/p99)")
    ap.add_argument("--solve-restart", type=int, default=1500)
    ap.add_argument("--two-sphere-reps", type=int, default=50,
                    help="timed solves of the two-sphere case at gap 0.01 (0: skip)")
    ap.add_argument("--apply-only", type=int, default=0, metavar="N",
                    help="profiling aid: N products on the headline workload with seeded full-rank "
                         "factors, then the counter calibration kernels; nothing else runs")
    ap.add_argument("--apply-precision", choices=["fp64", "mixed_eq"], default="fp64",
                    help="form of the --apply-only products")
    ap.add_argument("--full-solve", type=int, default=0, metavar="P",
                    help="mobility solve of the P-sphere packing, FP64 against SMFS_MIXED_EQ")
    ap.add_argument("--full-tol", type=float, default=1e-5)
    ap.add_argument("--full-forms", nargs="+", default=["mixed_eq", "fp64"], choices=["mixed_eq", "fp64"])
    ap.add_argument("--full-restart", type=int, default=1000)
    ap.add_argument("--full-save", default="", help="path prefix for the rigid motions found (.npy)")
    ap.add_argument("--sections-out", default="", help="JSON file for the optional sections")
    ap.add_argument("--block", type=int, default=0, metavar="NRHS",
                    help="block product of NRHS vectors vs single products (0: skip)")
    ap.add_argument("--block-product-spheres", type=int, default=100)
    ap.add_argument("--block-spheres", type=int, default=0,
                    help="spheres of the many-right-hand-side solve comparison (0: skip)")
    ap.add_argument("--block-restart", type=int, default=200)
    ap.add_argument("--block-tol", type=float, default=1e-8)
    ap.add_argument("--block-max-it", type=int, default=3000)
    ap.add_argument("--block-sequential", type=int, default=4)
    ap.add_argument("--block-precision", choices=["fp64", "mixed_far", "mixed_eq"], default="mixed_eq",
                    help="products of the block solve (the sequential solves are FP64)")
    ap.add_argument("--serve-requests", type=int, default=16,
                    help="requests of the serving stream (0: skip; the full stream is 512)")
    ap.add_argument("--serve-late", action="store_true",
                    help="serve after the headline line (an optional section) instead of inside it")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-arena", type=int, default=64, metavar="GIB")
    ap.add_argument("--serve-proxy", type=int, default=120)
    ap.add_argument("--serve-colloc", type=int, default=160)
    ap.add_argument("--serve-image", type=int, default=6)
    ap.add_argument("--serve-tol", type=float, default=1e-6)
    ap.add_argument("--serve-workers", type=int, default=1, help="set-up worker threads")
    ap.add_argument("--serve-precision", choices=["fp64", "mixed_far"], default="mixed_far",
                    help="products inside the served GMRES iterations")
    ap.add_argument("--serve-sequential", type=int, default=2,
                    help="requests solved one after another for the comparison")
    ap.add_argument("--serve-svd", choices=["rocsolver", "jacobi"], default="jacobi",
                    help="SVD of the served requests' self blocks at set-up")
    ap.add_argument("--serve-setup-batch", type=int, default=4,
                    help="most requests a set-up worker factorises together (smaller: resident sooner)")
    ap.add_argument("--serve-iters", type=int, default=8,
                    help="GMRES iterations per server step (no host round trip between them)")
    ap.add_argument("--serve-only", action="store_true",
                    help="run the serving section alone (no headline line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(how it would shard is written up in the design notes); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    budget = Budget(args.budget_s)

    reqs = arrivals = None
    if args.serve_requests > 0 and not args.apply_only:
        reqs, arrivals = serving_requests(args)     # before the GPU is touched (spawned workers)

    import torch
    from paper_2407_03343_amd import smfs, workloads as wl

    if args.apply_only:
        apply_only(args, torch, smfs, wl)
        return
    if args.serve_only:
        if reqs is None:
            print("--serve-only needs --serve-requests", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({"serving": serving(args, torch, smfs, reqs, arrivals)}), flush=True)
        return

    pk, pb, result = headline(args, torch, smfs, wl, budget)
    del pb
    torch.cuda.empty_cache()
    skipped = []
    if not args.no_cpu_baseline:
        if budget.fits(3 * args.cpu_seconds + 30 + args.reserve_s):
            log("cpu baseline (oracle) ...")
            result["cpu_baseline"] = cpu_baseline(pk, args.cpu_seconds)
            log(f"  {result['cpu_baseline']['value']:.3e} pair-evals/s: {result['cpu_baseline']['sample']}")
        else:
            skipped.append("cpu_baseline")
    if args.solve_spheres > 0:
        if budget.fits(60 + args.reserve_s):
            result["solve"] = solve_section(args, torch, smfs, wl, budget)
            torch.cuda.empty_cache()
        else:
            skipped.append("solve")
    if args.two_sphere_reps > 0:
        if budget.fits(15 + args.reserve_s):
            result["two_sphere"] = two_sphere(args, torch, smfs, wl, budget)
        else:
            skipped.append("two_sphere")
    if args.serve_requests > 0 and not args.serve_late:
        # the makespan is set-up bound (about 4 s per request here) plus the
        # sequential sample (about 10 s per request)
        if budget.fits(4.0 * args.serve_requests + 10.0 * args.serve_sequential + 10 + args.reserve_s):
            result["serving"] = serving(args, torch, smfs, reqs, arrivals)
            log("serving: p50 {latency_ms_p50:.0f} ms, p99 {latency_ms_p99:.0f} ms, {solves_per_s:.3f} solves/s "
                "against {sequential_solves_per_s:.3f} one after another".format(**result["serving"]))
        else:
            skipped.append("serving")
    if skipped:
        result["skipped_for_wall_budget"] = skipped
    result["wall_s"] = time.perf_counter() - budget.t0
    print(json.dumps(result), flush=True)

    # optional sections: stderr and --sections-out only
    extra = {}
    if args.block:
        extra["block_vs_single"] = block_section(args, torch, smfs, wl)
        torch.cuda.empty_cache()
    if args.block_spheres > 0:
        extra["block_solve"] = block_solve(args, torch, smfs, wl)
        torch.cuda.empty_cache()
    if args.serve_requests > 0 and args.serve_late:
        extra["serving"] = serving(args, torch, smfs, reqs, arrivals)
    if args.full_solve > 0:
        extra["full_solve"] = full_solve(args, torch, smfs, wl)
    if extra:
        log("sections: " + json.dumps(extra))
        if args.sections_out:
            with open(args.sections_out, "w") as f:
                json.dump(extra, f, indent=1)


if __name__ == "__main__":
    main()
