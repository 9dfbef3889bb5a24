#!/usr/bin/env python
"""Benchmark of the one-body preconditioned MFS resistance solve on one MI355X.

Workload (default): 100 unit spheres in a cube at volume fraction 0.2,
cluster-grown so that gaps are log-uniform in [1e-3, 1e-1]; 600 proxy
Stokeslets on R_p = 0.7, 780 base collocation nodes, 20 image nodes (S, R, D)
per contact with gap < 0.2, two caps of 360 nodes per contact; plain FP64;
GMRES to 1e-10.  Random rigid-body velocities, N(0, 1).

A step is one complete resistance solve: right-hand side, GMRES (every
iteration one product with G_hat = pseudo-inverse apply + direct sum, plus
Arnoldi), FP64 true residual, back-transform to strengths, forces and
torques, and the surface velocity at the residual check points.  The
self-block factorisation (setup) runs once before the timed region and is
reported separately.

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
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
# HBM bytes per launch of the direct sum on the 100-sphere workload (62 source
# splits): rocprofv3 FETCH_SIZE (x2, the factor a plain 1 GiB elementwise
# copy reads back) plus WRITE_SIZE (x1), KiB per dispatch, from the counter
# summary of this kernel under profiles/
DIRECT_TRAFFIC_BYTES = (2 * 225712.4 + 387462.0) * 1024


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(pk, stride: int, two_sphere: bool = True):
    """The FP64 oracle's direct sum (its dominant step) on a bounded sample:
    every stride-th collocation node of the same workload against all
    sources, same-sphere pairs skipped.  Returns pair-evals/s, and with
    two_sphere the oracle's two-sphere solve times."""
    from oracle import geometry as geo
    from oracle.pairsum import pairsum, build
    build(force=False)
    g = geo.build(pk.centers, pk.radius)
    rows = np.arange(0, g.T, stride)
    lam = np.random.default_rng(7).standard_normal((g.S, 3))
    t0 = time.perf_counter()
    pairsum(g.targets[rows], g.src_pos, g.src_kind, lam, 1.0, g.target_sphere[rows], g.src_sphere, True)
    dt = time.perf_counter() - t0
    own = np.bincount(g.src_sphere, minlength=g.P)
    pairs = float(np.sum(g.S - own[g.target_sphere[rows]]))
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = dict(value=pairs / dt, unit="pair-evals/s", cores=cores, kind="oracle",
               sample=(f"oracle C direct sum (OpenMP), {rows.size} of {g.T} collocation nodes "
                       f"(every {stride}) x {g.S} sources, same-sphere pairs skipped: "
                       f"{pairs:.3g} pairs in {dt:.1f} s"))
    if two_sphere:
        out["two_sphere_solve"] = oracle_two_sphere()
    return out


def oracle_two_sphere():
    """The oracle's complete solve of the two-sphere case (gap 0.01, FP64 to
    1e-10), set-up (LAPACK SVDs) and solve timed apart: the CPU counterpart
    of the benchmark's two-sphere section."""
    from oracle import geometry as geo, mfs
    from paper_2407_03343_amd import workloads as wl
    pk, rbm = wl.workload_two_sphere_gap001()
    t0 = time.perf_counter()
    pb = mfs.Problem(geo.build(pk.centers, pk.radius)).setup()
    t1 = time.perf_counter()
    o = mfs.solve_resistance(pb, rbm[0], tol=1e-10)
    t2 = time.perf_counter()
    return dict(setup_s=t1 - t0, solve_ms=(t2 - t1) * 1e3, iterations=int(o["iterations"]),
                force_sphere0=[float(x) for x in o["ft"][0, :3]])


FORMS = (("fp64", 0), ("mixed", 1), ("mixed_far", 2))   # SMFS_FP64, SMFS_MIXED, SMFS_MIXED_FAR


def mixed_vs_fp64(args, torch, smfs, wl):
    """Solve time to 1e-3 relative surface velocity, plain FP64 against the
    mixed forms (FP32 pseudo-inverse and far field; FP32 far field only), on
    a cut of the volume-fraction-0.3 packing with 5% of the
    spheres in near-contact pairs.  The reference is the FP64 solve at
    tolerance 1e-10; for each form the fastest GMRES tolerance whose
    check-point velocities meet 1e-3 (relative to the largest) is reported,
    with its force/torque error beside it."""
    pk = wl.workload_packing2000(args.mixed_spheres, seed=args.seed)
    pb = smfs.Problem(pk.centers, pk.radius, gmres_restart=1000, gmres_max_it=1000)
    pb.bind()
    t0 = time.perf_counter()
    pb.setup()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    rbm = torch.from_numpy(wl.random_rbm(pb.P, 1, 77)[0].reshape(-1)).cuda()
    pb.set_solver(smfs.SMFS_FP64, 1e-10)
    ref = pb.solve_resistance(rbm)
    u_ref = ref["u_check"].cpu().numpy()
    ft_ref = ref["ft"].cpu().numpy()
    log(f"mixed section: {pb.P} spheres, T={pb.T}, S={pb.S}, setup {setup_s:.1f} s, "
        f"reference it {ref['iterations']}")
    out = {"spheres": pb.P, "collocation_nodes": pb.T, "sources": pb.S,
           "pairs_per_apply": pb.pairs_per_apply, "reference_iterations": ref["iterations"],
           "setup_s": setup_s, "forms": {}}
    for name, prec in FORMS:
        rows = []
        pb.profile(True)
        for tol in args.mixed_tols:
            pb.set_solver(prec, tol)
            ts = []
            for _ in range(args.mixed_reps):
                t1 = time.perf_counter()
                o = pb.solve_resistance(rbm)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t1) * 1e3)
            u = o["u_check"].cpu().numpy()
            du = float(np.abs(u - u_ref).max() / np.abs(u_ref).max())
            dft = float(np.abs(o["ft"].cpu().numpy() - ft_ref).max() / np.abs(ft_ref).max())
            rows.append(dict(tol=tol, iterations=o["iterations"], refinements=o["refinements"],
                             solve_ms_p50=float(np.percentile(ts, 50)),
                             solve_ms_p99=float(np.percentile(ts, 99)),
                             u_rel_err=du, ft_rel_err=dft,
                             pair_evals=o["pair_evals"], pair_evals_f32=o["pair_evals_f32"],
                             pair_evals_per_s=o["pair_evals"] / (np.percentile(ts, 50) * 1e-3)))
            log(f"  {name} tol {tol:.0e}: it {o['iterations']} (+{o['refinements']}), "
                f"{rows[-1]['solve_ms_p50']:.1f} ms, u err {du:.2e}, F/T err {dft:.2e}")
        pb.profile(False)
        ok = [r for r in rows if r["u_rel_err"] <= 1e-3]
        best = min(ok, key=lambda r: r["solve_ms_p50"]) if ok else None
        out["forms"][name] = {"scan": rows, "at_1e-3_surface_velocity": best,
                              "kernels": mixed_kernel_rates(pb.profile_read())}
    # mobility (forces and torques in), each form at the tolerance that met
    # the surface-velocity target above; error of the rigid motions against
    # the FP64 mobility solve at 1e-10
    ft = torch.from_numpy(wl.random_ft(pb.P, 1, 78)[0].reshape(-1)).cuda()
    pb.set_solver(smfs.SMFS_FP64, 1e-10)
    v_ref = pb.solve_mobility(ft)["rbm"].cpu().numpy()
    out["mobility"] = {}
    for name, prec in FORMS:
        best = out["forms"][name]["at_1e-3_surface_velocity"]
        tol = best["tol"] if best else 1e-6
        pb.set_solver(prec, tol)
        t1 = time.perf_counter()
        o = pb.solve_mobility(ft)
        torch.cuda.synchronize()
        solve_ms = (time.perf_counter() - t1) * 1e3
        dv = float(np.abs(o["rbm"].cpu().numpy() - v_ref).max() / np.abs(v_ref).max())
        out["mobility"][name] = dict(tol=tol, iterations=o["iterations"], refinements=o["refinements"],
                                     solve_ms=solve_ms,
                                     true_rel_residual=o["true_rel_residual"], converged=o["converged"],
                                     rbm_rel_err=dv)
        log(f"  mobility {name} tol {tol:.0e}: it {o['iterations']}, {solve_ms:.1f} ms, V err {dv:.2e}")
    f64 = out["forms"]["fp64"]["at_1e-3_surface_velocity"]
    for name, _ in FORMS[1:]:
        mx = out["forms"][name]["at_1e-3_surface_velocity"]
        if f64 and mx:
            out[f"speedup_{name}_over_fp64"] = f64["solve_ms_p50"] / mx["solve_ms_p50"]
        mb = out["mobility"]
        out[f"mobility_speedup_{name}_over_fp64"] = mb["fp64"]["solve_ms"] / mb[name]["solve_ms"]
    return out


def two_sphere(args, torch, smfs, wl):
    """The paper's two-sphere case (Section 5, the comparison with Brenner's
    series): unit spheres at gap 0.01 moving apart at unit relative speed,
    FP64, GMRES to 1e-10.  Set-up once (timed), then repeated complete
    solves (right-hand side, GMRES, back-transform, forces and torques,
    check-point velocities) for p50/p99."""
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
        t1 = time.perf_counter()
        o = pb.solve_resistance(r)
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t1) * 1e3)
        pairs += o["pair_evals"]
    ft = o["ft"].cpu().numpy().reshape(-1, 6)
    out = dict(spheres=2, gap=0.01, collocation_nodes=pb.T, sources=pb.S, setup_s=setup_s,
               reps=len(ts), solve_ms_p50=float(np.percentile(ts, 50)),
               solve_ms_p99=float(np.percentile(ts, 99)), iterations=o["iterations"],
               true_rel_residual=o["true_rel_residual"], eps_res_max=o["eps_res_max"],
               force_sphere0=[float(x) for x in ft[0, :3]],
               pair_evals_per_s=pairs / (sum(ts) * 1e-3))
    log(f"two spheres, gap 0.01: setup {setup_s:.2f} s, solve p50 {out['solve_ms_p50']:.2f} ms "
        f"p99 {out['solve_ms_p99']:.2f} ms, it {o['iterations']}, |F| {np.linalg.norm(ft[0, :3]):.6f}")
    return out


def mixed_kernel_rates(st):
    """Per-kernel rates over the profiled products of one form: the FP32 far
    field against the FP32 vector peak, the FP64 direct sum (all of the sum
    in the FP64 form, the near part in the mixed forms) against the FP64
    vector peak."""
    out = {}
    for key, label, peak in (("far32", "k_far_f32", PEAK_FP32_VALU_TFLOPS),
                             ("mixed64", "k_direct_f64 (near part)", PEAK_FP64_VALU_TFLOPS),
                             ("direct", "k_direct_f64", PEAK_FP64_VALU_TFLOPS)):
        n = st[f"{key}_launches"]
        if not n:
            continue
        ms = st[f"{key}_ms"] / n
        tf = st[f"{key}_flops"] / (ms * 1e-3) / 1e12
        out[key] = dict(kernel=label, launches=n, avg_launch_ms=ms,
                        flops_per_launch=st[f"{key}_flops"], achieved=tf, peak=peak,
                        unit="TFLOP/s", frac=tf / peak)
    return out


def apply_only(pb, n, wl, torch, block=0):
    for fid in range(pb.sizes.n_factors):
        info = pb.factor_info(fid)
        if info["sphere"] < 0:
            continue
        U, s, V = wl.random_factors(info["rows"], info["cols"], info["cols"], seed=100 + fid)
        pb.import_factor(fid, U, s, V)
    mu = torch.from_numpy(wl.random_vector(3 * pb.T, 3)).cuda()
    y = torch.empty_like(mu)
    pb.profile(True)
    for _ in range(n):
        pb.apply(mu, out=y)
    torch.cuda.synchronize()
    pb.profile(False)
    st = pb.profile_read()
    x = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    z = torch.empty_like(x)
    x.fill_(1.0)                  # calibration: writes exactly 1 GiB
    torch.mul(x, 2.0, out=z)      # calibration: reads 1 GiB, writes 1 GiB
    torch.cuda.synchronize()
    del x, z
    out = {"apply_only": n, "direct_avg_ms": st["direct_ms"] / max(1, st["direct_launches"]),
           "pinv_avg_ms": st["pinv_ms"] / max(1, st["pinv_launches"]),
           "direct_flops": st["direct_flops"], "pinv_bytes": st["pinv_bytes"],
           "copy_bytes": 1 << 30}
    if block:
        out["block"] = block_vs_single(pb, torch, block, 2)
    print(json.dumps(out), flush=True)


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
        "block_pinv": {"kernel": "k_pinv_block_u + k_pinv_block_v (FP64 MFMA)", "bound": "mfma",
                       "avg_launch_ms": bp_s * 1e3, "flops_per_launch": st["bpinv_flops"],
                       "achieved": st["bpinv_flops"] / bp_s / 1e12 if bp_s > 0 else None,
                       "peak": PEAK_FP64_MFMA_TFLOPS, "unit": "TFLOP/s"},
        "single_direct_avg_ms": d_s * 1e3,
        "single_pinv_avg_ms": p_s * 1e3,
    }


def block_solve(args, torch, smfs, wl):
    """Many-right-hand-side solve against the same systems solved one after
    another: a cut of the volume-fraction-0.35 workload (40% of the spheres
    in near-contact pairs), 64 rigid motions, both forms GMRES(m) with the
    same restart length and tolerance in FP64.  The sequential time is
    measured on a sample of the systems and scaled to all of them."""
    pk, rbm = wl.workload_block500(args.block_spheres, seed=args.seed)
    nrhs, m = rbm.shape[0], args.block_restart
    pb = smfs.Problem(pk.centers, pk.radius, gmres_restart=m, gmres_max_it=args.block_max_it,
                      gmres_tol=args.block_tol)
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
    t2 = time.perf_counter()
    for q in range(k):
        o = pb.solve_resistance(R[q].reshape(-1).contiguous(), want_check=False)
        its.append(o["iterations"])
        f = o["ft"].cpu().numpy().reshape(-1, 6)
        dft = max(dft, float(np.abs(f - ft_blk[q]).max() / np.abs(f).max()))
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t2) / k * nrhs
    return {
        "spheres": pb.P, "collocation_nodes": pb.T, "sources": pb.S, "nrhs": nrhs, "restart": m,
        "tol": args.block_tol, "setup_s": setup_s,
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


def serving_requests(args):
    """The request stream (generated in worker processes before the GPU is
    touched): packings and rigid motions, and Poisson arrival offsets."""
    import multiprocessing as mp
    n = args.serve_requests
    rng = np.random.default_rng(args.seed + 77)
    arrivals = np.concatenate([[0.0], np.cumsum(rng.exponential(1.0 / args.serve_rate, n - 1))])
    log(f"serving: generating {n} requests ...")
    with mp.get_context("spawn").Pool(min(16, os.cpu_count() or 4)) as pool:
        reqs = pool.map(_gen_request, [(i, args.seed, dict(rate=args.serve_rate)) for i in range(n)])
    return reqs, arrivals


def serving(args, torch, smfs, reqs, arrivals):
    """Poisson stream of independent resistance solves through the
    continuous-batching server; p50/p99 latency from arrival to result and
    solves/s, beside the same requests solved one after another with the
    single-problem path (a sample of them, timed end to end)."""
    n = len(reqs)
    disc = dict(n_proxy=args.serve_proxy, n_colloc_base=args.serve_colloc, n_image=args.serve_image,
                n_check_base=0)
    solver = dict(gmres_tol=args.serve_tol, gmres_restart=100, gmres_max_it=3000)
    srv = smfs.Server(arena_bytes=args.serve_arena << 30, max_active=args.serve_slots,
                      setup_workers=args.serve_workers, **disc, **solver)
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
        "mean_resident_per_step": st["request_iterations"] / max(1, st["steps"]),
        "setup_ms_total": st["setup_ms"], "step_ms_total": st["step_ms"], "tick_ms_total": st["tick_ms"],
        "setup_batches": st["setup_batches"],
        "arena_peak_gib": st["arena_peak"] / 2**30,
    }
    # the same requests one after another through the single-problem path
    k = min(n, args.serve_sequential)
    t1 = time.perf_counter()
    for r in reqs[:k]:
        pb = smfs.Problem(r["centers"], 1.0, **disc, **solver).bind().setup()
        o = pb.solve_resistance(torch.from_numpy(r["rbm"].reshape(-1)).cuda(), want_check=False)
        torch.cuda.synchronize()
        del pb
    seq_s = time.perf_counter() - t1
    out["sequential_sample"] = k
    out["sequential_solves_per_s"] = k / seq_s
    out["speedup_served_over_sequential"] = out["solves_per_s"] / out["sequential_solves_per_s"]
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-stride", type=int, default=1)
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-vs-FP64 comparison on the volume-fraction-0.3 packing")
    ap.add_argument("--mixed-spheres", type=int, default=200)
    ap.add_argument("--mixed-tols", type=float, nargs="+", default=[1e-5, 7e-6, 5e-6, 3e-6],
                    help="GMRES tolerances scanned for the 1e-3 surface-velocity target (a grid fine "
                         "around the tolerances that meet it, the same for every form)")
    ap.add_argument("--mixed-reps", type=int, default=1, help="timed solves per tolerance")
    ap.add_argument("--apply-only", type=int, default=0, metavar="N",
                    help="profiling aid: N products with G_hat on the same workload with "
                         "seeded full-rank factors instead of the SVD setup, then one plain "
                         "1 GiB device copy (the counter calibration kernel)")
    ap.add_argument("--block", type=int, default=64, metavar="NRHS",
                    help="right-hand sides of the block-product comparison (0: skip)")
    ap.add_argument("--block-spheres", type=int, default=24,
                    help="spheres of the many-right-hand-side solve comparison (0: skip)")
    ap.add_argument("--block-restart", type=int, default=200)
    ap.add_argument("--block-tol", type=float, default=1e-8)
    ap.add_argument("--block-max-it", type=int, default=3000)
    ap.add_argument("--block-sequential", type=int, default=4)
    ap.add_argument("--serve-requests", type=int, default=20,
                    help="requests of the serving stream (the full stream is 512)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-arena", type=int, default=64, metavar="GIB")
    ap.add_argument("--serve-proxy", type=int, default=120)
    ap.add_argument("--serve-colloc", type=int, default=160)
    ap.add_argument("--serve-image", type=int, default=6)
    ap.add_argument("--serve-tol", type=float, default=1e-6)
    ap.add_argument("--serve-workers", type=int, default=1, help="set-up worker threads")
    ap.add_argument("--serve-sequential", type=int, default=3,
                    help="requests solved one after another for the comparison")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving comparison")
    ap.add_argument("--mixed-only", action="store_true", help="run only the mixed-vs-FP64 comparison")
    ap.add_argument("--two-sphere-reps", type=int, default=50,
                    help="timed solves of the two-sphere case at gap 0.01 (0: skip)")
    ap.add_argument("--two-sphere-only", action="store_true", help="run only the two-sphere case")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(how it would shard is written up in the design notes); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_03343_amd import smfs, workloads as wl

    reqs = arrivals = None
    if args.serve_requests > 0:
        reqs, arrivals = serving_requests(args)
    if args.serve_only:
        print(json.dumps({"serving": serving(args, torch, smfs, reqs, arrivals)}), flush=True)
        return
    if args.mixed_only:
        print(json.dumps({"mixed_vs_fp64": mixed_vs_fp64(args, torch, smfs, wl)}), flush=True)
        return
    if args.two_sphere_only:
        print(json.dumps({"two_sphere": two_sphere(args, torch, smfs, wl)}), flush=True)
        return
    pk, _ = wl.workload_cluster100(args.seed)
    log(f"workload: {pk.P} spheres, box {pk.box:.2f}, min gap {pk.min_gaps().min():.2e}")
    pb = smfs.Problem(pk.centers, pk.radius, gmres_restart=2000, gmres_max_it=2000)
    log(f"T={pb.T} S={pb.S} check={pb.n_check} factors={pb.sizes.n_factors} "
        f"workspace={pb.sizes.workspace_bytes / 2**30:.2f} GiB pairs/apply={pb.pairs_per_apply:.3e}")
    pb.bind()
    torch.cuda.synchronize()
    if args.apply_only:
        apply_only(pb, args.apply_only, wl, torch, args.block)
        return
    t0 = time.perf_counter()
    pb.setup()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    log(f"setup (device assembly + batched SVD of {pb.sizes.n_factors - 1} self blocks): {setup_s:.1f} s")

    rbms = [torch.from_numpy(wl.random_rbm(pb.P, 1, 1000 + i)[0].reshape(-1)).cuda()
            for i in range(args.warmup + args.steps)]
    for i in range(args.warmup):
        out = pb.solve_resistance(rbms[i])
        log(f"warmup {i}: it {out['iterations']} true res {out['true_rel_residual']:.2e}")
    torch.cuda.synchronize()

    pb.profile(True)
    step_ms, pairs, outs = [], 0, []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        out = pb.solve_resistance(rbms[args.warmup + i])
        torch.cuda.synchronize()
        step_ms.append((time.perf_counter() - ts) * 1e3)
        pairs += out["pair_evals"]
        outs.append(out)
        log(f"step {i}: {step_ms[-1]:.1f} ms, it {out['iterations']}, est {out['rel_residual']:.2e}, "
            f"true {out['true_rel_residual']:.2e}, eps_res {out['eps_res_max']:.2e}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    pb.profile(False)
    st = pb.profile_read()

    direct_avg_s = st["direct_ms"] / max(1, st["direct_launches"]) * 1e-3
    achieved = st["direct_flops"] / direct_avg_s / 1e12
    pinv_avg_s = st["pinv_ms"] / max(1, st["pinv_launches"]) * 1e-3
    result = {
        "metric": "Stokeslet pair-evals/s (FP64 resistance solve, 100-sphere cluster); "
                  "solve time at 1e-3 relative surface velocity, mixed vs FP64, p50/p99",
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
        "data": "synthetic",
        "config": {
            "workload": "100 unit spheres, cube at volume fraction 0.2, gaps log-uniform [1e-3, 1e-1]; "
                        "N=600 proxy on R_p=0.7, 780 base nodes, 20 S+R+D image nodes per contact "
                        "(gap < 0.2), caps 2x360; FP64; GMRES tol 1e-10 (unrestarted, <= 2000 iterations); "
                        "one resistance solve per step",
            "spheres": pb.P, "collocation_nodes": pb.T, "sources": pb.S,
            "pairs_per_apply": pb.pairs_per_apply, "precision": "fp64",
        },
        "solve_ms_p50": float(np.percentile(step_ms, 50)),
        "solve_ms_p99": float(np.percentile(step_ms, 99)),
        "setup_s": setup_s,
        "gmres_iterations": [o["iterations"] for o in outs],
        "true_rel_residual": [o["true_rel_residual"] for o in outs],
        "eps_res_max": [o["eps_res_max"] for o in outs],
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
        },
        "pinv_apply": {
            "bound": "hbm",
            "achieved": st["pinv_bytes"] / pinv_avg_s / 1e9 if pinv_avg_s > 0 else None,
            "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "avg_launch_ms": pinv_avg_s * 1e3, "bytes_per_launch": st["pinv_bytes"],
        },
    }
    if args.block:
        log(f"block product of {args.block} vectors vs {args.block} single products ...")
        result["block_vs_single"] = block_vs_single(pb, torch, args.block, 2)
    del pb
    torch.cuda.empty_cache()
    if args.two_sphere_reps > 0:
        result["two_sphere"] = two_sphere(args, torch, smfs, wl)
        torch.cuda.empty_cache()
    if args.block_spheres > 0:
        result["block_solve"] = block_solve(args, torch, smfs, wl)
        torch.cuda.empty_cache()
    if not args.no_mixed:
        result["mixed_vs_fp64"] = mixed_vs_fp64(args, torch, smfs, wl)
        torch.cuda.empty_cache()
    if args.serve_requests > 0:
        result["serving"] = serving(args, torch, smfs, reqs, arrivals)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(pk, args.cpu_stride, two_sphere=args.two_sphere_reps > 0)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
