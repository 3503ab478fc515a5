#!/usr/bin/env python3
"""Benchmark of the multigrid-preconditioned CG hot path on one MI355X.

Workload (default "inclusions513"): -div(k grad phi) = f on a 513^3 vertex grid
(511^3 = 133,432,831 unknowns), two-phase k (random spheres, radius 4-16 cells,
20 % volume, k = 1e3 inside, 1 outside), f ~ U(-1,1), 9 levels (coarsest 3^3),
Chebyshev-Jacobi degree 2 pre/post, levels N <= 9 agglomerated into the
persistent coarse kernel.

One step = the whole hot path once:
  hierarchy setup from k  ->  mixed-precision PCG solve to an FP64 relative
  residual of 1e-8  ->  adjoint gradient dL/d ln k for L = 0.5 ||phi - phi_obs||^2
  (adjoint PCG solve + link-gradient kernel).
value = fine-grid unknowns solved per second = 2 solves x 511^3 / step time,
with the steps timed with kernel profiling off; every timed solve must reach
the tolerance (else the run fails).  Beside it: T_solve, the median of 5
forward solves with setup excluded, as unknowns/s; the same figures for plain
FP64; the error of both forward solutions against the stored FP64 oracle
solution (sampled); per-kernel HBM figures from one separate profiled step;
the agglomeration sweep on 33^3-129^3 grids; the 1025^3 combined workload.

Inputs are generated on the host (1025^3: on the GPU) and copied to HBM before
the timed region.  Kernel durations come from HIP events the library records
around every finest-level launch on its stream during the profiled step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# Algorithmic HBM bytes per interior fine-grid unknown for each finest-level
# kernel class: every array read or written once, neighbours from cache.
BYTES_PER_POINT = {
    "fp64": {"apply_dot": 40, "residual": 48, "update_r": 24, "update_xp": 40, "update_p": 16, "cheb_first": 24, "cheb_pre2": 48,
             "cheb_step": 48, "cheb_step_prev": 56, "cheb_step_dot": 56, "level_residual": 44,
             "restrict": 5, "prolong": 17, "face_gradient": 64, "cheb_post2": 56, "pre2_res": 52},
    "mixed": {"apply_dot": 36, "residual": 48, "update_r": 28, "update_xp": 28, "update_p": 8, "cheb_first": 20, "cheb_pre2": 18,
              "cheb_step": 18, "cheb_step_prev": 22, "cheb_step_dot": 30, "level_residual": 16,
              "restrict": 2.5, "prolong": 8.5, "face_gradient": 64, "cheb_post2": 26, "pre2_res": 20},
}

WORKLOADS = {
    "inclusions513": dict(n=513, levels=9, kind="inclusions", k_seed=4, kobs_seed=7, f_seed=5,
                          desc="513^3 two-phase inclusions (k=1e3 in 1, 20% volume, r 4-16 cells), "
                               "f~U(-1,1), 9 levels, V(2,2) Chebyshev-Jacobi, rtol 1e-8, forward + adjoint"),
    "lognormal257": dict(n=257, levels=8, kind="lognormal", k_seed=2, kobs_seed=7, f_seed=3, clip=2.0,
                         desc="257^3 log-normal k (sigma 8 cells, contrast 1e4), f~U(-1,1), 8 levels, "
                              "V(2,2) Chebyshev-Jacobi, rtol 1e-8, forward + adjoint"),
    "lognormal1025": dict(n=1025, levels=10, kind="lognormal", k_seed=10, kobs_seed=11, f_seed=12, clip=3.0,
                          desc="1025^3 log-normal k (contrast 1e6), f~U(-1,1), 10 levels, forward + adjoint"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_inputs(w):
    """Seeded inputs of a workload: numpy arrays, or (log-normal fields at 1025^3
    and up, too slow to filter on the host) torch tensors drawn on the GPU by
    the same recipe."""
    from paper_1604_07163_amd import inputs
    n = w["n"]
    if w["kind"] != "inclusions" and n >= 1025:
        k = inputs.lognormal_k_gpu(n, w["k_seed"], clip=w["clip"])
        kobs = inputs.lognormal_k_gpu(n, w["kobs_seed"], clip=w["clip"])
        return k, kobs, inputs.uniform_rhs_gpu(n, w["f_seed"])
    if w["kind"] == "inclusions":
        kx, ky, kz, _ = inputs.inclusion_k(n, w["k_seed"])
        kox, koy, koz, _ = inputs.inclusion_k(n, w["kobs_seed"])
    else:
        kx, ky, kz = inputs.lognormal_k(n, w["k_seed"], clip=w["clip"])
        kox, koy, koz = inputs.lognormal_k(n, w["kobs_seed"], clip=w["clip"])
    f = inputs.uniform_rhs(n, w["f_seed"])
    return (kx, ky, kz), (kox, koy, koz), f


def _dev(a):
    import torch
    return a if torch.is_tensor(a) else torch.from_numpy(a).cuda()


def _host(a):
    import torch
    return a.cpu().numpy() if torch.is_tensor(a) else a


def check_leg(info, rtol, what):
    """A timed solve that did not converge must not be reported as throughput."""
    if info["status"] != "GMG_OK" or not (info["rel_res_true"] <= rtol):
        raise RuntimeError(f"{what}: status {info['status']}, FP64 true relative residual "
                           f"{info['rel_res_true']:.3e} (tolerance {rtol:.1e})")


def run_steps(solver, k, f, phi_obs, steps, rtol, profile=False):
    """Run `steps` full steps; returns (seconds per step, last forward and adjoint
    infos, kernel-class profile (profile=True only), last forward solution).
    Every solve's status and true residual are checked."""
    import torch
    from paper_1604_07163_amd import gmg
    times, fwd, adj, phi = [], None, None, None
    prof = gmg.Profile(solver) if profile else None
    if prof:
        prof.__enter__()
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        solver.set_coefficients(*k)
        phi, fwd = solver.solve(f, rtol=rtol, max_it=2000)
        dl = phi - phi_obs  # the loss gradient (user side of the step)
        gx, gy, gz, lam, adj = solver.adjoint_gradient(phi, dl, rtol=rtol, max_it=2000, want_lambda=False)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        check_leg(fwd, rtol, "forward solve")
        check_leg(adj, rtol, "adjoint solve")
    if prof:
        prof.__exit__(None, None, None)
    return times, fwd, adj, (prof.result if prof else {}), phi


def t_solve(solver, f, rtol, reps=5):
    """Median of `reps` forward solves from x0 = 0 (setup excluded), each timed
    by the library with HIP events on its stream; after one untimed solve."""
    import numpy as np
    solver.solve(f, rtol=rtol, max_it=2000)
    ms, info = [], None
    for _ in range(reps):
        _, info = solver.solve(f, rtol=rtol, max_it=2000)
        check_leg(info, rtol, "forward solve")
        ms.append(info["solve_ms"])
    return float(np.median(ms)), info


def kernel_table(prof, prec, n_unk):
    out = {}
    for c, v in prof.items():
        entry = dict(v)
        if c in BYTES_PER_POINT[prec]:
            entry["GBs"] = BYTES_PER_POINT[prec][c] * n_unk / (v["avg_ms"] / 1e3) / 1e9
            entry["frac_peak"] = entry["GBs"] / HBM_PEAK_GBS
        out[c] = entry
    return out


def error_vs_oracle(x, workload):
    """Sampled relative L2 difference between a forward solution and the stored
    FP64 oracle solution of the same workload (4096 seeded interior points,
    written by tests/golden/make_golden.py from the oracle alone), or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{workload}.json")
    if not os.path.exists(path):
        return None
    g = json.load(open(path))
    import torch
    pts = torch.as_tensor(np.asarray(g["sample_points"]), device=x.device)
    ref = np.asarray(g["sample_values"])
    v = x[pts[:, 0], pts[:, 1], pts[:, 2]].cpu().numpy()
    return {"rel_l2_sampled": float(np.linalg.norm(v - ref) / np.linalg.norm(ref)), "samples": int(len(ref)),
            "oracle_iterations": g["iterations"], "oracle_rel_res_true": g["rel_res_true"]}


def copy_bandwidth(nbytes=2 << 30, reps=5, planes=1):
    """Achievable HBM bandwidth of a streaming copy (read + write bytes / time);
    planes > 1: the z-march pattern of the stencil kernels."""
    import torch
    from paper_1604_07163_amd import gmg
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    gmg.calibration_copy(b, a, planes)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        gmg.calibration_copy(b, a, planes)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms / 1e3) / 1e9


def cpu_baseline(w, k, f, its_needed, iters=2):
    """Time the FP64 CPU oracle for `iters` PCG iterations at the full size on
    all the host threads OpenMP uses, then one iteration on one thread, and
    scale both to the iteration count the solve needs (setup not timed)."""
    import ctypes
    import oracle
    oracle.build(force=False)
    H = oracle.Hierarchy(*k, levels=w["levels"])
    t0 = time.perf_counter()
    _, info = H.solve(f, rtol=1e-8, max_it=iters)
    dt = time.perf_counter() - t0
    per_it = dt / max(info["iterations"], 1)
    n_unk = (w["n"] - 2) ** 3
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    out = {"value": n_unk / (per_it * its_needed), "unit": "unknowns/s", "cores": cores, "kind": "oracle",
           "sample": f"{info['iterations']} FP64 PCG iterations of the oracle at {w['n']}^3 "
                     f"({dt:.1f} s, setup excluded), scaled to the {its_needed} iterations of one solve",
           "seconds_per_iteration": per_it}
    try:  # the same loop on one thread (the oracle's OpenMP runtime)
        gomp = ctypes.CDLL("libgomp.so.1")
        gomp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        _, i1 = H.solve(f, rtol=1e-8, max_it=1)
        dt1 = time.perf_counter() - t0
        gomp.omp_set_num_threads(cores)
        out["one_thread"] = {"value": n_unk / (dt1 * its_needed), "seconds_per_iteration": dt1,
                             "sample": "1 FP64 PCG iteration of the oracle on 1 thread, scaled likewise"}
    except OSError:
        pass
    H.close()
    return out


def sweep(args):
    """Switch-level sweep (grid launches vs the persistent coarse kernel) and the
    truncation arm, forward solves on the chosen workload; prints one JSON line.
    Every solve must converge; the iteration count must not depend on the
    switch level, LDS staging or team size (they change no arithmetic)."""
    import numpy as np
    import torch
    from paper_1604_07163_amd import gmg
    w = WORKLOADS[args.workload]
    n, levels = w["n"], w["levels"]
    k_in, _, f_in = make_inputs(w)
    k = [_dev(a) for a in k_in]
    f = _dev(f_in)
    rows = []
    sizes = [0] + [s for s in (65, 33, 17, 9) if s < n]
    configs = [dict(precision=p, switch_n=sw, persistent_wgs=1) for p in ("fp64", "mixed") for sw in sizes]
    # the same one-workgroup persistent kernel sweeping its levels in HBM/L2 instead of LDS
    configs += [dict(precision=p, switch_n=sw, persistent_wgs=1, persistent_lds=False)
                for p in ("fp64", "mixed") for sw in sizes if sw > 0]
    configs += [dict(precision=p, switch_n=sw, persistent_wgs=t) for p in ("fp64", "mixed")
                for sw in sizes if sw > 0 for t in args.teams]
    for t in args.teams:  # two-stage: team on the middle levels, one workgroup from 9^3 down
        for sw in [s for s in sizes if s > 17]:
            configs.append(dict(precision="mixed", switch_n=sw, persistent_wgs=t, switch2_n=9))
    for lt in args.truncate:
        configs.append(dict(precision="fp64", levels=lt, coarse_solver="cg", coarse_rtol=1e-4, flexible=True))
    for g in args.galerkin:  # Galerkin (g = 1) or hybrid (g > 1) coarse operators
        configs += [dict(precision=p, switch_n=sw, galerkin=g) for p in ("fp64", "mixed") for sw in (0, 17)]
    base_its = {}
    for cfg in configs:
        kw = dict(cfg)
        lv = kw.pop("levels", levels)
        s = gmg.Solver(*k, levels=lv, **kw)
        ms, info = t_solve(s, f, args.rtol, reps=max(1, args.steps))
        with gmg.Profile(s) as pr:
            s.solve(f, rtol=args.rtol, max_it=3000)
        coarse = pr.result.get("persistent") or pr.result.get("coarse_solve") or {}
        if lv == levels and not cfg.get("galerkin"):  # same arithmetic for every switch / team / LDS row
            ref = base_its.setdefault(cfg["precision"], info["iterations"])
            if info["iterations"] != ref:
                raise RuntimeError(f"{cfg}: {info['iterations']} iterations, {ref} with the grid path")
        row = {"levels": lv, **cfg, "iterations": info["iterations"], "coarse_iterations": info["coarse_iterations"],
               "ms": ms, "ms_per_iteration": ms / info["iterations"],
               "coarse_kernel_us": 1e3 * coarse.get("avg_ms", 0.0), "rel_res_true": info["rel_res_true"],
               "setup_ms": info["setup_ms"], "lds_bytes": s.persistent_lds_bytes}
        log(json.dumps(row))
        rows.append(row)
        s.close()
    print(json.dumps({"workload": args.workload, "n": n, "rtol": args.rtol, "rows": rows}), flush=True)


def agglomeration_sweep(rtol=1e-8, reps=5, teams=(1, 8, 32)):
    """Forward solves on the small grids where the coarse levels are launch- and
    latency-bound: the 33^3 constant-k sine problem (4 levels, coarsest 5^3) and
    log-normal grids (contrast 1e4) at 65^3 and 129^3, for every switch level
    (0 = grid launches on every level) and persistent team size, FP64 and
    MIXED.  Every solve must converge and, per grid and precision, take the same
    iteration count on every row.  Returns per grid the rows (median of `reps`
    solves, setup excluded; the coarse part's microseconds per V-cycle) and the
    argmin per precision."""
    import torch
    from paper_1604_07163_amd import gmg, inputs
    out = {}
    for n in (33, 65, 129):
        if n == 33:
            name, levels, k_in, f_in = "poisson33", 4, inputs.const_k(n), inputs.sine_rhs(n)
        else:
            name, levels = f"lognormal{n}", gmg.default_levels(n)
            k_in, f_in = inputs.lognormal_k(n, 2), inputs.uniform_rhs(n, 3)
        k = [torch.from_numpy(a).cuda() for a in k_in]
        f = torch.from_numpy(f_in).cuda()
        switches = [0] + [sw for sw in (65, 33, 17, 9) if sw < n]
        rows, best = [], {}
        for prec in ("fp64", "mixed"):
            its = None
            for sw in switches:
                for team in (teams if sw > 0 else (1,)):
                    s = gmg.Solver(*k, levels=levels, precision=prec, switch_n=sw, persistent_wgs=team)
                    ms, info = t_solve(s, f, rtol, reps)
                    with gmg.Profile(s) as pr:
                        s.solve(f, rtol=rtol, max_it=2000)
                    s.close()
                    coarse = pr.result.get("persistent") or pr.result.get("coarse_solve") or {}
                    its = info["iterations"] if its is None else its
                    if info["iterations"] != its:
                        raise RuntimeError(f"{name} {prec} switch {sw} team {team}: {info['iterations']} "
                                           f"iterations, {its} on the first row")
                    row = {"precision": prec, "switch_n": sw, "persistent_wgs": team, "iterations": its,
                           "ms": ms, "us_per_iteration": 1e3 * ms / its,
                           "coarse_us_per_vcycle": 1e3 * coarse.get("avg_ms", 0.0),
                           "unknowns_per_s": (n - 2) ** 3 / (ms / 1e3)}
                    rows.append(row)
                    if prec not in best or ms < best[prec]["ms"]:
                        best[prec] = row
        none = {p: next(r for r in rows if r["precision"] == p and r["switch_n"] == 0) for p in best}
        out[name] = {"n": n, "levels": levels, "unknowns": (n - 2) ** 3, "rows": rows,
                     "argmin": {p: {"switch_n": b["switch_n"], "persistent_wgs": b["persistent_wgs"], "ms": b["ms"],
                                    "unknowns_per_s": b["unknowns_per_s"],
                                    "speedup_vs_grid_launches": none[p]["ms"] / b["ms"]} for p, b in best.items()}}
        log(f"[agglomeration] {name}: " + ", ".join(f"{p} best switch {b['switch_n']} team {b['persistent_wgs']} "
                                                   f"{b['ms']:.2f} ms ({none[p]['ms'] / b['ms']:.2f}x vs none)"
                                                   for p, b in best.items()))
        del k, f
    return out


def large_block(rtol, switch_n):
    """The 1025^3 combined workload (log-normal k, contrast 1e6, 10 levels):
    MIXED forward T_solve (median of 3), the adjoint, per-kernel figures from a
    profiled forward solve, the FP64 forward T_solve (median of 2) and the
    MIXED-vs-FP64 difference.  Inputs are drawn on the GPU."""
    import torch
    from paper_1604_07163_amd import gmg
    w = WORKLOADS["lognormal1025"]
    n, levels = w["n"], w["levels"]
    n_unk = (n - 2) ** 3
    t0 = time.perf_counter()
    k, kobs, f = make_inputs(w)
    log(f"[1025] inputs generated in {time.perf_counter() - t0:.1f}s")
    out = {"workload": f"lognormal1025: {w['desc']}", "n": n, "levels": levels, "unknowns": n_unk,
           "switch_n": switch_n}
    s = gmg.Solver(*k, levels=levels, precision="mixed", switch_n=switch_n)
    out["setup_ms_mixed"] = s.solve(f, rtol=rtol, max_it=2000)[1]["setup_ms"]
    s.set_coefficients(*kobs)
    phi_obs, io = s.solve(f, rtol=1e-10, max_it=2000)
    check_leg(io, 1e-10, "observation solve")
    del kobs
    s.set_coefficients(*k)
    ms_m, im = t_solve(s, f, rtol, reps=3)
    x_m, _ = s.solve(f, rtol=rtol, max_it=2000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, _, _, _, ia = s.adjoint_gradient(x_m, x_m - phi_obs, rtol=rtol, max_it=2000, want_lambda=False)
    torch.cuda.synchronize()
    adj_wall = time.perf_counter() - t1
    check_leg(ia, rtol, "adjoint solve")
    with gmg.Profile(s) as pr:
        s.solve(f, rtol=rtol, max_it=2000)
    s.close()
    del s, phi_obs
    torch.cuda.empty_cache()
    out["mixed"] = {"T_solve_ms": ms_m, "unknowns_per_s": n_unk / (ms_m / 1e3), "iterations": im["iterations"],
                    "restarts": im["restarts"], "rel_res_true": im["rel_res_true"],
                    "adjoint_iterations": ia["iterations"], "adjoint_ms": 1e3 * adj_wall,
                    "kernels": kernel_table(pr.result, "mixed", n_unk)}
    log(f"[1025] mixed: {ms_m:.0f} ms per forward solve, {im['iterations']} its; adjoint {1e3 * adj_wall:.0f} ms")
    s64 = gmg.Solver(*k, levels=levels, precision="fp64", switch_n=switch_n)
    ms_d, i64 = t_solve(s64, f, rtol, reps=2)
    x64, _ = s64.solve(f, rtol=rtol, max_it=2000)
    s64.close()
    del s64
    diff = float(torch.linalg.vector_norm(x_m - x64) / torch.linalg.vector_norm(x64))
    out["fp64"] = {"T_solve_ms": ms_d, "unknowns_per_s": n_unk / (ms_d / 1e3), "iterations": i64["iterations"],
                   "rel_res_true": i64["rel_res_true"]}
    out["speedup_mixed_forward"] = ms_d / ms_m
    out["mixed_vs_fp64_rel_l2"] = diff
    log(f"[1025] fp64: {ms_d:.0f} ms per forward solve; speedup {ms_d / ms_m:.2f}x; mixed vs fp64 {diff:.2e}")
    del k, f, x_m, x64
    torch.cuda.empty_cache()
    return out


def profile_summary(d, top=25):
    """Markdown summary of a rocprofv3 output folder (CSV format): per kernel and
    grid size the dispatch count and average duration from the kernel trace, and
    the per-dispatch averages of any collected counters.  Host-only."""
    import csv
    import glob
    from collections import defaultdict

    def short(name):
        name = name.split("(")[0]
        return name.replace("void ", "").replace("gmg::", "").replace("unsigned short", "bf16")

    out = []
    for path in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)):
        agg = defaultdict(lambda: [0, 0.0])
        for r in csv.DictReader(open(path)):
            key = (short(r["Kernel_Name"]), int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
            a = agg[key]
            a[0] += 1
            a[1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
        total = sum(v[1] for v in agg.values())
        out.append(f"kernel trace: {os.path.relpath(path, d)}  (total kernel time {total / 1e3:.1f} ms)\n")
        out.append("| kernel | grid (threads) | calls | avg us | total ms | share |")
        out.append("|---|---:|---:|---:|---:|---:|")
        for (nm, g), (c, t) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
            out.append(f"| `{nm}` | {g} | {c} | {t / c:.1f} | {t / 1e3:.2f} | {100 * t / total:.1f}% |")
        out.append("")
    for path in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        agg = defaultdict(lambda: [0, 0.0])
        for r in csv.DictReader(open(path)):
            grid = r.get("Grid_Size") or r.get("Grid_Size_X") or "0"
            key = (short(r["Kernel_Name"]), int(float(grid)), r["Counter_Name"])
            a = agg[key]
            a[0] += 1
            a[1] += float(r["Counter_Value"])
        out.append(f"counters: {os.path.relpath(path, d)}\n")
        out.append("| kernel | grid (threads) | counter | dispatches | avg per dispatch |")
        out.append("|---|---:|---|---:|---:|")
        for (nm, g, cn), (c, v) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
            out.append(f"| `{nm}` | {g} | {cn} | {c} | {v / c:.1f} |")
        out.append("")
    print("\n".join(out))


# Finest-level kernel of each class in the MIXED step, as rocprofv3 names it.
CLASS_KERNELS = {
    "apply_dot": "k_apply_x2<true, float, 4>",  # 512 x 1 tiles on long rows
    "update_r": "k_update_r<float>",
    "update_xp": "k_update_xp<float, float>",
    "cheb_pre2": "k_cheb_pre2<float, bf16, false>",
    "cheb_step": "k_cheb_step<float, bf16, 0, false>",
    "cheb_step_dot": "k_cheb_step<float, bf16, 2, true>",
    "cheb_post2": "k_post2<float, bf16, 1, 8>",
    "pre2_res": "k_pre2_res<float, bf16, 16>",
    "level_residual": "k_residual_zr<float, bf16>",
    "restrict": "k_restrict_xy<float>",
    "prolong": "k_prolong<float>",
}
def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
COPY_BYTES = 2 << 30  # copy_bandwidth(): bytes read (and written) per calibration copy


def source_digest():
    """sha256 of the kernel and driver sources with comments and blank space
    removed: counter figures hold for this code only, whatever its comments say."""
    import hashlib
    import re
    hsh = hashlib.sha256()
    for rel in ("paper_1604_07163_amd/csrc/kernels.hpp", "paper_1604_07163_amd/csrc/gmg.hip"):
        with open(os.path.join(ROOT, rel), encoding="utf-8") as fh:
            src = fh.read()
        # the sources hold no string literal with "//" or "/*" in it
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        hsh.update(" ".join(src.split()).encode())
    return hsh.hexdigest()[:16]


def _short(name):
    return name.split("(")[0].replace("void ", "").replace("gmg::", "").replace("unsigned short", "bf16")


def pmc_traffic(fetch_dir, write_dir, n=513):
    """HBM bytes per finest-level launch from rocprofv3 FETCH_SIZE and WRITE_SIZE
    runs (KiB per dispatch), each scaled so that the plain calibration copy reads
    and writes exactly COPY_BYTES.  Only level-0 dispatches count: within one
    kernel name, those with at least half the largest reading.  Host only;
    prints a markdown report that `traffic_for` reads back."""
    import csv
    import glob
    from collections import defaultdict
    n_unk = (n - 2) ** 3
    vals = {}
    for d, counter in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        per = defaultdict(list)
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(path)):
                if r["Counter_Name"] == counter:
                    per[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
        vals[counter] = per
    scale = {}
    for c in ("FETCH_SIZE", "WRITE_SIZE"):
        cp = vals[c]["k_copy_march"]
        scale[c] = COPY_BYTES / (1024.0 * sum(cp) / len(cp))
    lines = [f"source_digest: {source_digest()}",
             f"calibration: k_copy_march of {COPY_BYTES} bytes; FETCH_SIZE x {scale['FETCH_SIZE']:.4f}, "
             f"WRITE_SIZE x {scale['WRITE_SIZE']:.4f}", "",
             "| class | kernel | level-0 dispatches | read GB | written GB | traffic GB | algorithmic GB | ratio |",
             "|---|---|---:|---:|---:|---:|---:|---:|"]
    figures = []
    for cls, name in CLASS_KERNELS.items():
        out = []
        for c in ("FETCH_SIZE", "WRITE_SIZE"):
            v = vals[c].get(name, [])
            if not v:
                break
            top = max(v)
            sel = [x for x in v if x >= 0.5 * top]
            out.append((len(sel), 1024.0 * scale[c] * sum(sel) / len(sel)))
        if len(out) != 2:
            continue
        rd, wr = out[0][1], out[1][1]
        alg = BYTES_PER_POINT["mixed"][cls] * n_unk
        lines.append(f"| {cls} | `{name}` | {out[0][0]} | {rd / 1e9:.3f} | {wr / 1e9:.3f} | {(rd + wr) / 1e9:.3f} | "
                     f"{alg / 1e9:.3f} | {(rd + wr) / alg:.3f} |")
        figures.append(f"traffic_bytes {cls}: {rd + wr:.6e}")
    print("\n".join(lines + [""] + figures))


def sq_summary(d, n=513):
    """Markdown table of rocprofv3 SQ counter passes (CSV folders under d):
    per kernel, the dispatches with the largest grid averaged.  Per-wave
    figures for every kernel; per-unknown figures (x 64 lanes, i.e. wave
    instructions per 64 unknowns) only for the finest-level kernels of the
    MIXED step (CLASS_KERNELS), divided by the finest level's (n-2)^3
    unknowns.  Host only."""
    import csv
    import glob
    from collections import defaultdict
    res = defaultdict(lambda: defaultdict(list))
    for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(path)):
            grid = int(float(r.get("Grid_Size") or r.get("Grid_Size_X") or "0"))
            res[(_short(r["Kernel_Name"]), grid)][r["Counter_Name"]].append(float(r["Counter_Value"]))
    largest = {}
    for nm, g in res:
        largest[nm] = max(g, largest.get(nm, 0))
    finest = set(CLASS_KERNELS.values())
    wp = (n - 2) ** 3 / 64.0
    cols = ["SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_VMEM", "SQ_INSTS_LDS"]
    out = ["| kernel | grid (threads) | dispatches | waves | VALU/wave | SALU/wave | VMEM/wave | LDS/wave | "
           "VALU per 64 finest unknowns | wait any | wait inst | VALU active |",
           "|---|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|---:|"]
    for nm in sorted(largest):
        g = largest[nm]
        c = {k: sum(v) / len(v) for k, v in res[(nm, g)].items()}
        waves = c.get("SQ_WAVES")
        if not waves:
            continue
        disp = len(res[(nm, g)]["SQ_WAVES"])
        per = [f"{c[k] / waves:.0f}" if k in c else "" for k in cols]
        pu = f"{c['SQ_INSTS_VALU'] / wp:.1f}" if nm in finest and "SQ_INSTS_VALU" in c else "(not finest)"
        wc = c.get("SQ_WAVE_CYCLES")
        fr = [f"{c[k] / wc:.3f}" if wc and k in c else "" for k in ("SQ_WAIT_ANY", "SQ_WAIT_INST_ANY",
                                                                     "SQ_ACTIVE_INST_VALU")]
        out.append(f"| `{nm}` | {g} | {disp} | {waves:.0f} | " + " | ".join(per) + f" | {pu} | " + " | ".join(fr) + " |")
    print("\n".join(out))


def traffic_for(cls, workload):
    """Counter-measured HBM bytes per launch of `cls` on `workload`, or None when
    no figure was taken or the sources have changed since it was."""
    try:
        txt = open(traffic_file(workload)).read()
    except OSError:
        return None
    if f"source_digest: {source_digest()}" not in txt:
        return None
    for line in txt.splitlines():
        if line.startswith(f"traffic_bytes {cls}:"):
            return float(line.split(":")[1])
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="inclusions513", choices=sorted(WORKLOADS))
    ap.add_argument("--switch-n", type=int, default=9)
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=3)
    ap.add_argument("--sweep", action="store_true",
                    help="switch-level / truncation sweep of forward solves instead of the benchmark step")
    ap.add_argument("--teams", type=int, nargs="*", default=[],
                    help="with --sweep: also time persistent teams of these workgroup counts")
    ap.add_argument("--truncate", type=int, nargs="*", default=[],
                    help="with --sweep: also time truncated hierarchies with these level counts")
    ap.add_argument("--profile-summary", metavar="DIR",
                    help="print a markdown summary of a rocprofv3 CSV output folder and exit (host only)")
    ap.add_argument("--pmc-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print HBM traffic per finest-level launch from rocprofv3 FETCH_SIZE / WRITE_SIZE "
                         "folders and exit (host only)")
    ap.add_argument("--sq-summary", metavar="DIR",
                    help="print a table of rocprofv3 SQ counter folders under DIR and exit (host only)")
    ap.add_argument("--galerkin", type=int, nargs="*", default=[],
                    help="with --sweep: also time Galerkin coarse operators from these first levels")
    ap.add_argument("--no-agglomeration", action="store_true",
                    help="skip the 33^3-129^3 switch-level / team sweep of the bench line")
    ap.add_argument("--no-large", action="store_true", help="skip the 1025^3 block of the bench line")
    ap.add_argument("--post-fused", default="auto", choices=["auto", "0", "1"],
                    help="one-sweep post-smoothing: auto (the library default: one sweep), 0 two sweeps, 1 one sweep")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(args.profile_summary)
        return
    if args.pmc_traffic:
        pmc_traffic(*args.pmc_traffic)
        return
    if args.sq_summary:
        sq_summary(args.sq_summary)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1).", flush=True)
        sys.exit(2)
    if args.sweep:
        sweep(args)
        return

    import numpy as np
    import torch
    from paper_1604_07163_amd import gmg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    w = WORKLOADS[args.workload]
    n, levels = w["n"], w["levels"]
    n_unk = (n - 2) ** 3
    t0 = time.perf_counter()
    k_in, kobs_in, f_in = make_inputs(w)
    log(f"inputs generated in {time.perf_counter() - t0:.1f}s")
    k = [_dev(a) for a in k_in]
    kobs = [_dev(a) for a in kobs_in]
    f = _dev(f_in)
    del kobs_in

    copy_gbs = copy_bandwidth()
    copy_march = {str(pl): copy_bandwidth(planes=pl) for pl in (8, 32)}
    log(f"streaming copy: {copy_gbs:.0f} GB/s one element per thread; z-march copy {copy_march} GB/s")
    legs = {}
    results = {}
    for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
        s = gmg.Solver(*k, levels=levels, precision=prec, switch_n=args.switch_n,
                       post_fused="auto" if args.post_fused == "auto" else args.post_fused == "1")
        # phi_obs: forward solve with the observation coefficients (untimed)
        s.set_coefficients(*kobs)
        phi_obs, io = s.solve(f, rtol=1e-10, max_it=2000)
        check_leg(io, 1e-10, "observation solve")
        s.set_coefficients(*k)
        steps = args.steps if prec == "mixed" else max(1, (args.steps + 1) // 2)
        run_steps(s, k, f, phi_obs, args.warmup, args.rtol)
        log(f"[{prec}] warmup done; timing {steps} steps")
        times, fwd, adj, _, phi = run_steps(s, k, f, phi_obs, steps, args.rtol)
        tsol, tinfo = t_solve(s, f, args.rtol)
        _, _, _, prof, _ = run_steps(s, k, f, phi_obs, 1, args.rtol, profile=True)
        legs[prec] = {"ms_per_step": 1e3 * float(np.mean(times)), "ms_min": 1e3 * float(np.min(times)),
                      "forward": fwd, "adjoint": adj, "kernels": prof, "T_solve_ms": tsol}
        results[prec] = phi.clone()
        legs[prec]["error_vs_oracle"] = error_vs_oracle(phi, args.workload)
        log(f"[{prec}] {legs[prec]['ms_per_step']:.1f} ms/step; T_solve {tsol:.1f} ms; fwd its {fwd['iterations']} "
            f"true {fwd['rel_res_true']:.2e}; adj its {adj['iterations']}; vs oracle {legs[prec]['error_vs_oracle']}")
        s.close()
        del s, phi_obs, phi
        torch.cuda.empty_cache()

    mixed = legs["mixed"]
    ms = mixed["ms_per_step"]
    value = 2 * n_unk / (ms / 1e3)
    # dominant finest-level HBM kernel of the mixed step (profiled step)
    bpp = BYTES_PER_POINT["mixed"]
    cands = {c: v for c, v in mixed["kernels"].items() if c in bpp}
    dom = max(cands, key=lambda c: cands[c]["total_ms"])
    bytes_per_launch = bpp[dom] * n_unk
    achieved = bytes_per_launch / (cands[dom]["avg_ms"] / 1e3) / 1e9
    kernels = {f"{prec}:{c}": v for prec, leg in legs.items() for c, v in kernel_table(leg["kernels"], prec, n_unk).items()}

    out = {
        "metric": "fine-grid unknowns solved/s to 1e-8 rel res (mixed vs FP64) + stencil HBM GB/s",
        "value": value,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+bf16 V-cycle, f64 outer",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {w['desc']}", "n": n, "levels": levels,
                   "unknowns": n_unk, "switch_n": args.switch_n, "post_fused": args.post_fused, "rtol": args.rtol,
                   "step": "setup + mixed PCG solve + adjoint gradient"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_for(dom, args.workload),
                     "bytes_per_launch": bytes_per_launch, "avg_ms": cands[dom]["avg_ms"],
                     "copy_GBs": copy_gbs, "copy_march_GBs": copy_march},
        "T_solve": {"definition": "median of 5 forward solves from x0 = 0, setup excluded (HIP events)",
                    "mixed_ms": mixed["T_solve_ms"], "mixed_unknowns_per_s": n_unk / (mixed["T_solve_ms"] / 1e3)},
        "forward": {"iterations": mixed["forward"]["iterations"], "rel_res_true": mixed["forward"]["rel_res_true"],
                    "restarts": mixed["forward"]["restarts"], "solve_ms": mixed["forward"]["solve_ms"]},
        "adjoint": {"iterations": mixed["adjoint"]["iterations"], "solve_ms": mixed["adjoint"]["solve_ms"],
                    "rel_res_true": mixed["adjoint"]["rel_res_true"]},
        "error_vs_oracle": {p: legs[p]["error_vs_oracle"] for p in legs},
        "kernels": kernels,
    }
    if "fp64" in legs:
        f64 = legs["fp64"]
        out["T_solve"].update({"fp64_ms": f64["T_solve_ms"], "fp64_unknowns_per_s": n_unk / (f64["T_solve_ms"] / 1e3),
                               "speedup_mixed": f64["T_solve_ms"] / mixed["T_solve_ms"]})
        out["fp64"] = {"ms_per_step": f64["ms_per_step"], "value": 2 * n_unk / (f64["ms_per_step"] / 1e3),
                       "forward_iterations": f64["forward"]["iterations"],
                       "forward_solve_ms": f64["forward"]["solve_ms"],
                       "rel_res_true": f64["forward"]["rel_res_true"],
                       "speedup_mixed": f64["ms_per_step"] / ms,
                       "speedup_mixed_forward": f64["forward"]["solve_ms"] / mixed["forward"]["solve_ms"]}
        d = torch.linalg.vector_norm(results["mixed"] - results["fp64"]) / torch.linalg.vector_norm(results["fp64"])
        out["fp64"]["mixed_vs_fp64_rel_l2"] = float(d)
    del results, k, kobs, f
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        its = legs.get("fp64", mixed)["forward"]["iterations"]
        log("timing the CPU oracle sample ...")
        out["cpu_baseline"] = cpu_baseline(w, [_host(a) for a in k_in], _host(f_in), its, iters=args.cpu_iters)
    del k_in, f_in
    if not args.no_agglomeration:
        out["agglomeration"] = agglomeration_sweep(args.rtol)
        p33 = out["agglomeration"]["poisson33"]["argmin"]["fp64"]
        out["config1_fp64_unknowns_per_s"] = p33["unknowns_per_s"]
    if not args.no_large:
        out["large"] = large_block(args.rtol, args.switch_n)
    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
