#!/usr/bin/env python3
"""Benchmark of the multigrid-preconditioned CG hot path on one MI355X.

Workload (default "inclusions513"): -div(k grad phi) = f on a 513^3 vertex grid
(511^3 = 133,432,831 unknowns), two-phase k (random spheres, radius 4-16 cells,
20 % volume, k = 1e3 inside, 1 outside), f ~ U(-1,1), 9 levels (coarsest 3^3),
Chebyshev-Jacobi degree 2 pre/post, levels N <= 17 agglomerated into the
persistent coarse kernel.

One step = the whole hot path once:
  hierarchy setup from k  ->  mixed-precision PCG solve to an FP64 relative
  residual of 1e-8  ->  adjoint gradient dL/d ln k for L = 0.5 ||phi - phi_obs||^2
  (adjoint PCG solve + link-gradient kernel).
value = fine-grid unknowns solved per second = 2 solves x 511^3 / step time.
The same step in plain FP64 is timed beside it (speedup, error).

Inputs are generated on the host and copied to HBM before the timed region.
Kernel durations come from HIP events the library records around every
finest-level launch on its stream during the timed steps.
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
             "restrict": 5, "prolong": 17, "face_gradient": 64, "cheb_post2": 56},
    "mixed": {"apply_dot": 36, "residual": 48, "update_r": 28, "update_xp": 28, "update_p": 8, "cheb_first": 20, "cheb_pre2": 18,
              "cheb_step": 18, "cheb_step_prev": 22, "cheb_step_dot": 30, "level_residual": 16,
              "restrict": 2.5, "prolong": 8.5, "face_gradient": 64, "cheb_post2": 26},
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


def run_steps(solver, k, f, phi_obs, steps, rtol, profile=False):
    """Time `steps` full steps; returns (seconds per step list, last infos, profile dict)."""
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
    if prof:
        prof.__exit__(None, None, None)
    return times, fwd, adj, (prof.result if prof else {}), phi


def copy_bandwidth(nbytes=2 << 30, reps=5):
    """Achievable HBM bandwidth of a plain streaming copy (read + write bytes / time)."""
    import torch
    from paper_1604_07163_amd import gmg
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    gmg.calibration_copy(b, a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        gmg.calibration_copy(b, a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms / 1e3) / 1e9


def cpu_baseline(w, k, f, its_needed, iters=2):
    """Time the FP64 CPU oracle for `iters` PCG iterations at the full size and
    scale to the iteration count the solve needs (setup not timed)."""
    import oracle
    oracle.build(force=False)
    H = oracle.Hierarchy(*k, levels=w["levels"])
    t0 = time.perf_counter()
    _, info = H.solve(f, rtol=1e-8, max_it=iters)
    dt = time.perf_counter() - t0
    H.close()
    per_it = dt / max(info["iterations"], 1)
    t_solve = per_it * its_needed
    n_unk = (w["n"] - 2) ** 3
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    return {"value": n_unk / t_solve, "unit": "unknowns/s", "cores": cores, "kind": "oracle",
            "sample": f"{info['iterations']} FP64 PCG iterations of the oracle at {w['n']}^3 "
                      f"({dt:.1f} s, setup excluded), scaled to the {its_needed} iterations of one solve",
            "seconds_per_iteration": per_it}


def sweep(args):
    """Switch-level sweep (grid launches vs the persistent coarse kernel) and the
    truncation arm, forward solves on the chosen workload; prints one JSON line."""
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
    for cfg in configs:
        kw = dict(cfg)
        lv = kw.pop("levels", levels)
        s = gmg.Solver(*k, levels=lv, **kw)
        s.solve(f, rtol=args.rtol, max_it=3000)
        ts, info = [], None
        for _ in range(max(1, args.steps)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, info = s.solve(f, rtol=args.rtol, max_it=3000)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        with gmg.Profile(s) as pr:
            s.solve(f, rtol=args.rtol, max_it=3000)
        coarse = pr.result.get("persistent") or pr.result.get("coarse_solve") or {}
        row = {"levels": lv, **cfg, "iterations": info["iterations"], "coarse_iterations": info["coarse_iterations"],
               "ms": 1e3 * float(np.median(ts)), "ms_per_iteration": 1e3 * float(np.median(ts)) / info["iterations"],
               "coarse_kernel_us": 1e3 * coarse.get("avg_ms", 0.0), "rel_res_true": info["rel_res_true"],
               "setup_ms": info["setup_ms"], "lds_bytes": s.persistent_lds_bytes}
        log(json.dumps(row))
        rows.append(row)
        s.close()
    print(json.dumps({"workload": args.workload, "n": n, "rtol": args.rtol, "rows": rows}), flush=True)


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
    "apply_dot": "k_apply_x2<true, float>",
    "update_r": "k_update_r<float>",
    "update_xp": "k_update_xp<float, float>",
    "cheb_pre2": "k_cheb_pre2<float, bf16, false>",
    "cheb_step": "k_cheb_step<float, bf16, 0, false>",
    "cheb_step_dot": "k_cheb_step<float, bf16, 2, true>",
    "cheb_post2": "k_post2<float, bf16, true, 8>",
    "level_residual": "k_residual_zr<float, bf16>",
    "restrict": "k_restrict_xy<float>",
    "prolong": "k_prolong<float>",
}
def traffic_file(workload):
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.md")
COPY_BYTES = 2 << 30  # copy_bandwidth(): bytes read (and written) per calibration copy


def source_digest():
    """sha256 of the kernel and driver sources: counter figures hold for this build only."""
    import hashlib
    hsh = hashlib.sha256()
    for rel in ("paper_1604_07163_amd/csrc/kernels.hpp", "paper_1604_07163_amd/csrc/gmg.hip"):
        with open(os.path.join(ROOT, rel), "rb") as fh:
            hsh.update(fh.read())
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
        cp = vals[c]["k_copy_flat"]
        scale[c] = COPY_BYTES / (1024.0 * sum(cp) / len(cp))
    lines = [f"source_digest: {source_digest()}",
             f"calibration: k_copy_flat of {COPY_BYTES} bytes; FETCH_SIZE x {scale['FETCH_SIZE']:.4f}, "
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
    ap.add_argument("--galerkin", type=int, nargs="*", default=[],
                    help="with --sweep: also time Galerkin coarse operators from these first levels")
    ap.add_argument("--post-fused", default="auto", choices=["auto", "0", "1"],
                    help="one-sweep post-smoothing: auto (the library default: one sweep), 0 two sweeps, 1 one sweep")
    args = ap.parse_args()
    if args.profile_summary:
        profile_summary(args.profile_summary)
        return
    if args.pmc_traffic:
        pmc_traffic(*args.pmc_traffic)
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
    log(f"plain copy: {copy_gbs:.0f} GB/s")
    legs = {}
    results = {}
    for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64"]):
        s = gmg.Solver(*k, levels=levels, precision=prec, switch_n=args.switch_n,
                       post_fused="auto" if args.post_fused == "auto" else args.post_fused == "1")
        # phi_obs: forward solve with the observation coefficients (untimed)
        s.set_coefficients(*kobs)
        phi_obs, _ = s.solve(f, rtol=1e-10, max_it=2000)
        s.set_coefficients(*k)
        steps = args.steps if prec == "mixed" else max(1, (args.steps + 1) // 2)
        run_steps(s, k, f, phi_obs, args.warmup, args.rtol)
        log(f"[{prec}] warmup done; timing {steps} steps")
        times, fwd, adj, prof, phi = run_steps(s, k, f, phi_obs, steps, args.rtol, profile=True)
        legs[prec] = {"ms_per_step": 1e3 * float(np.mean(times)), "ms_min": 1e3 * float(np.min(times)),
                      "forward": fwd, "adjoint": adj, "kernels": prof}
        results[prec] = phi.clone()
        log(f"[{prec}] {legs[prec]['ms_per_step']:.1f} ms/step; fwd its {fwd['iterations']} "
            f"true {fwd['rel_res_true']:.2e}; adj its {adj['iterations']}")
        s.close()
        del s
        torch.cuda.empty_cache()

    mixed = legs["mixed"]
    ms = mixed["ms_per_step"]
    value = 2 * n_unk / (ms / 1e3)
    # dominant finest-level HBM kernel of the mixed step
    bpp = BYTES_PER_POINT["mixed"]
    cands = {c: v for c, v in mixed["kernels"].items() if c in bpp}
    dom = max(cands, key=lambda c: cands[c]["total_ms"])
    bytes_per_launch = bpp[dom] * n_unk
    achieved = bytes_per_launch / (cands[dom]["avg_ms"] / 1e3) / 1e9
    kernels = {}
    for prec, leg in legs.items():
        for c, v in leg["kernels"].items():
            entry = dict(v)
            if c in BYTES_PER_POINT[prec]:
                entry["GBs"] = BYTES_PER_POINT[prec][c] * n_unk / (v["avg_ms"] / 1e3) / 1e9
                entry["frac_peak"] = entry["GBs"] / HBM_PEAK_GBS
            kernels[f"{prec}:{c}"] = entry

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
                     "copy_GBs": copy_gbs},
        "forward": {"iterations": mixed["forward"]["iterations"], "rel_res_true": mixed["forward"]["rel_res_true"],
                    "restarts": mixed["forward"]["restarts"], "solve_ms": mixed["forward"]["solve_ms"]},
        "adjoint": {"iterations": mixed["adjoint"]["iterations"], "solve_ms": mixed["adjoint"]["solve_ms"]},
        "kernels": kernels,
    }
    if "fp64" in legs:
        f64 = legs["fp64"]
        out["fp64"] = {"ms_per_step": f64["ms_per_step"], "value": 2 * n_unk / (f64["ms_per_step"] / 1e3),
                       "forward_iterations": f64["forward"]["iterations"],
                       "forward_solve_ms": f64["forward"]["solve_ms"],
                       "rel_res_true": f64["forward"]["rel_res_true"],
                       "speedup_mixed": f64["ms_per_step"] / ms,
                       "speedup_mixed_forward": f64["forward"]["solve_ms"] / mixed["forward"]["solve_ms"]}
        d = torch.linalg.vector_norm(results["mixed"] - results["fp64"]) / torch.linalg.vector_norm(results["fp64"])
        out["fp64"]["mixed_vs_fp64_rel_l2"] = float(d)
    if not args.no_cpu_baseline:
        its = legs.get("fp64", mixed)["forward"]["iterations"]
        log("timing the CPU oracle sample ...")
        out["cpu_baseline"] = cpu_baseline(w, [_host(a) for a in k_in], _host(f_in), its, iters=args.cpu_iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
