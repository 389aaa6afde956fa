"""Benchmark: RHS solved per second at relative residual 1e-6 on one MI355X.

Workload (default): 1024 x 1024 physical cells, h = 1/1024, omega = 2 pi 40,
seeded layered medium (6 layers, 1.5 -> 4.5, 5% smoothed noise), 8 x 8
subdomains, PML 20, overlap 10, 16 surface Gaussian shots; flexible GMRES
right-preconditioned by one diagonal-sweep application per iteration, stopped
per RHS at true FP64 relative residual 1e-6.  A step is one such batched solve
of all 16 RHS with the factors resident in HBM (factorisation reported
separately).  `value` is the complex64-factor + FP64-refinement path over
the K timed steps (default 5; every step's time and their median are given,
and end_to_end_s = factorisation + the median step); the plain complex128
path is measured beside it.

Prints one JSON line.  --gpus must be 1 (this build runs on one GPU).
"""
import argparse
import json
import math
import statistics
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

HBM_PEAK_GBS = 8000.0
FP32_MATRIX_PEAK_TFLOPS = 157.3   # dense FP32 MFMA (the complex64 factors)
FP64_VECTOR_PEAK_TFLOPS = 78.6    # FP64 vector FMA (the complex128 solves)


def _inputs(name):
    import synth
    w = synth.workload(name)
    c = synth.medium_for(w)
    f = synth.sources_for(w)
    pml = w.pml
    F = np.stack([np.pad(s, pml) for s in f]).astype(np.complex128)
    return w, c, F


def _plan(w, c, prec, kg, graph=False, tune=False):
    import torch
    import paper_2002_05327_amd as dsw
    m = torch.from_numpy(1.0 / c ** 2).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = dsw.Plan(n=w.n, h=w.h, omega=w.omega, pml=w.pml, overlap=w.overlap, parts=w.parts,
                    m=m, precision=prec, max_rhs=w.nrhs, rhs_per_group=kg)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"# {prec} plan ready ({plan.local_solver} local solver): factorisation {dt:.2f} s",
          file=sys.stderr, flush=True)
    if tune:
        t1 = time.perf_counter()
        res = plan.autotune()
        print(f"# {prec} autotune {time.perf_counter() - t1:.2f} s -> {res}", file=sys.stderr,
              flush=True)
    if graph:
        plan.use_graph(True)
    return plan, dt


def _solve_steps(plan, b, tol, maxit, restart, warmup, steps):
    import torch
    for _ in range(warmup):
        plan.gmres(b, tol=tol, maxit=maxit, restart=restart)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = None
    marks = [t0]
    for _ in range(steps):
        last = plan.gmres(b, tol=tol, maxit=maxit, restart=restart)   # returns host values: synchronised
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    x, its, rel, ok = last
    step_ms = [round((marks[i + 1] - marks[i]) * 1e3, 3) for i in range(steps)]
    return dt, its, rel, ok, x[0].cpu().numpy().ravel(), step_ms


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_bcr_c2_traffic.md")


def _kernel_source_hash():
    """sha256 over the source that decides the solve kernel's memory traffic: the
    kernel and its launchers, and the builder of its job tables and launch shapes."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2002_05327_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "kernels.hip")) as f:
        k = f.read()
    a, b = k.index("// ---- solve jobs"), k.index("// a4: local right-hand sides")
    h.update(k[a:b].encode())
    with open(os.path.join(csrc, "plan.hip")) as f:
        p = f.read()
    a = p.index("void bcr_group_jobs(const dsd_plan* pl, const std::vector<int2>& mem, std::vector<BcrJob>& jobs,\n                    std::vector<BcrLaunch>& out) {")
    b = p.index("\n}\n", a)
    h.update(p[a:b].encode())
    a = p.index("  int cg_wide = ")
    h.update(p[a:p.index("\n", p.index("int wide_kg", a))].encode())
    return h.hexdigest()


def _measured_traffic(workload):
    """HBM bytes per solve-kernel dispatch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE passes, each scaled by what the counter
    reads for a 1 GiB device copy); None when the summary was taken on another
    workload or before the kernels last changed."""
    try:
        vals = {}
        with open(TRAFFIC_FILE) as f:
            for line in f:
                if ":" in line and line.startswith("- "):
                    k, v = line[2:].split(":", 1)
                    vals[k.strip()] = v.strip().strip("`")
        if vals.get("workload") != workload or vals.get("solve-kernel source sha256") != _kernel_source_hash():
            return None
        return float(vals["HBM bytes per dispatch"])
    except (OSError, KeyError, ValueError):
        return None


def _roofline(plan, b, workload, matrix_peak=None):
    """Average duration, algorithmic bytes and flops of the subdomain-solve
    launches over one preconditioner application, timed with HIP events on the
    plan's stream.  The binding roof is the one whose ideal time is longer: HBM
    for few right-hand sides (C2: 16), the FP32 matrix cores when the
    right-hand-side count passes the ridge (C3, C4r); the other is reported
    beside it.  With matrix_peak (the complex128 path, vector FP64 FMAs) the
    compute roof is that ALU peak instead."""
    import torch
    plan.timing(True)
    plan.sweep_apply(b)
    torch.cuda.synchronize()
    t = plan.timing_read()
    plan.timing(False)
    nl = max(1, t["solve_launches"])
    avg_ms = t["solve_ms"] / nl
    avg_bytes = t["solve_bytes"] / nl
    avg_flops = t["solve_flops"] / nl
    gbs = avg_bytes / (avg_ms * 1e-3) / 1e9
    tfs = avg_flops / (avg_ms * 1e-3) / 1e12
    hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4)}
    peak_tf = FP32_MATRIX_PEAK_TFLOPS if matrix_peak is None else matrix_peak
    mfma = {"bound": "mfma" if matrix_peak is None else "alu", "achieved": round(tfs, 2),
            "peak": peak_tf, "unit": "TFLOP/s", "frac": round(tfs / peak_tf, 4)}
    mfma_bound = avg_flops / (peak_tf * 1e12) > avg_bytes / (HBM_PEAK_GBS * 1e9)
    out = dict(mfma if mfma_bound else hbm)
    out.update({"traffic": _measured_traffic(workload) if matrix_peak is None else None,
                "kernel": {"bcr": "k_bcr (block cyclic reduction solves)",
                           "chain": "k_chain (block LDL^T chain solves)",
                           "chain-steps": "k_bcr (block LDL^T chain steps)"}[plan.local_solver],
                "launches": t["solve_launches"],
                "avg_launch_ms": round(avg_ms, 4), "avg_launch_bytes": round(avg_bytes),
                "avg_launch_flops": round(avg_flops),
                "other_roof": hbm if mfma_bound else mfma,
                "traffic_unit": "HBM bytes per dispatch"})
    return out


def _cpu_baseline(w, c, F):
    """The FP64 oracle (numpy/scipy) on one host core: DDM-preconditioned FGMRES
    for one RHS of the same workload; the local factorisations are excluded
    (as on the GPU side, where factors are resident)."""
    from threadpoolctl import threadpool_limits
    from oracle.krylov import fgmres
    from oracle.sweep import DiagonalSweepDDM
    with threadpool_limits(limits=1):
        ddm = DiagonalSweepDDM(w.n, w.h, w.omega, w.pml, w.overlap, w.parts, 1.0 / c ** 2)
        b = F[0].ravel()
        t0 = time.perf_counter()
        x, its, hist = fgmres(lambda v: ddm.M @ v, ddm.apply, b, tol=1e-6, restart=30, maxit=60)
        dt = time.perf_counter() - t0
    return {"value": round(1.0 / dt, 5), "unit": "RHS/s", "cores": 1, "kind": "oracle",
            "sample": f"1 of the {w.nrhs} RHS, FGMRES to 1e-6 ({its} iterations, relres "
                      f"{hist[-1]:.1e}) in {dt:.1f} s; local factorisations excluded; "
                      f"SuperLU, scipy.sparse and BLAS on one thread",
            "host_cpu": _host_cpu(), "host_logical_cpus": os.cpu_count()}


def _host_cpu():
    """Model name of the host CPU (from /proc/cpuinfo; empty if unavailable)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return ""


def _oracle_error(w, c, F, sols):
    """Relative error of the timed solutions of RHS 0 (at the benchmark's
    tolerance) against the oracle's global sparse LU solution of the same
    PML problem (2D workloads up to 2M unknowns; null otherwise)."""
    N = int(np.prod([k + 2 * w.pml for k in w.n]))
    if w.dim != 2 or N > 2_000_000:
        return None
    from oracle.pml import assemble, global_axes
    from oracle.sweep import global_solve
    M = assemble(global_axes(w.n, w.pml, w.h), 1.0 / c ** 2, w.h, w.omega, w.pml)
    u = global_solve(M, F[0].ravel())
    out = {"reference": "oracle global sparse LU, RHS 0"}
    for k, x in sols.items():
        if x is not None:
            out[k] = float(np.linalg.norm(x - u) / np.linalg.norm(u))
    return out


def _copy_probe(gib=1.0):
    """A plain device copy of known size, whose FETCH_SIZE / WRITE_SIZE counters
    calibrate the per-dispatch byte counts of the other kernels."""
    import torch
    n = int(gib * 2 ** 30) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--maxit", type=int, default=60)
    ap.add_argument("--restart", type=int, default=30)
    ap.add_argument("--kg", type=int, default=0, help="RHS per workgroup in the block solves")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time the solve-launch shapes first (reported separately)")
    ap.add_argument("--graph", action="store_true",
                    help="run preconditioner applications as captured HIP graphs")
    ap.add_argument("--no-c128", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run a 1 GiB device copy first (calibrates PMC byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if args.copy_probe:
        _copy_probe()
    w, c, F = _inputs(args.workload)
    b = torch.from_numpy(F).cuda()
    print(f"# workload {w.name}: n={w.n} parts={w.parts} nrhs={w.nrhs}", file=sys.stderr, flush=True)

    plan64, tf64 = _plan(w, c, "c64", args.kg, args.graph, args.autotune)
    print(f"# c64 factorisation {tf64:.2f} s", file=sys.stderr, flush=True)
    dt64, its64, rel64, ok64, x64, steps64 = _solve_steps(plan64, b, args.tol, args.maxit,
                                                          args.restart, args.warmup, args.steps)
    print(f"# c64 solve {dt64 / args.steps * 1e3:.1f} ms/step iters {its64}", file=sys.stderr,
          flush=True)
    roof = _roofline(plan64, b, w.name)
    info64 = plan64.info()
    plan64.close()
    del plan64

    c128 = None
    if not args.no_c128:
        plan128, tf128 = _plan(w, c, "c128", args.kg, args.graph, args.autotune)
        n128 = max(1, min(args.steps, 5))
        dt128, its128, rel128, ok128, x128, steps128 = _solve_steps(
            plan128, b, args.tol, args.maxit, args.restart, min(args.warmup, 1), n128)
        c128 = {"value": round(w.nrhs * n128 / dt128, 3), "unit": "RHS/s",
                "ms_per_step": round(dt128 / n128 * 1e3, 2),
                "median_ms_per_step": round(statistics.median(steps128), 2),
                "factor_s": round(tf128, 3),
                "iters": its128, "max_relres": max(rel128), "converged": ok128}
        print(f"# c128 solve {dt128 / n128 * 1e3:.1f} ms/step iters {its128}", file=sys.stderr,
              flush=True)
        c128["roofline"] = _roofline(plan128, b, w.name, FP64_VECTOR_PEAK_TFLOPS)
        plan128.close()
        del plan128

    cpu = None
    err = None
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu = _cpu_baseline(w, c, F)
        print("# error against the oracle's global solve ...", file=sys.stderr, flush=True)
        err = _oracle_error(w, c, F, {"c64": x64, "c128": None if c128 is None else x128})

    value = w.nrhs * args.steps / dt64
    out = {
        "metric": "RHS solved/sec at rel. residual 1e-6; batched c64+FP64-IR vs plain FP64 path",
        "value": round(value, 3), "unit": "RHS/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt64 / args.steps * 1e3, 2),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "c64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {'x'.join(map(str, w.n))} {w.medium} medium, "
                               f"omega=2pi*{w.omega / (2 * math.pi):g}, "
                               f"{'x'.join(map(str, w.parts))} subdomains, PML {w.pml}, overlap "
                               f"{w.overlap}, {w.nrhs} RHS, FGMRES(restart {args.restart}) to "
                               f"{args.tol:g}",
                   "global_batch": w.nrhs, "precision": "c64 factors + FP64 refinement"},
        "iters": its64, "max_relres": max(rel64), "converged": ok64,
        "median_ms_per_step": round(statistics.median(steps64), 2), "step_ms": steps64,
        "factor_s": round(tf64, 3), "factor_bytes": info64["factor_bytes"],
        "end_to_end_s": round(tf64 + statistics.median(steps64) * 1e-3, 3),
        "c128": c128, "rel_err_vs_oracle": err, "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
