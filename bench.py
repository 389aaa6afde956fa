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


def _plan(w, c, prec, kg, graph=False, tune=False, solver="auto", nd_leaf=0, nd_top=0, nd_wide=0,
          nd_wave=0, nd_fuse=0):
    import torch
    import paper_2002_05327_amd as dsw
    m = torch.from_numpy(1.0 / c ** 2).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = dsw.Plan(n=w.n, h=w.h, omega=w.omega, pml=w.pml, overlap=w.overlap, parts=w.parts,
                    m=m, precision=prec, max_rhs=w.nrhs, rhs_per_group=kg, local_solver=solver,
                    nd_leaf=nd_leaf, nd_top_cells=nd_top, nd_wide=nd_wide, nd_wave_steps=nd_wave,
                    nd_fuse=nd_fuse)
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


TRAFFIC_FILES = {"bcr": os.path.join(ROOT, "profiles", "k_bcr_c2_traffic.md"),
                 "nd": os.path.join(ROOT, "profiles", "k_nd_c2_traffic.md")}


def _kernel_source_hash(solver="bcr"):
    """sha256 over the source that decides the solve kernels' memory traffic: the
    kernels and their launchers, and the builder of their job tables and launch
    shapes."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2002_05327_amd", "csrc")
    h = hashlib.sha256()
    with open(os.path.join(csrc, "plan.hip")) as f:
        p = f.read()
    if solver == "nd":
        with open(os.path.join(csrc, "nd.hip")) as f:
            k = f.read()
        h.update(k[k.index("// Solve kernels"):k.index("// Factorisation kernels")].encode())
        a = p.index("void nd_group_jobs(")
        h.update(p[a:p.index("\n}\n", a)].encode())
        a = p.index("void nd_shape(")                 # launch shapes and the solve phase
        h.update(p[a:p.index("\n}\n", p.index("void nd_phase(", a))].encode())
        return h.hexdigest()
    with open(os.path.join(csrc, "kernels.hip")) as f:
        k = f.read()
    a, b = k.index("// ---- solve jobs"), k.index("// a4: local right-hand sides")
    h.update(k[a:b].encode())
    a = p.index("void bcr_group_jobs(const dsd_plan* pl, const std::vector<int2>& mem, std::vector<BcrJob>& jobs,\n                    std::vector<BcrLaunch>& out) {")
    b = p.index("\n}\n", a)
    h.update(p[a:b].encode())
    a = p.index("  int cg_wide = ")
    h.update(p[a:p.index("\n", p.index("int wide_kg", a))].encode())
    return h.hexdigest()


def _measured_traffic(workload, solver):
    """HBM bytes per solve-kernel dispatch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE passes, each scaled by what the counter
    reads for a 1 GiB device copy); None when the summary was taken on another
    workload or before the kernels last changed."""
    if solver not in TRAFFIC_FILES:
        return None
    try:
        vals = {}
        with open(TRAFFIC_FILES[solver]) as f:
            for line in f:
                if ":" in line and line.startswith("- "):
                    k, v = line[2:].split(":", 1)
                    vals[k.strip()] = v.strip().strip("`")
        if vals.get("workload") != workload or \
                vals.get("solve-kernel source sha256") != _kernel_source_hash(solver):
            return None
        return float(vals["HBM bytes per dispatch"])
    except (OSError, KeyError, ValueError):
        return None


def band_work(plan, w, nrhs, tsize):
    """The algorithmic work of one preconditioner application's local solves, as
    the band solve counts it: every one of the 2^dim * N_sub solves streams its
    band LU factor once for the whole RHS block -- N_loc (2b + 1) complex entries,
    b the band half-width (the shorter local dimension in 2D, the product of the
    two shorter ones in 3D) -- and moves 4 N_loc vector entries per RHS (read
    the right-hand side and write the solution, each once per triangular
    sweep); 16 N_loc b real flops per RHS.  Returns (bytes, flops)."""
    nsub = int(np.prod(w.parts))
    sweeps = 2 ** w.dim
    fac = vec = flops = 0.0
    for sid in range(nsub):
        dims, _ = plan.subdomain_grid(sid)
        dims = sorted(dims[:w.dim])
        nloc = float(np.prod(dims))
        bw = float(dims[0] if w.dim == 2 else dims[0] * dims[1])
        fac += sweeps * nloc * (2 * bw + 1) * tsize
        vec += sweeps * 4 * nloc * tsize * nrhs
        flops += sweeps * 16 * nloc * bw * nrhs
    return fac + vec, flops


def _roofline(plan, b, w, tsize, matrix_peak=None):
    """Roofline of the subdomain-solve kernel over one preconditioner application.

    achieved = the algorithmic bytes (band_work: band-LU factor once per RHS
    block plus the vectors, summed over the application's local solves) divided
    by the summed device time of the solve launches, timed with a pair of HIP
    events around every launch on the plan's stream; the same over the flops
    for the compute roof.  The binding roof is the one whose ideal time is
    longer (HBM for C2's 16 RHS, the matrix cores past the ridge); the other is
    reported beside it.  kernel_format_bytes is the library's own count of the
    bytes its factor format has to stream (a diagnostic).  With matrix_peak (the
    complex128 path, vector FP64 FMAs) the compute roof is that ALU peak."""
    import torch
    plan.timing(True)
    plan.sweep_apply(b)
    torch.cuda.synchronize()
    t = plan.timing_read()
    plan.timing(False)
    nl = max(1, t["solve_launches"])
    k = b.shape[0]
    app_bytes, app_flops = band_work(plan, w, k, tsize)
    sec = t["solve_ms"] * 1e-3
    gbs = app_bytes / sec / 1e9
    tfs = app_flops / sec / 1e12
    hbm = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gbs / HBM_PEAK_GBS, 4)}
    peak_tf = FP32_MATRIX_PEAK_TFLOPS if matrix_peak is None else matrix_peak
    mfma = {"bound": "mfma" if matrix_peak is None else "alu", "achieved": round(tfs, 2),
            "peak": peak_tf, "unit": "TFLOP/s", "frac": round(tfs / peak_tf, 4)}
    mfma_bound = app_flops / (peak_tf * 1e12) > app_bytes / (HBM_PEAK_GBS * 1e9)
    out = dict(mfma if mfma_bound else hbm)
    out.update({"traffic": _measured_traffic(w.name, plan.local_solver) if matrix_peak is None else None,
                "kernel": KERNEL_NAMES[plan.local_solver],
                "launches": t["solve_launches"],
                "solve_ms_per_application": round(t["solve_ms"], 3),
                "avg_launch_ms": round(t["solve_ms"] / nl, 4),
                "avg_launch_bytes": round(app_bytes / nl),
                "avg_launch_flops": round(app_flops / nl),
                "other_roof": hbm if mfma_bound else mfma,
                "traffic_unit": "HBM bytes per dispatch",
                "algorithmic_bytes": "band LU: N_loc (2b+1) factor entries per solve per RHS "
                                     "block + 4 N_loc entries per RHS",
                "kernel_format_bytes_per_launch": round(t["solve_bytes"] / nl),
                "kernel_format_GBps": round(t["solve_bytes"] / sec / 1e9, 1)})
    # the same launches against the work the local solver's own factor format
    # implies (its factor bytes once per launch plus the vectors; 8 flops per
    # factor entry and RHS): with nested dissection that is less than the band
    # solve's, so the band-based fraction can pass 1 (full C4)
    fgbs, ftfs = t["solve_bytes"] / sec / 1e9, t["solve_flops"] / sec / 1e12
    f_mfma = t["solve_flops"] / (peak_tf * 1e12) > t["solve_bytes"] / (HBM_PEAK_GBS * 1e9)
    out["format"] = ({"bound": out["bound"] if matrix_peak is not None else "mfma",
                      "achieved": round(ftfs, 2), "peak": peak_tf, "unit": "TFLOP/s",
                      "frac": round(ftfs / peak_tf, 4)} if f_mfma else
                     {"bound": "hbm", "achieved": round(fgbs, 1), "peak": HBM_PEAK_GBS,
                      "unit": "GB/s", "frac": round(fgbs / HBM_PEAK_GBS, 4)})
    return out


KERNEL_NAMES = {"bcr": "k_bcr (block cyclic reduction solves)",
                "chain": "k_chain (block LDL^T chain solves)",
                "chain-steps": "k_bcr (block LDL^T chain steps)",
                "nd": "k_nd_fwd + k_nd_top + k_nd_bwd (nested-dissection solves)"}


_CPU = {}


def _cpu_worker(i):
    """One RHS of the oracle's DDM-preconditioned FGMRES on one thread (pool worker;
    the factors come from the parent by fork)."""
    from threadpoolctl import threadpool_limits
    from oracle.krylov import fgmres
    ddm, F = _CPU["ddm"], _CPU["F"]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        x, its, hist = fgmres(lambda v: ddm.M @ v, ddm.apply, F[i].ravel(), tol=1e-6, restart=30,
                              maxit=60)
        return its, hist[-1], time.perf_counter() - t0


def _cpu_baseline(w, c, F):
    """The FP64 oracle (numpy/scipy, as it stands) on the host cores, with the
    phases of the method timed separately: the local factorisations (one sparse
    LU per subdomain), the global sparse LU of the whole PML problem (the
    reference the error is measured against), and the DDM-preconditioned FGMRES
    solves.  The solves run one worker process per core over the RHS (factors
    shared by fork; one BLAS thread each): `value` is that throughput, with the
    single-RHS time of one worker beside it.  Runs before the GPU is touched,
    so the workers fork from a process without a GPU context."""
    import multiprocessing as mp
    from threadpoolctl import threadpool_limits
    from oracle.sweep import DiagonalSweepDDM
    out = {"kind": "oracle", "unit": "RHS/s", "host_cpu": _host_cpu(),
           "host_logical_cpus": os.cpu_count()}
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        ddm = DiagonalSweepDDM(w.n, w.h, w.omega, w.pml, w.overlap, w.parts, 1.0 / c ** 2)
        out["local_factor_s"] = round(time.perf_counter() - t0, 2)
        u_glob = None
        N = int(np.prod([k + 2 * w.pml for k in w.n]))
        if w.dim == 2 and N <= 2_000_000:
            from oracle.sweep import global_solve
            t0 = time.perf_counter()
            u_glob = global_solve(ddm.M, F[0].ravel())
            out["global_splu_s"] = round(time.perf_counter() - t0, 2)
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    workers = max(1, min(16, ncpu, w.nrhs))
    _CPU.update(ddm=ddm, F=F)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_cpu_worker, range(w.nrhs))
    wall = time.perf_counter() - t0
    _CPU.clear()
    its = [r[0] for r in res]
    per = [r[2] for r in res]
    out.update({
        "value": round(w.nrhs / wall, 5), "cores": workers,
        "sample": f"all {w.nrhs} RHS, FGMRES to 1e-6 ({min(its)}-{max(its)} iterations, relres "
                  f"<= {max(r[1] for r in res):.1e}) in {wall:.1f} s wall on {workers} worker "
                  f"processes (one BLAS thread each); local factorisations and global LU timed "
                  f"separately",
        "ddm_gmres_wall_s": round(wall, 2),
        "single_core_rhs_per_s": round(1.0 / statistics.median(per), 5),
    })
    return out, u_glob


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


def _oracle_error(u, sols):
    """Relative error of the timed solutions of RHS 0 (at the benchmark's
    tolerance) against the oracle's global sparse LU solution of the same PML
    problem (2D workloads up to 2M unknowns; null otherwise)."""
    if u is None:
        return None
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
    ap.add_argument("--restart", type=int, default=0, help="FGMRES restart (0: the workload's)")
    ap.add_argument("--kg", type=int, default=0, help="RHS per workgroup in the block solves")
    ap.add_argument("--solver", default="", help="local solver: auto, nd, bcr, chain, chain-steps "
                                                 "(default: the workload's)")
    ap.add_argument("--nd-leaf", type=int, default=0, help="nested dissection: leaf box cells (0: library)")
    ap.add_argument("--nd-top", type=int, default=0, help="nested dissection: dense-top cells (0: library)")
    ap.add_argument("--nd-wide", type=int, default=0,
                    help="nested dissection: fronts of at least this many cells in wide mode (0: library)")
    ap.add_argument("--nd-wave", type=int, default=0,
                    help="nested dissection: 64-lane steps up to which a level runs a node per wave (0: library)")
    ap.add_argument("--nd-fuse", type=int, default=0,
                    help="nested dissection: front size below which subtree levels run fused (0: library; 1: off)")
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
    w, c, F = _inputs(args.workload)
    if args.restart <= 0:
        args.restart = w.restart
    if not args.solver:
        args.solver = w.solver
    cpu, u_glob = None, None
    if not args.no_cpu_baseline:
        # before any GPU call: the oracle's worker processes fork from this one
        print("# cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        cpu, u_glob = _cpu_baseline(w, c, F)
        print(f"# cpu baseline: {cpu['value']} RHS/s on {cpu['cores']} cores", file=sys.stderr,
              flush=True)
    import torch
    if args.copy_probe:
        _copy_probe()
    b = torch.from_numpy(F).cuda()
    print(f"# workload {w.name}: n={w.n} parts={w.parts} nrhs={w.nrhs}", file=sys.stderr, flush=True)

    plan64, tf64 = _plan(w, c, "c64", args.kg, args.graph, args.autotune, args.solver,
                         args.nd_leaf, args.nd_top, args.nd_wide, args.nd_wave, args.nd_fuse)
    print(f"# c64 factorisation {tf64:.2f} s", file=sys.stderr, flush=True)
    dt64, its64, rel64, ok64, x64, steps64 = _solve_steps(plan64, b, args.tol, args.maxit,
                                                          args.restart, args.warmup, args.steps)
    print(f"# c64 solve {dt64 / args.steps * 1e3:.1f} ms/step iters {its64}", file=sys.stderr,
          flush=True)
    roof = _roofline(plan64, b, w, 8)
    info64 = plan64.info()
    local_solver64 = plan64.local_solver
    roof["pivot_ratio"] = plan64.pivots()["ratio"]
    plan64.close()
    del plan64

    c128 = None
    if not args.no_c128:
        plan128, tf128 = _plan(w, c, "c128", args.kg, args.graph, args.autotune, args.solver,
                               args.nd_leaf, args.nd_top, args.nd_wide, args.nd_wave, args.nd_fuse)
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
        c128["roofline"] = _roofline(plan128, b, w, 16, FP64_VECTOR_PEAK_TFLOPS)
        plan128.close()
        del plan128

    err = _oracle_error(u_glob, {"c64": x64, "c128": None if c128 is None else x128})

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
                   "global_batch": w.nrhs, "precision": "c64 factors + FP64 refinement",
                   "local_solver": local_solver64},
        "iters": its64, "max_relres": max(rel64), "converged": ok64,
        "median_ms_per_step": round(statistics.median(steps64), 2), "step_ms": steps64,
        "factor_s": round(tf64, 3), "factor_bytes": info64["factor_bytes"],
        "end_to_end_s": round(tf64 + statistics.median(steps64) * 1e-3, 3),
        "c128": c128, "rel_err_vs_oracle": err, "roofline": roof, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
