"""GPU parity: every entry point of libdsweep.so against the FP64 CPU oracle.

Tolerances: complex128 path 1e-10 relative (1e-11 for a single local solve),
complex64 path bounded by the single-precision rounding of the factors
(a few 1e-6 per local solve, 1e-4 for a sweep application), FP64 operator
1e-14.  Every comparison bounds both the relative 2-norm error and the
element-wise error max |u - u_ref| / max |u_ref| (``close``), so an error
confined to a PML strip, a transfer box or one subdomain cannot hide in the
norm of the whole grid.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from _cases import close, embed_physical, medium, rel, slowness2, sources, sub_tuple
from oracle.pml import assemble, global_axes
from oracle.sweep import DiagonalSweepDDM, global_solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _plan(n, h, om, pml, d, parts, c, prec, k, kg=0, schedule="dag", solver="auto", dense_top=0):
    """solver "nd-wide": nested dissection with every node in wide mode (tiled
    products over all right-hand sides of a group, vectors streamed through LDS);
    "nd-mfma": nested dissection with 16 right-hand sides per workgroup, where its
    LDS-front kernels run on the matrix cores; "nd-fused": leaves of at most 16
    cells and the subtree levels whose fronts have at most 128 cells fused into
    one workgroup per subtree; "nd-fused-all": every subtree level fused."""
    import paper_2002_05327_amd as dsw
    m = torch.from_numpy(slowness2(c)).cuda()
    wide = 1 if solver == "nd-wide" else 0
    if solver == "nd-mfma" and kg == 0:
        kg = 16
    leaf = 16 if solver.startswith("nd-fused") else 0
    fuse = 512 if solver == "nd-fused-all" else 0
    return dsw.Plan(n=n, h=h, omega=om, pml=pml, overlap=d, parts=parts, m=m, precision=prec,
                    max_rhs=k, rhs_per_group=kg, schedule=schedule,
                    local_solver="nd" if solver.startswith("nd") else solver,
                    dense_top=dense_top, nd_wide=wide, nd_leaf=leaf, nd_fuse=fuse)


SOLVERS = ["bcr", "chain", "chain-steps", "nd", "nd-wide", "nd-mfma", "nd-fused", "nd-fused-all"]


def _cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


CASES = {
    # name: n, h, omega, pml, overlap, parts, medium
    "c1": ((128, 128), 1 / 128, 2 * np.pi * 8, 16, 8, (2, 2), "const"),
    "lay33": ((72, 66), 1 / 72, 2 * np.pi * 5, 8, 4, (3, 3), "layered"),
    "rag34": ((61, 70), 1 / 61, 2 * np.pi * 4, 6, 4, (3, 4), "random"),
    "d3": ((14, 13, 12), 1 / 14, 2 * np.pi * 1.5, 3, 3, (2, 2, 2), "random"),
    # blocks wider than 192 and 256 cells: four-tile chain kernels, several row groups
    "wide2": ((400, 60), 1 / 400, 2 * np.pi * 4, 8, 4, (2, 2), "random"),
    "wide3": ((24, 22, 10), 1 / 24, 2 * np.pi * 1.5, 3, 3, (2, 2, 2), "random"),
}


def _case(name):
    n, h, om, pml, d, parts, med = CASES[name]
    return n, h, om, pml, d, parts, medium(med, n, seed=3)


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("name", ["c1", "rag34", "d3", "wide2", "wide3"])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_local_solve_matches_oracle(name, prec, solver):
    n, h, om, pml, d, parts, c = _case(name)
    k = 3
    plan = _plan(n, h, om, pml, d, parts, c, prec, k, solver=solver)
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c))
    nsub = int(np.prod(parts))
    for sid in sorted({0, nsub - 1, nsub // 2}):
        st = sub_tuple(sid, parts)
        sp = ddm.spaces[st]
        dims, g0 = plan.subdomain_grid(sid)
        assert dims == tuple(ax.n for ax in sp.axes) and g0 == tuple(ax.g0 for ax in sp.axes)
        rng = np.random.default_rng(sid)
        r = rng.standard_normal((k, sp.N)) + 1j * rng.standard_normal((k, sp.N))
        u_ref = sp.solve(r.T).T
        u = plan.local_solve(sid, _cuda(r.reshape((k,) + sp.shape))).cpu().numpy().reshape(k, -1)
        tol = 1e-11 if prec == "c128" else 2e-4
        close(u, u_ref, tol, f"{name} {prec} {solver} sub {sid}")


@pytest.mark.parametrize("name", ["lay33", "d3"])
def test_operator_matches_oracle(name):
    n, h, om, pml, d, parts, c = _case(name)
    plan = _plan(n, h, om, pml, d, parts, c, "c128", 2)
    M = assemble(global_axes(n, pml, h), slowness2(c), h, om, pml)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((2,) + plan.gshape) + 1j * rng.standard_normal((2,) + plan.gshape)
    y = plan.apply_operator(_cuda(x)).cpu().numpy()
    y_ref = (M @ x.reshape(2, -1).T).T.reshape(y.shape)
    close(y, y_ref, 1e-14, f"{name} operator")


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("name", ["c1", "lay33", "rag34", "d3", "wide2", "wide3"])
def test_sweep_apply_c128_matches_oracle_real_mode(name, solver):
    """One application of Algorithm 3.1 / 4.1 (real local PML solves)."""
    n, h, om, pml, d, parts, c = _case(name)
    k = 2
    f = sources(n, h, pml, k)
    plan = _plan(n, h, om, pml, d, parts, c, "c128", k, solver=solver)
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c))
    u_ref = ddm.apply(f.reshape(k, -1).T).T
    u = plan.sweep_apply(_cuda(f)).cpu().numpy().reshape(k, -1)
    e = rel(u, u_ref)
    print(f"{name} {solver}: GPU c128 sweep vs oracle {e:.2e}; DDM vs global solve "
          f"{rel(u_ref, global_solve(ddm.M, f.reshape(k, -1).T).T):.2e}", flush=True)
    close(u, u_ref, 1e-10, f"{name} {solver} c128 sweep")


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("name", ["c1", "lay33", "wide3"])
def test_sweep_apply_c64_close_to_oracle(name, solver):
    n, h, om, pml, d, parts, c = _case(name)
    k = 2
    f = sources(n, h, pml, k)
    plan = _plan(n, h, om, pml, d, parts, c, "c64", k, solver=solver)
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c))
    u_ref = ddm.apply(f.reshape(k, -1).T).T
    u = plan.sweep_apply(_cuda(f)).cpu().numpy().reshape(k, -1)
    close(u, u_ref, 1e-4, f"{name} {solver} c64 sweep")


def test_sweep_apply_deterministic():
    n, h, om, pml, d, parts, c = _case("rag34")
    f = _cuda(sources(n, h, pml, 2))
    plan = _plan(n, h, om, pml, d, parts, c, "c64", 2)
    a = plan.sweep_apply(f).cpu().numpy()
    b = plan.sweep_apply(f).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("solver", ["bcr", "chain-steps", "nd"])
@pytest.mark.parametrize("prec,tol", [("c128", 1e-10), ("c64", 1e-4)])
def test_autotuned_plan_matches_oracle(prec, tol, solver):
    """The autotuner only picks launch shapes: the tuned plan still matches the oracle."""
    n, h, om, pml, d, parts, c = _case("lay33")
    k = 3
    f = sources(n, h, pml, k)
    plan = _plan(n, h, om, pml, d, parts, c, prec, k, solver=solver)
    res = plan.autotune(reps=1)
    assert res["rhs_per_group"] >= 1 and res["ms_per_application"] > 0
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c))
    u_ref = ddm.apply(f.reshape(k, -1).T).T
    u = plan.sweep_apply(_cuda(f)).cpu().numpy().reshape(k, -1)
    close(u, u_ref, tol, f"autotune {prec}: {res}")
    # a saved shape applied to a fresh plan reproduces the tuned plan bitwise
    plan2 = _plan(n, h, om, pml, d, parts, c, prec, k, solver=solver)
    plan2.solve_shape = res["shape"]
    assert plan2.solve_shape == res["shape"]
    u2 = plan2.sweep_apply(_cuda(f)).cpu().numpy().reshape(k, -1)
    assert np.array_equal(u2, u)


@pytest.mark.parametrize("shape", [(4, 32, 8, 1, 0, 2, 0, 8, 1, 12, 8, 3, 0), (2, 16, 4, 2, 0, 4, 1, 12, 1, 4, 0, 12, 1),
                                   (8, 1 << 30, 1 << 30, 1, 0, 1, 0, 1, 0, 8, 0, 1, 0),
                                   (1, 8, 2, 12, 1, 3, 1, 1, 1, 1, 4, 4, 1)])
@pytest.mark.parametrize("solver", ["bcr", "chain-steps"])
def test_solve_shapes_match_oracle(shape, solver):
    """Every launch shape the autotuner may pick solves the same problem."""
    n, h, om, pml, d, parts, c = _case("rag34")
    k = 3
    f = sources(n, h, pml, k)
    plan = _plan(n, h, om, pml, d, parts, c, "c128", k, solver=solver)
    plan.solve_shape = shape
    assert plan.solve_shape == tuple(shape)
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c))
    u_ref = ddm.apply(f.reshape(k, -1).T).T
    u = plan.sweep_apply(_cuda(f)).cpu().numpy().reshape(k, -1)
    close(u, u_ref, 1e-10, f"shape {shape} {solver}")


@pytest.mark.parametrize("solver", SOLVERS)
def test_graph_replays_equal_eager_application(solver):
    """A captured application replays bitwise like the eager one, also with eager
    work in between and after the output buffer was overwritten."""
    n, h, om, pml, d, parts, c = _case("rag34")
    f = _cuda(sources(n, h, pml, 3))
    plan = _plan(n, h, om, pml, d, parts, c, "c64", 3, solver=solver)
    ref = plan.sweep_apply(f).cpu().numpy()
    plan.use_graph(True)
    out = torch.empty_like(f)
    for rep in range(4):
        out.fill_(float("nan"))
        plan.sweep_apply(f, out=out)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), f"replay {rep}"
        plan.apply_operator(f)                     # eager work between replays
    x_graph, its_g, _, ok_g = plan.gmres(f, tol=1e-10, maxit=60)
    plan.use_graph(False)
    x_eager, its_e, _, ok_e = plan.gmres(f, tol=1e-10, maxit=60)
    assert ok_g and ok_e and list(its_g) == list(its_e)
    assert np.array_equal(x_graph.cpu().numpy(), x_eager.cpu().numpy())


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("name", ["rag34", "d3"])
def test_dependency_schedule_equals_sequential_steps(name, solver):
    """Launching each solve at its dependency level reorders nothing that is summed."""
    n, h, om, pml, d, parts, c = _case(name)
    f = _cuda(sources(n, h, pml, 3))
    a = _plan(n, h, om, pml, d, parts, c, "c64", 3, schedule="dag",
              solver=solver).sweep_apply(f).cpu().numpy()
    b = _plan(n, h, om, pml, d, parts, c, "c64", 3, schedule="sequential",
              solver=solver).sweep_apply(f).cpu().numpy()
    assert np.array_equal(a, b)


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("kg", [1, 2, 4])
def test_rhs_grouping_does_not_change_result(kg, solver):
    n, h, om, pml, d, parts, c = _case("lay33")
    k = 5
    f = _cuda(sources(n, h, pml, k))
    ref = _plan(n, h, om, pml, d, parts, c, "c128", k, kg=1, solver=solver).sweep_apply(f)
    got = _plan(n, h, om, pml, d, parts, c, "c128", k, kg=kg, solver=solver).sweep_apply(f)
    close(got.cpu().numpy(), ref.cpu().numpy(), 1e-13, f"kg {kg} {solver}")


@pytest.mark.parametrize("kg", [2, 4, 8])
def test_rhs_grouping_c64_matrix_core_path(kg):
    """complex64 groups of 2, 4 and 8 RHS all run on the matrix cores."""
    n, h, om, pml, d, parts, c = _case("lay33")
    k = 9
    f = _cuda(sources(n, h, pml, k))
    ref = _plan(n, h, om, pml, d, parts, c, "c64", k, kg=2, solver="bcr").sweep_apply(f)
    got = _plan(n, h, om, pml, d, parts, c, "c64", k, kg=kg, solver="bcr").sweep_apply(f)
    close(got.cpu().numpy(), ref.cpu().numpy(), 1e-6, f"c64 kg {kg}")


@pytest.mark.parametrize("name", ["lay33", "rag34", "d3"])
def test_cyclic_reduction_equals_chains(name):
    """Every local solver inverts the same subdomain operators (complex128)."""
    n, h, om, pml, d, parts, c = _case(name)
    f = _cuda(sources(n, h, pml, 2))
    a = _plan(n, h, om, pml, d, parts, c, "c128", 2, solver="bcr").sweep_apply(f).cpu().numpy()
    b = _plan(n, h, om, pml, d, parts, c, "c128", 2, solver="chain").sweep_apply(f).cpu().numpy()
    s = _plan(n, h, om, pml, d, parts, c, "c128", 2, solver="chain-steps").sweep_apply(f).cpu().numpy()
    e = _plan(n, h, om, pml, d, parts, c, "c128", 2, solver="nd").sweep_apply(f).cpu().numpy()
    close(a, b, 1e-12, f"{name} reduction vs chains")
    close(s, b, 1e-12, f"{name} chain steps vs chains")
    close(e, b, 1e-12, f"{name} nested dissection vs chains")


@pytest.mark.parametrize("dense_top", [-1, 2, 3, 8])
@pytest.mark.parametrize("name", ["c1", "rag34", "wide2", "d3"])
def test_dense_top_level_matches_oracle(name, dense_top):
    """Stopping the reduction at a small level and applying that reduced system's
    dense inverse solves the same local problems (c128 to rounding) as reducing
    to a single block (dense_top = -1)."""
    n, h, om, pml, d, parts, c = _case(name)
    k = 3
    plan = _plan(n, h, om, pml, d, parts, c, "c128", k, solver="bcr", dense_top=dense_top)
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c))
    nsub = int(np.prod(parts))
    for sid in sorted({0, nsub - 1}):
        sp = ddm.spaces[sub_tuple(sid, parts)]
        rng = np.random.default_rng(sid + 7)
        r = rng.standard_normal((k, sp.N)) + 1j * rng.standard_normal((k, sp.N))
        u_ref = sp.solve(r.T).T
        u = plan.local_solve(sid, _cuda(r.reshape((k,) + sp.shape))).cpu().numpy().reshape(k, -1)
        close(u, u_ref, 1e-11, f"{name} dense_top={dense_top} sub {sid}")
    f = sources(n, h, pml, k)
    u_ref = ddm.apply(f.reshape(k, -1).T).T
    u = plan.sweep_apply(_cuda(f)).cpu().numpy().reshape(k, -1)
    close(u, u_ref, 1e-10, f"{name} dense_top={dense_top} sweep")


@pytest.mark.parametrize("prec,tol,bound", [("c128", 1e-12, 1e-10), ("c64", 1e-11, 1e-8)])
def test_gmres_matches_global_solve(prec, tol, bound):
    n, h, om, pml, d, parts, c = _case("lay33")
    k = 3
    f = sources(n, h, pml, k)
    plan = _plan(n, h, om, pml, d, parts, c, prec, k)
    x, its, res, ok = plan.gmres(_cuda(f), tol=tol, maxit=80)
    M = assemble(global_axes(n, pml, h), slowness2(c), h, om, pml)
    x_ref = global_solve(M, f.reshape(k, -1).T).T
    xg = x.cpu().numpy().reshape(k, -1)
    true_res = [np.linalg.norm(f[i].ravel() - M @ xg[i]) / np.linalg.norm(f[i]) for i in range(k)]
    print(f"{prec}: iters {its} relres {res} true {true_res} err {rel(xg, x_ref):.2e}", flush=True)
    assert ok and max(true_res) <= tol * 1.01
    close(xg, x_ref, bound, f"{prec} FGMRES vs global LU")


def test_gmres_c1_reaches_global_solution():
    """Config 1 reading: GMRES-DDM driven to relres 1e-13 equals the global LU to 1e-10."""
    n, h, om, pml, d, parts, c = _case("c1")
    f = embed_physical(__import__("synth").gaussian_source(n, h, (0.5, 0.5), 2 * h), pml)[None]
    plan = _plan(n, h, om, pml, d, parts, c, "c128", 1)
    x, its, res, ok = plan.gmres(_cuda(f.astype(complex)), tol=1e-13, maxit=40)
    M = assemble(global_axes(n, pml, h), slowness2(c), h, om, pml)
    x_ref = global_solve(M, f.reshape(-1))
    print(f"c1 gmres iters {its} relres {res}")
    assert ok
    close(x.cpu().numpy().ravel(), x_ref, 1e-10, "c1 FGMRES vs global LU")


def test_adjoint_solve():
    n, h, om, pml, d, parts, c = _case("lay33")
    k = 2
    f = sources(n, h, pml, k)
    plan = _plan(n, h, om, pml, d, parts, c, "c128", k)
    y, _, _, ok = plan.adjoint_solve(_cuda(f), tol=1e-12, maxit=80)
    M = assemble(global_axes(n, pml, h), slowness2(c), h, om, pml).tocsc()
    y_ref = spla.splu(M.conj().T.tocsc()).solve(f.reshape(k, -1).T).T
    assert ok
    close(y.cpu().numpy().reshape(k, -1), y_ref, 1e-10, "adjoint solve")


def test_fwi_gradient_matches_oracle():
    import synth
    from oracle.fwi import FWIOracle
    import paper_2002_05327_amd as dsw
    N, pml, parts, d = 48, 8, (3, 3), 4
    n, h, om = (N, N), 1 / N, 2 * np.pi * 3
    c_true = synth.layered_medium(N, N, seed=0)
    c0 = synth.smooth_medium(c_true, 4.0)
    src = synth.surface_gaussian_sources(N, N, h, 4)
    iy, ix = synth.surface_receivers(N, N, h, 12)
    fw = FWIOracle(n, h, om, pml, src, (iy, ix))
    d_obs = fw.observed(slowness2(c_true))
    J_ref, g_ref = fw.gradient(slowness2(c0), d_obs)
    gshape = (N + 2 * pml, N + 2 * pml)
    f = np.stack([embed_physical(s, pml) for s in src]).astype(complex)
    rec = torch.tensor((iy + pml) * gshape[1] + (ix + pml), dtype=torch.int64).cuda()
    for prec, tol, bound in [("c128", 1e-12, 1e-8), ("c64", 1e-11, 1e-7)]:
        plan = _plan(n, h, om, pml, d, parts, c0, prec, 4)
        J, g = plan.fwi_gradient(_cuda(f), rec, _cuda(d_obs.T.copy()), tol=tol, maxit=80)
        print(f"fwi {prec}: misfit rel {abs(J - J_ref) / J_ref:.2e}")
        assert abs(J - J_ref) / J_ref < bound
        close(g.cpu().numpy(), g_ref, bound * 10, f"fwi {prec} gradient")


@pytest.mark.parametrize("solver", SOLVERS)
def test_timing_hooks_bytes_and_flops(solver):
    """The measurement hooks behind bench.py's roofline, over one application:
    launches and device time are positive; the flops (8 per complex factor
    entry and right-hand side) scale exactly with the right-hand-side count,
    the bytes only through their vector part, so 2 B(4) - B(8) is the factor
    bytes F and the flops at 4 RHS are 4 F."""
    n, h, om, pml, d, parts, c = _case("lay33")
    plan = _plan(n, h, om, pml, d, parts, c, "c64", 8, solver=solver)
    reads = {}
    for k in (4, 8):
        f = _cuda(sources(n, h, pml, k))
        plan.timing(True)
        plan.sweep_apply(f)
        torch.cuda.synchronize()
        reads[k] = plan.timing_read()
        plan.timing(False)
    a, b = reads[4], reads[8]
    assert a["solve_launches"] == b["solve_launches"] > 0
    assert a["solve_ms"] > 0 and b["solve_ms"] > 0
    assert b["solve_flops"] == pytest.approx(2 * a["solve_flops"], rel=1e-12)
    fac = 2 * a["solve_bytes"] - b["solve_bytes"]
    assert fac > 0
    assert a["solve_flops"] == pytest.approx(4 * fac, rel=1e-9)


def _three_layer_case(N, freq, parts):
    import synth
    pml, d = 8, 4
    h, om = 1.0 / N, 2 * np.pi * freq
    c = synth.three_layer_medium(N, N)
    f = synth.point_source(N, N, h, pml, 0.25 / parts[0], (1.0 / 3.0) / parts[1])
    return (N, N), h, om, pml, d, c, f


@pytest.mark.parametrize("prec", ["c128", "c64"])
@pytest.mark.parametrize("parts", [(1, 2), (3, 3)])
def test_ddm_iterate_matches_oracle(parts, prec):
    """dsd_ddm_iterate (the sweeps as a stand-alone solver, Section 5.2) against
    the oracle's iteration on the three-layer case: the residual history
    (complex128: entry by entry; complex64: the first two iterations to the
    single-precision sweep error) and the iterate, which converges to the
    global solution in either precision because the residual is FP64."""
    from oracle.krylov import ddm_iterate
    n, h, om, pml, d, c, f = _three_layer_case(64, 4, parts)
    M = assemble(global_axes(n, pml, h), slowness2(c), h, om, pml)
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c))
    iters = 10
    x_ref, hist_ref = ddm_iterate(lambda v: M @ v, ddm.apply, f.ravel(), iters)
    plan = _plan(n, h, om, pml, d, parts, c, prec, 1)
    x, hist = plan.ddm_iterate(_cuda(f[None]), iters)
    hist = [v[0] for v in hist]
    u = global_solve(M, f.ravel())
    ex = rel(x.cpu().numpy().ravel(), u)
    print(f"{parts} {prec}: history {['%.3e' % v for v in hist]}; iterate vs global {ex:.2e}")
    assert hist[0] == 1.0
    if prec == "c128":
        for a, b in zip(hist, hist_ref):
            assert abs(a - b) <= 1e-12 + 1e-7 * b
        close(x.cpu().numpy().ravel(), x_ref, 1e-10, f"{parts} iterate")
    else:
        for a, b in zip(hist[1:3], hist_ref[1:3]):
            assert abs(a - b) <= 1e-3 * b
    assert hist[-1] < 1e-8 and ex < 1e-7


@pytest.mark.parametrize("name", ["d3", "wide3"])
def test_sweep_apply_3d_l1_order_matches_oracle(name):
    """The other 3D sweep order of Section 4.1 (L1 distance from the first
    direction non-decreasing): GPU sweeps (complex128) against the oracle's
    real mode with the same order, and different from the default order."""
    import paper_2002_05327_amd as dsw
    n, h, om, pml, d, parts, c = _case(name)
    k = 2
    f = sources(n, h, pml, k)
    m = torch.from_numpy(slowness2(c)).cuda()
    plan = dsw.Plan(n=n, h=h, omega=om, pml=pml, overlap=d, parts=parts, m=m, precision="c128",
                    max_rhs=k, sweep_order="l1")
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c), order_variant=1)
    u_ref = ddm.apply(f.reshape(k, -1).T).T
    u = plan.sweep_apply(_cuda(f)).cpu().numpy().reshape(k, -1)
    u0 = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c)).apply(f.reshape(k, -1).T).T
    print(f"{name}: default vs l1 order {rel(u0, u_ref):.2e}")
    close(u, u_ref, 1e-10, f"{name} l1-order sweep")
    assert rel(u0, u_ref) > 1e-8


@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("name", ["lay33", "rag34", "d3"])
def test_additive_ddm_matches_oracle(name, solver):
    """schedule="additive" (Algorithms 2.1 / 2.2 of Section 2 on the same
    kernels) against the oracle's additive DDM in real mode (complex128), and
    FGMRES with it as the preconditioner converges to the global solution."""
    from oracle.sweep import AdditiveDDM
    n, h, om, pml, d, parts, c = _case(name)
    k = 2
    f = sources(n, h, pml, k)
    plan = _plan(n, h, om, pml, d, parts, c, "c128", k, schedule="additive", solver=solver)
    add = AdditiveDDM(n, h, om, pml, d, parts, slowness2(c))
    u_ref = add.apply(f.reshape(k, -1).T).T
    u = plan.sweep_apply(_cuda(f)).cpu().numpy().reshape(k, -1)
    close(u, u_ref, 1e-10, f"{name} {solver} additive DDM")
    x, iters, relres, ok = plan.gmres(_cuda(f), tol=1e-10, maxit=60)
    print(f"{name} {solver}: FGMRES {iters} its")
    assert ok
    close(x.cpu().numpy().reshape(k, -1), global_solve(add.M, f.reshape(k, -1).T).T, 1e-8,
          f"{name} {solver} additive FGMRES vs global")
