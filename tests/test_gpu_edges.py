"""Edge and degenerate cases through the C ABI.

* One subdomain: the only local problem is the global PML problem, so one
  application of the sweeps is the global solution and FGMRES stops after one
  iteration.
* Strip partitions (1 x N, N x 1, 1 x 1 x N): the sweeps with one part along an
  axis match the oracle.
* Batches: a zero right-hand side inside a batch comes back as zero with zero
  iterations; a batch larger than max_rhs or empty and a NaN right-hand side
  are refused with an error and the plan stays usable; the sweeps may run in
  place.
* Error paths: an FGMRES capped at one iteration returns DSD_NOT_CONVERGED
  with valid outputs (the iterate after one step, its true FP64 residual); an
  exactly singular subdomain block is reported as DSD_EPIVOT at plan creation
  (no GPU fault: the pivot search finds an exact zero); the FWI calls and
  HelmholtzMisfit refuse gradients of unconverged solves.
"""
import numpy as np
import pytest

from _cases import close, medium, rel, slowness2, sources
from oracle.sweep import DiagonalSweepDDM, global_solve

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _plan(n, parts, prec="c128", k=2, **kw):
    import paper_2002_05327_amd as dsw
    h = 1.0 / n[0]
    om = 2 * np.pi * (3 if len(n) == 2 else 1.5)
    pml = 6 if len(n) == 2 else 3
    d = 4 if len(n) == 2 else 3
    c = medium("random", n, seed=4)
    m = torch.from_numpy(slowness2(c)).cuda()
    plan = dsw.Plan(n=n, h=h, omega=om, pml=pml, overlap=d, parts=parts, m=m, precision=prec,
                    max_rhs=k, **kw)
    return plan, (n, h, om, pml, d, c)


@pytest.mark.parametrize("n", [(40, 36), (12, 11, 10)])
def test_single_subdomain_is_the_global_solve(n):
    parts = (1,) * len(n)
    plan, (n, h, om, pml, d, c) = _plan(n, parts)
    f = sources(n, h, pml, 2)
    u = plan.sweep_apply(torch.from_numpy(f).cuda()).cpu().numpy().reshape(2, -1)
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c))
    ug = global_solve(ddm.M, f.reshape(2, -1).T).T
    x, iters, relres, ok = plan.gmres(torch.from_numpy(f).cuda(), tol=1e-10, maxit=10)
    print(f"{n} single subdomain: FGMRES iterations {iters}")
    close(u, ug, 1e-10, f"{n} single subdomain sweeps vs global")
    assert ok and max(iters) == 1


@pytest.mark.parametrize("n,parts", [((48, 40), (1, 3)), ((48, 40), (4, 1)),
                                     ((12, 11, 16), (1, 1, 3))])
def test_strip_partitions_match_oracle(n, parts):
    plan, (n, h, om, pml, d, c) = _plan(n, parts)
    f = sources(n, h, pml, 2)
    u = plan.sweep_apply(torch.from_numpy(f).cuda()).cpu().numpy().reshape(2, -1)
    u_ref = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c)).apply(f.reshape(2, -1).T).T
    close(u, u_ref, 1e-10, f"{n} {parts}: sweeps vs oracle")


def test_zero_rhs_in_a_batch():
    plan, (n, h, om, pml, d, c) = _plan((48, 40), (2, 2), prec="c64", k=3)
    f = sources(n, h, pml, 3)
    f[1] = 0
    x, iters, relres, ok = plan.gmres(torch.from_numpy(f).cuda(), tol=1e-8, maxit=40)
    x = x.cpu().numpy()
    assert ok and iters[1] == 0 and relres[1] == 0.0 and not np.any(x[1])
    assert iters[0] > 0 and iters[2] > 0


def test_bad_batches_are_refused_and_the_plan_stays_usable():
    from paper_2002_05327_amd._lib import DsweepError
    plan, (n, h, om, pml, d, c) = _plan((48, 40), (2, 2), k=2)
    f = torch.from_numpy(sources(n, h, pml, 3)).cuda()
    with pytest.raises(DsweepError):
        plan.sweep_apply(f)                           # 3 > max_rhs
    with pytest.raises(DsweepError):
        plan.sweep_apply(f[:0])                       # empty batch
    bad = f[:2].clone()
    bad[0, 10, 10] = float("nan")
    with pytest.raises(DsweepError):
        plan.gmres(bad, tol=1e-8, maxit=10)           # non-finite right-hand side
    u_ref = DiagonalSweepDDM(n, h, om, pml, d, (2, 2), slowness2(c)).apply(
        f[:2].cpu().numpy().reshape(2, -1).T).T
    u = plan.sweep_apply(f[:2]).cpu().numpy().reshape(2, -1)
    close(u, u_ref, 1e-10, "after refused batches")
    g = f[:2].clone()
    plan.sweep_apply(g, out=g)                        # in place: f is read before u is written
    close(g.cpu().numpy().reshape(2, -1), u_ref, 1e-10, "in-place sweep")


SOLVERS = ["bcr", "chain", "chain-steps", "nd"]


def test_not_converged_outputs_are_valid():
    """maxit = 1: DSD_NOT_CONVERGED, one iteration per RHS, and the returned
    relres is the true FP64 residual of the returned iterate under the oracle's
    operator (between tol and 1)."""
    from oracle.pml import assemble, global_axes
    plan, (n, h, om, pml, d, c) = _plan((48, 40), (2, 2), prec="c64", k=3)
    f = sources(n, h, pml, 3)
    x, iters, relres, ok = plan.gmres(torch.from_numpy(f).cuda(), tol=1e-12, maxit=1)
    assert not ok and list(iters) == [1, 1, 1]
    X = x.cpu().numpy().reshape(3, -1)
    assert np.all(np.isfinite(X))
    M = assemble(global_axes(n, pml, h), slowness2(c), h, om, pml)
    B = f.reshape(3, -1)
    true = np.linalg.norm((M @ X.T).T - B, axis=1) / np.linalg.norm(B, axis=1)
    print(f"maxit=1: relres {relres} true {true}")
    for a, b in zip(relres, true):
        assert 1e-12 < a < 1 and abs(a - b) <= 1e-9 * b


@pytest.mark.parametrize("solver", SOLVERS)
def test_singular_block_is_reported_as_epivot(solver):
    """pml = 0, a 2 x 1 grid, h = omega = 1, m = 3: the Dirichlet operator is
    [[-1, 1], [1, -1]] (an eigenvalue of the discrete Laplacian hit exactly, in
    small integers), so elimination meets an exact zero pivot."""
    import paper_2002_05327_amd as dsw
    from paper_2002_05327_amd._lib import DsweepError
    m = torch.full((1, 2), 3.0, dtype=torch.float64, device="cuda")
    with pytest.raises(DsweepError) as ei:
        dsw.Plan(n=(2, 1), h=1.0, omega=1.0, pml=0, overlap=3, parts=(1, 1), m=m,
                 precision="c128", max_rhs=1, local_solver=solver)
    print(ei.value)
    assert ei.value.code == -4
    # a regular medium on the same grid factors fine
    plan = dsw.Plan(n=(2, 1), h=1.0, omega=1.0, pml=0, overlap=3, parts=(1, 1),
                    m=torch.full((1, 2), 2.5, dtype=torch.float64, device="cuda"),
                    precision="c128", max_rhs=1, local_solver=solver)
    plan.close()


@pytest.mark.parametrize("solver", ["bcr", "chain", "nd"])
def test_pivot_report_flags_nearly_singular_blocks(solver):
    """The 2 x 1 Dirichlet grid of the test above, with m = 3 - delta: the
    operator [[delta - 1, 1], [1, delta - 1]] (up to sign) has eigenvalues delta
    and delta - 2, so elimination's second pivot is about 2 delta while the
    first is about 1: dsd_plan_pivots reports max|pivot| / min|pivot| ~ 1 / (2
    delta) for subdomain 0.  At m = 2.5 the ratio is a small number."""
    import paper_2002_05327_amd as dsw
    out = {}
    for m0 in (3.0 - 1e-6, 2.5):
        plan = dsw.Plan(n=(2, 1), h=1.0, omega=1.0, pml=0, overlap=3, parts=(1, 1),
                        m=torch.full((1, 2), m0, dtype=torch.float64, device="cuda"),
                        precision="c128", max_rhs=1, local_solver=solver)
        out[m0] = plan.pivots()
        plan.close()
    print(out)
    near, far = out[3.0 - 1e-6], out[2.5]
    assert near["subdomain"] == 0 and far["subdomain"] == 0
    assert 2e5 < near["ratio"] < 2e6
    assert 1.0 <= far["ratio"] < 10.0


def test_fwi_refuses_unconverged_gradients():
    import synth
    import paper_2002_05327_amd as dsw
    from paper_2002_05327_amd._lib import DsweepError
    N, pml, parts, d = 48, 8, (2, 2), 4
    n, h, om = (N, N), 1 / N, 2 * np.pi * 3
    c0 = synth.smooth_medium(synth.layered_medium(N, N, seed=0), 4.0)
    src = synth.surface_gaussian_sources(N, N, h, 2)
    iy, ix = synth.surface_receivers(N, N, h, 8)
    g = N + 2 * pml
    f = torch.from_numpy(np.stack([np.pad(s, pml) for s in src]).astype(complex)).cuda()
    rec = torch.tensor((iy + pml) * g + (ix + pml), dtype=torch.int64).cuda()
    d_obs = torch.zeros((2, 8), dtype=torch.complex128, device="cuda")
    kw = dict(n=n, h=h, omega=om, pml=pml, overlap=d, parts=parts, precision="c64")
    plan = dsw.Plan(m=torch.from_numpy(1 / c0 ** 2).cuda(), max_rhs=2, **kw)
    with pytest.raises(DsweepError) as ei:
        plan.fwi_gradient(f, rec, d_obs, tol=1e-12, maxit=1)
    assert ei.value.code == 1
    J, gr = plan.fwi_gradient(f, rec, d_obs, tol=1e-12, maxit=1, allow_not_converged=True)
    assert not plan.last_converged and np.isfinite(J) and bool(torch.isfinite(gr).all())
    J, gr = plan.fwi_gradient(f, rec, d_obs, tol=1e-8, maxit=60)
    assert plan.last_converged
    plan.close()
    mt = torch.from_numpy(1 / c0 ** 2).cuda().requires_grad_(True)
    with pytest.raises(DsweepError):
        dsw.HelmholtzMisfit.apply(mt, f, rec, d_obs, kw, 1e-12, 1)
