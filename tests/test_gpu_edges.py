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
"""
import numpy as np
import pytest

from _cases import medium, rel, slowness2, sources
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
    print(f"{n} single subdomain: sweeps vs global {rel(u, ug):.2e}; FGMRES iterations {iters}")
    assert rel(u, ug) < 1e-10 and ok and max(iters) == 1


@pytest.mark.parametrize("n,parts", [((48, 40), (1, 3)), ((48, 40), (4, 1)),
                                     ((12, 11, 16), (1, 1, 3))])
def test_strip_partitions_match_oracle(n, parts):
    plan, (n, h, om, pml, d, c) = _plan(n, parts)
    f = sources(n, h, pml, 2)
    u = plan.sweep_apply(torch.from_numpy(f).cuda()).cpu().numpy().reshape(2, -1)
    u_ref = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c)).apply(f.reshape(2, -1).T).T
    print(f"{n} {parts}: sweeps vs oracle {rel(u, u_ref):.2e}")
    assert rel(u, u_ref) < 1e-10


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
    assert rel(u, u_ref) < 1e-10
    g = f[:2].clone()
    plan.sweep_apply(g, out=g)                        # in place: f is read before u is written
    assert rel(g.cpu().numpy().reshape(2, -1), u_ref) < 1e-10
