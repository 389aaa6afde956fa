"""dsd_local_solve_noalloc (the allocation-free local solve, working memory in
the library's static device scratch) against dsd_local_solve on the same plan:
two calls in a row, the second with a smaller input (a smaller subdomain and
fewer right-hand sides), each equal to the allocating entry point's result and
to the oracle's local sparse LU; inputs beyond the static scratch are refused."""
import numpy as np
import pytest

from _cases import close, medium, slowness2, sub_tuple
from oracle.sweep import DiagonalSweepDDM

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _plan(n, h, om, pml, d, parts, c, prec, k, solver):
    """solver "nd-wide": nested dissection with every node in wide mode; "nd-fused":
    leaves of at most 16 cells, the small subtree levels fused."""
    import paper_2002_05327_amd as dsw
    m = torch.from_numpy(slowness2(c)).cuda()
    wide = 1 if solver == "nd-wide" else 0
    leaf = 16 if solver == "nd-fused" else 0
    return dsw.Plan(n=n, h=h, omega=om, pml=pml, overlap=d, parts=parts, m=m, precision=prec,
                    max_rhs=k, local_solver="nd" if solver.startswith("nd") else solver,
                    nd_wide=wide, nd_leaf=leaf)


@pytest.mark.parametrize("solver", ["bcr", "chain", "chain-steps", "nd", "nd-wide", "nd-fused"])
@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_noalloc_local_solve_equals_local_solve(solver, prec):
    n, h, om, pml, d, parts = (61, 70), 1 / 61, 2 * np.pi * 4, 6, 4, (3, 4)
    c = medium("random", n, seed=3)
    plan = _plan(n, h, om, pml, d, parts, c, prec, 3, solver)
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c))
    nsub = int(np.prod(parts))
    sizes = {s: int(np.prod(plan.subdomain_grid(s)[0])) for s in range(nsub)}
    big, small = max(sizes, key=sizes.get), min(sizes, key=sizes.get)
    assert sizes[small] < sizes[big]
    tol = 1e-11 if prec == "c128" else 2e-4
    for sid, k in [(big, 3), (small, 1)]:
        sp = ddm.spaces[sub_tuple(sid, parts)]
        rng = np.random.default_rng(sid + 17)
        r = rng.standard_normal((k, sp.N)) + 1j * rng.standard_normal((k, sp.N))
        rt = torch.from_numpy(r.reshape((k,) + sp.shape)).cuda()
        ref = plan.local_solve(sid, rt)
        u = torch.full_like(rt, float("nan"))
        plan.local_solve_noalloc(sid, rt, u)
        torch.cuda.synchronize()
        print(f"{solver} {prec} sub {sid} ({sizes[sid]} cells, {k} RHS)", flush=True)
        assert np.array_equal(u.cpu().numpy(), ref.cpu().numpy())
        close(u.cpu().numpy().reshape(k, -1), sp.solve(r.T).T, tol, "noalloc vs oracle LU")
    plan.close()


def test_noalloc_refuses_inputs_beyond_the_scratch():
    """One 400 x 400 subdomain with PML 8 (173,056 cells) and 13 complex128
    right-hand sides: 2 x 173,056 x 13 x 16 B = 72 MB > 64 MiB, refused before
    any launch; 12 fit and match dsd_local_solve."""
    from paper_2002_05327_amd import _lib
    from paper_2002_05327_amd._lib import DsweepError
    n = (400, 400)
    c = medium("random", n, seed=5)
    plan = _plan(n, 1 / 400, 2 * np.pi * 3, 8, 4, (1, 1), c, "c128", 13, "bcr")
    dims, _ = plan.subdomain_grid(0)
    assert np.prod(dims) * 13 * 16 * 2 > _lib.NOALLOC_SCRATCH_BYTES
    assert np.prod(dims) * 12 * 16 * 2 <= _lib.NOALLOC_SCRATCH_BYTES
    rng = np.random.default_rng(1)
    shape = (13,) + tuple(reversed(dims))
    r = torch.from_numpy(rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).cuda()
    u = torch.empty_like(r)
    with pytest.raises(DsweepError) as ei:
        plan.local_solve_noalloc(0, r, u)
    assert ei.value.code == -1
    ref = plan.local_solve(0, r[:12].contiguous())
    plan.local_solve_noalloc(0, r[:12].contiguous(), u[:12])
    torch.cuda.synchronize()
    assert np.array_equal(u[:12].cpu().numpy(), ref.cpu().numpy())
    plan.close()
