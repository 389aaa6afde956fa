"""Pins for the oracle's diagonal-sweeping DDM (oracle.sweep, oracle.partition).

* exact-solve mode reproduces the global PML solution to rounding for any
  medium and partition (discrete counterpart of Theorems 3.1 and 4.1, which
  holds exactly because of the index-form cutoffs; the paper's constant-medium
  assumption only makes local PML problems agree with the global one);
* the 5x5 (2D) and 5x5x5 (3D) walk-throughs printed in Sections 3 and 4.2:
  first step with a non-zero local source in each sweep, number of non-zero
  transfers generated, quadrant/octant built by each sweep (tests/golden);
* the routing behaviour the text states for the first sweeps (Section 3);
* the diagonal marching property of the additive DDM (end of Section 2.2);
* real mode: a 1x1 partition is the global solve; with constant medium the
  DDM error is the PML truncation error and decreases as the PML widens;
* the transfer operator computed with the sender's local operator equals the
  one computed with the receiver's (same coefficients on the support).
"""
import json
import os

import numpy as np
import pytest

from oracle.krylov import fgmres
from oracle.partition import directions
from oracle.pml import embed_physical, slowness2
from oracle.sweep import (AdditiveDDM, DiagonalSweepDDM, global_solve, route, step_groups, step_of,
                          sweep_order)
import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("parts,n,medium", [
    ((2, 2), (48, 40), "const"), ((3, 3), (60, 60), "layered"),
    ((5, 5), (80, 80), "random"), ((3, 4), (61, 70), "random"), ((4, 1), (64, 24), "layered")])
def test_exact_mode_reproduces_global_solution_2d(parts, n, medium):
    h, om, pml, d = 1 / n[0], 2 * np.pi * 4, 8, 4
    if medium == "const":
        c = np.ones(n[::-1])
    elif medium == "layered":
        c = synth.layered_medium(n[0], n[1], seed=3)
    else:
        c = 1 + 0.5 * np.random.default_rng(3).random(n[::-1])
    fb = np.stack([embed_physical(x, pml).ravel() for x in
                   np.random.default_rng(1).standard_normal((2,) + n[::-1])], axis=1)
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c), mode="exact")
    u = ddm.apply(fb)
    assert _rel(u, global_solve(ddm.M, fb)) < 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("parts,n", [((2, 2, 2), (12, 12, 12)), ((3, 3, 2), (12, 12, 9))])
def test_exact_mode_reproduces_global_solution_3d(parts, n, variant):
    """Both 3D sweep orders of Section 4.1 ((Sorder3D) and the L1-monotone one),
    with transfers routed by Rules 4.1/4.2 over the order in use."""
    h, om, pml, d = 1 / n[0], 2 * np.pi * 2, 3, 3
    c = 1 + 0.5 * np.random.default_rng(3).random(n[::-1])
    f = embed_physical(np.random.default_rng(1).standard_normal(n[::-1]), pml).ravel()
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c), mode="exact",
                           order_variant=variant)
    assert _rel(ddm.apply(f), global_solve(ddm.M, f)) < 1e-12


def _single_source_run(parts, cells_per_part, pml, d, src_sub, om):
    dim = len(parts)
    n = tuple(p * cells_per_part for p in parts)
    h = 1.0 / n[0]
    rng = np.random.default_rng(5)
    c = 1 + 0.3 * rng.random(n[::-1])
    ddm = DiagonalSweepDDM(n, h, om, pml, d, parts, slowness2(c), mode="exact")
    f = np.zeros(ddm.gshape)
    own = ddm.part.own_mask(src_sub, ddm.gaxes)
    f[own] = rng.standard_normal(int(own.sum()))
    trace = {}
    u = ddm.apply(f.ravel(), trace=trace)
    return ddm, f.ravel(), u, trace


def _nonzero(x, scale):
    return x > 1e-9 * scale


def test_walkthrough_2d_golden():
    g = json.load(open(os.path.join(GOLD, "walkthrough_2d.json")))
    src = tuple(i - 1 for i in g["source_subdomain_1based"])
    ddm, f, u, tr = _single_source_run(tuple(g["parts"]), 10, 6, 4, src, 2 * np.pi * 3)
    ug = global_solve(ddm.M, f)
    assert _rel(u, ug) < 1e-12
    scale = np.linalg.norm(f)
    assert len(step_groups(ddm.order[0], ddm.part.parts)) == g["steps_per_sweep"]
    # first step of each sweep with a non-zero local source
    for l, want in enumerate(g["first_nonzero_step_per_sweep"]):
        steps = [s for (ll, s, sub), v in tr["rhs_norm"].items() if ll == l and _nonzero(v, scale)]
        assert min(steps) == want
    # non-zero transfers generated in sweep 1
    for key, want in g["nonzero_transfers_generated_in_sweep1"].items():
        sub = tuple(int(i) - 1 for i in key.split(","))
        got = sum(1 for (l, s, t), v in tr["transfer_norm"].items()
                  if l == 0 and s == sub and _nonzero(v, scale))
        assert got == want, (key, got)
    # quadrant built by each sweep: cumulative u equals u away from inner borders
    for q in g["quadrant_built_by_sweep_1based"]:
        l = q["sweep"] - 1
        part = ddm.part
        sl = []
        for a, key in enumerate(("i", "j")):
            lo_p, hi_p = q[key][0] - 1, q[key][1] - 1
            lo = part.axis_parts[a][lo_p].o0 + (ddm.part.d - 1 if lo_p > 0 else 0)
            hi = part.axis_parts[a][hi_p].o1 - (ddm.part.d - 1 if hi_p < part.parts[a] - 1 else 0)
            sl.append(slice(lo, hi))
        region = (sl[1], sl[0])
        part_u = tr["after_sweep"][l][:, 0].reshape(ddm.gshape)[region]
        assert _rel(part_u, ug.reshape(ddm.gshape)[region]) < 1e-12


@pytest.mark.slow
def test_walkthrough_3d_golden():
    g = json.load(open(os.path.join(GOLD, "walkthrough_3d.json")))
    src = tuple(i - 1 for i in g["source_subdomain_1based"])
    ddm, f, u, tr = _single_source_run(tuple(g["parts"]), 3, 2, 3, src, 2 * np.pi * 1.5)
    ug = global_solve(ddm.M, f)
    assert _rel(u, ug) < 1e-12
    scale = np.linalg.norm(f)
    assert len(step_groups(ddm.order[0], ddm.part.parts)) == g["steps_per_sweep"]
    steps = [s for (l, s, sub), v in tr["rhs_norm"].items() if l == 0 and _nonzero(v, scale)]
    assert min(steps) == g["first_nonzero_step_sweep1"]
    for key, want in g["nonzero_transfers_generated_in_sweep1"].items():
        sub = tuple(int(i) - 1 for i in key.split(","))
        got = sum(1 for (l, s, t), v in tr["transfer_norm"].items()
                  if l == 0 and s == sub and _nonzero(v, scale))
        assert got == want, (key, got)
    for key, want in g["nonzero_sources_received_in_sweep1"].items():
        rec = tuple(int(i) - 1 for i in key.split(","))
        got = sum(1 for (l, s, t), v in tr["transfer_norm"].items()
                  if l == 0 and tuple(a + b for a, b in zip(s, t)) == rec
                  and route(0, t, 3) == 0 and _nonzero(v, scale))
        assert got == want, (key, got)
    oc = g["octant_built_by_sweep1_1based"]
    sl = []
    for a, key in enumerate(("i", "j", "k")):
        lo_p, hi_p = oc[key][0] - 1, oc[key][1] - 1
        lo = ddm.part.axis_parts[a][lo_p].o0 + ddm.part.d - 1
        hi = ddm.part.axis_parts[a][hi_p].o1
        sl.append(slice(lo, hi))
    region = tuple(reversed(sl))
    part_u = tr["after_sweep"][0][:, 0].reshape(ddm.gshape)[region]
    assert _rel(part_u, ug.reshape(ddm.gshape)[region]) < 1e-12


def test_routing_statements_of_section3():
    """Facts the 2D walk-through states about which sweep uses which transfer."""
    L = {D: l for l, D in enumerate(sweep_order(2))}
    s1, s2, s3, s4 = (L[(1, 1)], L[(-1, 1)], L[(1, -1)], L[(-1, -1)])
    # sweep 1 uses only (+1,0), (0,+1), (+1,+1) of its own transfers
    assert {t for t in directions(2) if route(s1, t, 2) == s1} == {(1, 0), (0, 1), (1, 1)}
    # sweep 2 uses (-1,0), (0,+1), (-1,+1) left by sweep 1
    for t in [(-1, 0), (0, 1), (-1, 1)]:
        assert route(s1, t, 2) in (s1, s2) and (t == (0, 1) or route(s1, t, 2) == s2)
    # downward transfers of sweep 1 wait for sweep 3; axial ones of sweep 2 never enter sweep 3
    assert route(s1, (0, -1), 2) == s3
    assert route(s2, (1, 0), 2) is None and route(s2, (0, -1), 2) == s4
    # the fourth sweep receives no horizontal or vertical transfer made in the first
    assert all(route(s1, t, 2) != s4 for t in [(1, 0), (-1, 0), (0, 1), (0, -1)])
    # step of a subdomain: (i-1)+(j-1)+1 for (+,+), (Nx-i)+(j-1)+1 for (-,+) ...
    assert step_of((2, 2), (1, 1), (5, 5)) == 5 and step_of((2, 2), (-1, 1), (5, 5)) == 5
    assert step_of((1, 2), (-1, 1), (5, 5)) == 6 and step_of((1, 1), (-1, -1), (5, 5)) == 7


def test_real_mode_single_subdomain_is_global_solve():
    n, h, om, pml = (40, 36), 1 / 40, 2 * np.pi * 4, 8
    c = synth.layered_medium(*n, seed=2)
    f = embed_physical(synth.gaussian_source(n, h, (0.4, 0.3), 2 * h), pml).ravel()
    ddm = DiagonalSweepDDM(n, h, om, pml, 4, (1, 1), slowness2(c))
    assert _rel(ddm.apply(f), global_solve(ddm.M, f)) < 1e-12


@pytest.mark.slow
def test_real_mode_error_decreases_with_pml_width():
    """Constant medium: the DDM differs from the global solution only through
    the truncation of the subdomain PMLs, which shrinks as the PML widens
    (fixed sigma0*width)."""
    n, h, om, d = (64, 64), 1 / 64, 2 * np.pi * 4, 6
    f0 = synth.gaussian_source(n, h, (0.37, 0.61), 2 * h)
    errs = []
    for pml in (4, 8, 16):
        f = embed_physical(f0, pml).ravel()
        ddm = DiagonalSweepDDM(n, h, om, pml, d, (3, 3), slowness2(np.ones(n[::-1])))
        errs.append(_rel(ddm.apply(f), global_solve(ddm.M, f)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-3


def test_transfer_same_with_receiver_operator():
    n, h, om, pml, d = (48, 40), 1 / 48, 2 * np.pi * 4, 6, 5
    c = 1 + 0.4 * np.random.default_rng(8).random(n[::-1])
    ddm = DiagonalSweepDDM(n, h, om, pml, d, (3, 2), slowness2(c))
    sub = (1, 0)
    sp_s = ddm.spaces[sub]
    v = np.random.default_rng(2).standard_normal((sp_s.N, 1)) + 0j
    for t in [(1, 0), (-1, 0), (0, 1), (1, 1), (-1, 1)]:
        nb = (sub[0] + t[0], sub[1] + t[1])
        gv, box = ddm.transfer(sub, t, v)
        rbox = ddm._receiver_box(sub, nb, box)
        # evaluate with the receiver's operator: embed beta v on the receiver grid
        sp_r = ddm.spaces[nb]
        bt = ddm.part.beta(sub, t, sp_s.axes).ravel()[:, None] * v
        w = np.zeros(sp_r.shape + (1,), dtype=complex)
        # copy the part of beta v that lies on the receiver's grid
        sl_s, sl_r = [], []
        for a in range(2):
            s_ax, r_ax = sp_s.axes[a], sp_r.axes[a]
            lo = max(s_ax.g0, r_ax.g0)
            hi = min(s_ax.g0 + s_ax.n, r_ax.g0 + r_ax.n)
            sl_s.append(slice(lo - s_ax.g0, hi - s_ax.g0))
            sl_r.append(slice(lo - r_ax.g0, hi - r_ax.g0))
        w[tuple(reversed(sl_r))] = bt.reshape(sp_s.shape + (1,))[tuple(reversed(sl_s))]
        g_r = -(sp_r.M @ w.reshape(-1, 1)).reshape(sp_r.shape + (1,))[rbox]
        assert np.array_equal(g_r, gv), t


def test_marching_step_formula():
    """Additive DDM property: with one source subdomain, (i,j) is reached at
    step |i-i0|+|j-j0|+1; the sweep step formula reproduces it for the sweep
    whose direction points from (i0,j0) to (i,j)."""
    parts, src = (5, 5), (2, 2)
    for i in range(5):
        for j in range(5):
            D = (1 if i >= src[0] else -1, 1 if j >= src[1] else -1)
            assert step_of((i, j), D, parts) - step_of(src, D, parts) == abs(i - 2) + abs(j - 2)


def test_fgmres_with_ddm_converges_to_global_solution():
    n, h, om, pml, d = (64, 64), 1 / 64, 2 * np.pi * 6, 10, 5
    c = synth.layered_medium(*n, seed=0)
    f = embed_physical(synth.gaussian_source(n, h, (0.3, 0.05), 2 * h), pml).ravel()
    ddm = DiagonalSweepDDM(n, h, om, pml, d, (3, 3), slowness2(c))
    x, it, hist = fgmres(lambda v: ddm.M @ v, ddm.apply, f, tol=1e-11, restart=30, maxit=60)
    assert hist[-1] <= 1e-11 and it < 30
    assert _rel(x, global_solve(ddm.M, f)) < 1e-8
    # identity preconditioner and exact preconditioner: textbook special cases
    import scipy.sparse.linalg as spla
    lu = spla.splu(ddm.M.tocsc())
    x1, it1, _ = fgmres(lambda v: ddm.M @ v, lu.solve, f, tol=1e-12, maxit=5)
    assert it1 == 1 and _rel(x1, lu.solve(f)) < 1e-12


@pytest.mark.parametrize("n,parts,pml,d", [((48, 44), (3, 3), 6, 4), ((60, 52), (4, 3), 6, 4),
                                           ((14, 13, 12), (2, 2, 2), 3, 3)])
@pytest.mark.parametrize("med", ["const", "random"])
def test_additive_ddm_exact_mode_reproduces_global_solution(n, parts, pml, d, med):
    """Algorithms 2.1 / 2.2 (the additive overlapping DDM of Section 2) in exact
    mode: the discrete counterpart of its exactness result, for any medium with
    the index-form cutoffs."""
    h = 1 / n[0]
    om = 2 * np.pi * (3 if len(n) == 2 else 1.5)
    rng = np.random.default_rng(3)
    c = np.ones(n[::-1]) if med == "const" else 1 + 0.5 * rng.random(n[::-1])
    f = embed_physical(np.random.default_rng(1).standard_normal(n[::-1]), pml).ravel()
    a = AdditiveDDM(n, h, om, pml, d, parts, slowness2(c), mode="exact")
    assert _rel(a.apply(f), global_solve(a.M, f)) < 1e-12
