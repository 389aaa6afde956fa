"""The diagonal sweeps as a stand-alone iterative solver (Section 5.2, the
three-layer residual-decay test), on the oracle.

Pins: the iteration's fixed point is the global solution; the first iterate is
one DDM application; and the shape of the paper's experiment -- with the
medium interfaces and every subdomain interface inside the middle layer, a 3x3
partition decays at the per-iteration rate of the two-subdomain (1x2)
partition, the optimal rate, which for a speed contrast of 2 is close to the
normal-incidence round-trip reflection R^2 = ((c2 - c1) / (c2 + c1))^2 = 1/9.
"""
import numpy as np
import pytest

import synth
from oracle.krylov import ddm_iterate
from oracle.pml import assemble, global_axes, slowness2
from oracle.sweep import DiagonalSweepDDM, global_solve

N, PML, D = 64, 8, 4
H, OMEGA = 1.0 / N, 2 * np.pi * 4


def _run(parts, iters=10):
    c = synth.three_layer_medium(N, N)
    m = slowness2(c)
    M = assemble(global_axes((N, N), PML, H), m, H, OMEGA, PML)
    # the shot at (1/4 of a subdomain width, 1/3 of a subdomain height)
    f = synth.point_source(N, N, H, PML, 0.25 / parts[0], (1.0 / 3.0) / parts[1]).ravel()
    ddm = DiagonalSweepDDM((N, N), H, OMEGA, PML, D, parts, m)
    x, hist = ddm_iterate(lambda v: M @ v, ddm.apply, f, iters)
    return M, f, ddm, x, hist


def _rate(hist, k0=2, k1=8):
    return (hist[k1] / hist[k0]) ** (1.0 / (k1 - k0))


def test_first_iterate_is_one_sweep_application():
    M, f, ddm, x, hist = _run((2, 2), iters=1)
    u = ddm.apply(f)
    assert np.array_equal(x, u)
    assert hist[1] == pytest.approx(np.linalg.norm(f - M @ u) / np.linalg.norm(f), rel=1e-12)


@pytest.mark.parametrize("parts", [(1, 2), (3, 3)])
def test_fixed_point_is_the_global_solution(parts):
    M, f, ddm, x, hist = _run(parts)
    u = global_solve(M, f)
    assert hist[-1] < 1e-8
    assert np.linalg.norm(x - u) / np.linalg.norm(u) < 100 * hist[-1]


def test_three_by_three_decays_at_the_two_subdomain_rate():
    r12 = _rate(_run((1, 2))[4])
    r33 = _rate(_run((3, 3))[4])
    print(f"per-iteration residual ratio: 1x2 {r12:.4f}, 3x3 {r33:.4f}, R^2 = {1 / 9:.4f}")
    assert 0.09 < r12 < 0.13 and 0.09 < r33 < 0.13
    assert abs(r33 - r12) < 0.1 * r12
