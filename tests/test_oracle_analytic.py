"""Pins of the free-space solutions behind the accuracy tables, and of the
oracle's discretisation against the paper's own printed errors.

* The Gaussian sources integrate to one (2D and 3D).
* The radial solutions satisfy  u'' + (dim - 1)/r u' + kappa^2 u = f  (the
  equation they are defined by; checked by centred differences), inside the
  source and beyond it, and the near-field quadrature meets the closed far form.
* The oracle's global sparse LU solution of the PML problem at the first row
  of Table 1 (Section 5.1: 2D, kappa/2pi = 25, mesh 560^2) has the printed L2
  error 3.13e-3 against the free-space solution, and the error falls by a
  factor of four per mesh halving at a lower frequency (second order).
"""
import json
import os

import numpy as np
import pytest
from scipy import integrate

from oracle.analytic import free_space, gaussian_source, l2_error, support_radius
from oracle.pml import assemble, global_axes
from oracle.sweep import global_solve

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "accuracy_tables.json")


@pytest.mark.parametrize("dim", [2, 3])
def test_source_integrates_to_one(dim):
    kappa = 2 * np.pi * (25 if dim == 2 else 10)
    R = support_radius(kappa)
    shell = 2 * np.pi if dim == 2 else 4 * np.pi
    total, _ = integrate.quad(lambda r: shell * r ** (dim - 1) * gaussian_source(kappa, dim, r),
                              0, R, epsabs=0, epsrel=1e-12, limit=200)
    assert abs(total - 1.0) < 1e-10


@pytest.mark.parametrize("dim", [2, 3])
def test_free_space_solves_the_radial_equation(dim):
    kappa = 2 * np.pi * (25 if dim == 2 else 10)
    R = support_radius(kappa)
    d = R / 400
    for r in [0.15 * R, 0.4 * R, 0.7 * R, 1.5 * R, 3.0 * R]:
        um, u0, up = free_space(kappa, dim, np.array([r - d, r, r + d]))
        lhs = (up - 2 * u0 + um) / d ** 2 + (dim - 1) / r * (up - um) / (2 * d) + kappa ** 2 * u0
        f = gaussian_source(kappa, dim, r)
        scale = max(abs(f), kappa ** 2 * abs(u0))
        assert abs(lhs - f) <= 2e-3 * scale, (dim, r / R, lhs, f)


@pytest.mark.parametrize("dim", [2, 3])
def test_near_table_meets_far_form(dim):
    """At the edge of the source's support the quadrature (inner and outer
    radial integrals) equals the closed far form (Fourier transform of f)."""
    from oracle.analytic import _far, _near_table
    kappa = 2 * np.pi * (25 if dim == 2 else 10)
    R = support_radius(kappa)
    rho, u = _near_table(kappa, dim, 400001)
    far = _far(kappa, dim, np.array([R]))[0]
    assert rho[-1] == R and abs(u[-1] - far) <= 1e-9 * abs(far)


def _table1_problem(N, kappa_over_2pi, l):
    kappa = 2 * np.pi * kappa_over_2pi
    h = 1.0 / N
    n = int(round(2 * l / h))
    pml = (N - n) // 2
    x0 = (0.09 + l, 0.268 + l)        # the paper's centre, domain shifted to [0, 2l]
    c = (np.arange(n) + 0.5) * h
    Y, X = np.meshgrid(c, c, indexing="ij")
    f = gaussian_source(kappa, 2, np.sqrt((X - x0[0]) ** 2 + (Y - x0[1]) ** 2))
    M = assemble(global_axes((n, n), pml, h), np.ones((n, n)), h, kappa, pml)
    u = global_solve(M, np.pad(f, pml).astype(complex).ravel()).reshape(N, N)
    return l2_error(u[pml:pml + n, pml:pml + n], h, x0, kappa)


def test_table1_first_row_reproduced_by_the_oracle():
    tab = json.load(open(GOLDEN))["table1_2d"]
    mesh, _, l2_paper, _ = tab["rows"][0]
    e = _table1_problem(mesh, tab["kappa_over_2pi"], tab["l"])
    print(f"Table 1, {mesh}^2: oracle L2 error {e:.4e} (paper {l2_paper:.2e})")
    assert f"{e:.2e}" == f"{l2_paper:.2e}"


def test_second_order_convergence_at_lower_frequency():
    l = json.load(open(GOLDEN))["table1_2d"]["l"]
    errs = [_table1_problem(N, 6, l) for N in (112, 224, 448)]
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    print("errors", errs, "ratios", ratios)
    assert all(3.9 < q < 4.2 for q in ratios)


def test_table2_oracle_values_and_printed_rate():
    """Table 2 (Section 5.1, 3D): tests/golden/table2_oracle.json holds the
    oracle's L2 errors at 80^3, 96^3, 128^3 and 160^3 with the printed
    unit-mass source (the values the GPU is held to; 160^3 is not run on the
    GPU).  The first three are reproduced here from oracle/ alone (separable
    direct solve, residual under the sparse operator <= 1e-9, 1e-7 at 128^3), and
    their ratio equals the printed ratio 2.67e-2 / 1.82e-2 within 1%: the
    printed rate is matched, the printed level is a constant 1.77 times
    lower, so parity with the printed values is unpinned."""
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(__file__), "golden"))
    from make_table2_oracle import table2_problem
    from oracle.separable import residual, solve_constant
    tab = json.load(open(GOLDEN))["table2_3d"]
    stored = json.load(open(os.path.join(os.path.dirname(GOLDEN), "table2_oracle.json")))["rows"]
    errs = {}
    for mesh in (80, 96, 128):
        dim, kappa, h, n, pml, x0, f = table2_problem(tab, mesh)
        u = solve_constant((n,) * dim, h, kappa, pml, 1.0, f.ravel())
        M = assemble(global_axes((n,) * dim, pml, h), np.ones((n,) * dim), h, kappa, pml)
        assert residual(M, u, f.ravel()) < (1e-9 if mesh < 128 else 1e-7)
        sl = (slice(pml, pml + n),) * dim
        errs[mesh] = l2_error(u.reshape(f.shape)[sl], h, x0, kappa)
        assert abs(errs[mesh] / stored[str(mesh)]["l2_error"] - 1) < 1e-10
    printed = {r[0]: r[2] for r in tab["rows"]}
    assert abs((errs[80] / errs[96]) / (printed[80] / printed[96]) - 1) < 0.01
    print("oracle / printed:", {k: errs[k] / printed[k] for k in errs})
