"""Pins for the oracle's global PML solve (the reference every DDM result is measured against).

* free-space solution: for a Gaussian source in constant medium the PML
  solution inside the physical box is the outgoing Helmholtz solution
  u = G * f with G(r) = -(i/4) H0^(1)(kappa r) (Section 1: Helmholtz with the
  Sommerfeld condition; Section 2.1: the PML solution equals u inside the box).
  It is evaluated here by the Graf addition theorem as two 1D quadratures and
  the discrete solution must converge to it at order 2;
* separable solve (``oracle.separable``): in constant medium the J-scaled
  operator is the Kronecker form S_y (x) T_x + T_y (x) S_x + kappa^2 S_y (x) S_x
  (3D alike), solved by 1D eigendecompositions (fast diagonalisation), an
  algorithm that shares nothing with the sparse LU; the two agree in 2D and 3D.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
from scipy.integrate import quad
from scipy.interpolate import RegularGridInterpolator
from scipy.special import hankel1, j0

from oracle.pml import assemble, embed_physical, global_axes
from oracle.separable import residual, solve_constant


def _free_space_radial(r, kappa, w):
    """u(r) for f(rho) = exp(-rho^2/(2 w^2)) in R^2, (Delta + kappa^2) u = f, outgoing."""
    f = lambda p: np.exp(-p * p / (2 * w * w))
    R = 12 * w

    def cquad(fun, a, b):
        re = quad(lambda p: fun(p).real, a, b, limit=200)[0]
        im = quad(lambda p: fun(p).imag, a, b, limit=200)[0]
        return re + 1j * im

    inner = cquad(lambda p: f(p) * j0(kappa * p) * p + 0j, 0.0, min(r, R)) if r > 0 else 0.0
    outer = cquad(lambda p: f(p) * hankel1(0, kappa * p) * p, r, max(r, R)) if r < R else 0.0
    return -(1j / 4) * 2 * np.pi * (hankel1(0, kappa * r) * inner + j0(kappa * r) * outer)


@pytest.mark.slow
def test_converges_to_free_space_solution():
    kappa = 2 * np.pi * 3
    w = 0.06
    centre = (0.5, 0.5)
    # fixed physical sample points, shared by all grids
    pts = np.array([[0.5 + 0.35 * np.cos(a), 0.5 + 0.35 * np.sin(a)]
                    for a in np.linspace(0, 2 * np.pi, 12, endpoint=False)] +
                   [[0.5 + 0.2, 0.5], [0.5, 0.5 - 0.15], [0.82, 0.11], [0.13, 0.9]])
    exact = np.array([_free_space_radial(np.hypot(*(p - centre)), kappa, w) for p in pts])
    errs = []
    for N in (80, 160, 320):
        h = 1.0 / N
        pml = N // 8
        n = (N, N)
        axes = global_axes(n, pml, h)
        M = assemble(axes, np.ones((N, N)), h, kappa, pml).tocsc()
        x = (np.arange(N) + 0.5) * h
        f = np.exp(-((x[None, :] - centre[0]) ** 2 + (x[:, None] - centre[1]) ** 2) / (2 * w * w))
        u = spla.splu(M).solve(embed_physical(f, pml).ravel().astype(complex))
        U = u.reshape(N + 2 * pml, N + 2 * pml)[pml:-pml, pml:-pml]
        # the points are not cell centres of every grid: interpolate (cubic, O(h^4))
        itp = RegularGridInterpolator((x, x), U.T, method="cubic")
        errs.append(np.max(np.abs(itp(pts) - exact)) / np.max(np.abs(exact)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert errs[-1] < 2e-2, errs
    assert min(rates) > 1.7, (errs, rates)


@pytest.mark.parametrize("n,pml", [((40, 32), 8), ((64, 64), 8), ((48, 56), 6),
                                   ((14, 12, 10), 4), ((20, 20, 20), 6)])
def test_separable_solver_matches_sparse_lu(n, pml):
    """oracle.separable (1D eigendecompositions of the Kronecker factors) against
    the sparse LU of the assembled operator, in 2D and 3D.  The 1D PML
    operators are far from normal, so their eigenvector bases lose a few digits
    as the PML widens; at these widths the route keeps ~1e-11."""
    h, omega, c0 = 1.0 / n[0], 2 * np.pi * 5, 1.2
    rng = np.random.default_rng(7)
    f = embed_physical(rng.standard_normal(n[::-1]), pml).ravel().astype(complex)
    axes = global_axes(n, pml, h)
    M = assemble(axes, np.full(n[::-1], 1 / c0 ** 2), h, omega, pml).tocsc()
    u_lu = spla.splu(M).solve(f)
    u_fd = solve_constant(n, h, omega, pml, c0, f)
    assert np.linalg.norm(u_lu - u_fd) / np.linalg.norm(u_lu) < 1e-9
    assert residual(M, u_fd, f) < 1e-9
