"""Pins for the oracle's grid, stretching and operator (oracle.pml).

* symmetry M = M^T, bitwise (the J-scaled form is complex symmetric);
* without PML and with constant medium the operator is the textbook 5/7-point
  Dirichlet Laplacian plus kappa^2, whose eigenvalues have a closed form;
* with PML the discrete operator is consistent, at second order, with the
  continuous J-scaled PML operator  div(A grad u) + kappa^2 J u  (Section 2.1,
  eq. (eq:PML) times J), evaluated analytically for a plane wave; a stretch
  taken at the wrong point (centre vs face), a missing J factor or a wrong
  sign fails the order test.
"""
import numpy as np
import pytest

from oracle.pml import assemble, global_axes, slowness2, stretch


def _grid(n, pml, h):
    return global_axes(n, pml, h)


def test_symmetric_bitwise():
    n, pml, h, om = (20, 17), 6, 1 / 20, 2 * np.pi * 3
    m = slowness2(1 + 0.3 * np.random.default_rng(0).random((n[1], n[0])))
    M = assemble(_grid(n, pml, h), m, h, om, pml)
    assert (M != M.T).nnz == 0
    n3 = (7, 6, 5)
    m3 = slowness2(1 + 0.3 * np.random.default_rng(1).random(n3[::-1]))
    M3 = assemble(_grid(n3, 3, 1 / 7), m3, 1 / 7, om, 3)
    assert (M3 != M3.T).nnz == 0


@pytest.mark.parametrize("n", [(9, 11), (5, 6, 4)])
def test_laplacian_eigenvalues_closed_form(n):
    """pml = 0, c = 1: eigenvalues are -4/h^2 sum_a sin^2(pi k_a / (2(n_a+1))) + omega^2."""
    h, om = 0.1, 2.0
    m = np.ones(n[::-1])
    M = assemble(_grid(n, 0, h), m, h, om, 0).toarray()
    ev = np.sort(np.linalg.eigvals(M).real)
    grids = np.meshgrid(*[np.arange(1, k + 1) for k in n], indexing="ij")
    lam = om ** 2 - 4 / h ** 2 * sum(np.sin(np.pi * g / (2 * (k + 1))) ** 2
                                     for g, k in zip(grids, n))
    assert np.allclose(ev, np.sort(lam.ravel()), rtol=0, atol=1e-9 * abs(lam).max())


def _continuous(axes, n, h, pml, om, kvec, c0, s0d=60.0):
    """Analytic J-scaled PML operator applied to u = exp(i k.x) at the cell centres."""
    dim = len(n)
    xs = [(ax.cells - pml + 0.5) * h for ax in axes]
    W = pml * h
    s, ds = [], []
    for a, ax in enumerate(axes):
        x = xs[a]
        s.append(stretch(x, ax, h, pml, om, s0d))
        t_lo = np.maximum(0, ax.lo - x)
        t_hi = np.maximum(0, x - ax.hi)
        dsig = (s0d / W) * 2 * (t_hi - t_lo) / W ** 2      # d sigma / dx
        ds.append(1j * dsig / om)
    mesh = np.meshgrid(*xs[::-1], indexing="ij")[::-1]     # x first, arrays [.., y, x]
    u = np.exp(1j * sum(k * X for k, X in zip(kvec, mesh)))

    def along(a, arr):
        sh = [1] * dim
        sh[dim - 1 - a] = arr.size
        return arr.reshape(sh)

    out = 0
    for a in range(dim):
        other = 1
        for b in range(dim):
            if b != a:
                other = other * along(b, s[b])
        ka = kvec[a]
        out = out + other * 1j * ka * u * (1j * ka / along(a, s[a]) - along(a, ds[a]) / along(a, s[a]) ** 2)
    jac = 1
    for b in range(dim):
        jac = jac * along(b, s[b])
    return out + om ** 2 / c0 ** 2 * jac * u, u


def _mask(axes, pml, dim):
    """Cells away from the outer boundary and from the PML inner faces."""
    masks = []
    for ax in axes:
        g = ax.cells
        ok = (g >= 1) & (g <= ax.n - 2)
        ok &= np.abs(g - pml) >= 2
        ok &= np.abs(g - (ax.n - pml)) >= 2
        masks.append(ok)
    m = masks[0]
    for mk in masks[1:]:
        m = np.multiply.outer(mk, m)
    return m


@pytest.mark.parametrize("dim,s0d,levels", [(2, 8.0, [32, 64, 128]),
                                          (2, 60.0, [64, 128, 256]),
                                          (3, 8.0, [16, 32])])
def test_consistency_with_continuous_pml_operator(dim, s0d, levels):
    """Max relative consistency error on a plane wave decays at order 2
    (fixed physical PML width 1/4, so the PML is resolved ever more finely)."""
    om, c0 = 2 * np.pi * 1.5, 1.3
    kvec = (3.0, -2.0, 1.5)[:dim]
    errs = []
    for N in levels:
        h = 1.0 / N
        pml = N // 4
        n = (N,) * dim
        axes = _grid(n, pml, h)
        m = np.full(n[::-1], 1.0 / c0 ** 2)
        M = assemble(axes, m, h, om, pml, sigma0_delta=s0d)
        ref, u = _continuous(axes, n, h, pml, om, kvec, c0, s0d)
        Mu = (M @ u.ravel()).reshape(u.shape)
        mk = _mask(axes, pml, dim)
        errs.append(np.max(np.abs(Mu - ref)[mk]) / np.max(np.abs(ref)[mk]))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert errs[-1] < 6e-3
    assert min(rates) > 1.8, (errs, rates)
