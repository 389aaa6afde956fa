"""Grid, complex coordinate stretching and the J-scaled finite-difference operator.

Paper: Section 2.1 -- the stretched coordinates (alpha_j = 1 + i sigma_j), the
PML equation  J^{-1} div(A grad u) + kappa^2 u = f  with
A = diag(a2/a1, a1/a2) (2D) or diag(a2 a3/a1, a1 a3/a2, a1 a2/a3) (3D) and
J = a1 a2 (a3); the shifted profile (eq:PMLprofile) for subdomain problems;
Section 5 -- second-order central differences (5-point / 7-point).

Readings (the paper leaves these open):
  * profile: s = 1 + i sigma/omega, sigma(t) = sigma0 (t/W)^2, sigma0 = S/W with
    W = (PML cells) * h and S = 60, t the physical distance beyond the inner
    face of the PML;
  * cell-centred grid: physical cell i of an axis has centre (i + 1/2) h, the
    PML adds ``pml`` cells on each side, homogeneous Dirichlet ghosts lie one
    cell beyond;
  * the operator is multiplied through by J, giving the complex-symmetric
        (M u)_c = sum_axes h^-2 [ a_{c+} (u_{c+1} - u_c) - a_{c-} (u_c - u_{c-1}) ]
                  + omega^2 m_c prod_b s_b(c) u_c,
    with the face coefficient along axis a equal to
        prod_{b != a} s_b(cell centre) / s_a(face);
  * the medium m = 1/c^2 is extended into the PML by clamping the index to the
    nearest physical cell.

An axis is described by :class:`Axis` (which global array cells it spans, where
its PML starts on each side, and the clamp range of its medium), so the same
assembly serves the global problem and every subdomain problem.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Sequence

import numpy as np
import scipy.sparse as sp


@dataclass(frozen=True)
class Axis:
    """One axis of a grid, in global array indices (PML cells included).

    Global array index ``g`` is physical cell ``g - pml``; its centre is at
    ``(g - pml + 1/2) h`` and its low face at ``(g - pml) h``.
    """
    g0: int          # global array index of the first cell
    n: int           # number of cells
    lo: float        # physical coordinate of the low-side PML inner face
    hi: float        # physical coordinate of the high-side PML inner face
    clo: int         # medium clamp range (global array indices, inclusive)
    chi: int

    @property
    def cells(self) -> np.ndarray:
        return np.arange(self.g0, self.g0 + self.n)


def global_axis(n_phys: int, pml: int, h: float) -> Axis:
    return Axis(0, n_phys + 2 * pml, 0.0, n_phys * h, pml, n_phys + pml - 1)


def stretch(x: np.ndarray, ax: Axis, h: float, pml: int, omega: float,
            sigma0_delta: float) -> np.ndarray:
    """s(x) = 1 + i sigma(x)/omega with sigma = sigma0 (t/W)^2 beyond [lo, hi]."""
    x = np.asarray(x, dtype=np.float64)
    if pml == 0:
        return np.ones_like(x, dtype=np.complex128)
    W = pml * h
    t = np.maximum(0.0, np.maximum(ax.lo - x, x - ax.hi))
    sigma = (sigma0_delta / W) * (t / W) ** 2
    return 1.0 + 1j * sigma / omega


def axis_stretches(ax: Axis, h: float, pml: int, omega: float, sigma0_delta: float):
    """Stretch at the cell centres (len n) and at the cell faces (len n + 1)."""
    g = np.arange(ax.g0, ax.g0 + ax.n + 1)
    xc = (g[:-1] - pml + 0.5) * h
    xf = (g - pml) * h
    return (stretch(xc, ax, h, pml, omega, sigma0_delta),
            stretch(xf, ax, h, pml, omega, sigma0_delta))


def medium_on(axes: Sequence[Axis], m_phys: np.ndarray, pml: int) -> np.ndarray:
    """m = 1/c^2 on the grid of ``axes`` (shape reversed(n)), clamped extension."""
    idx = [np.clip(ax.cells, ax.clo, ax.chi) - pml for ax in axes]
    # m_phys is indexed [.., iy, ix]; build the open mesh slowest axis first
    return m_phys[np.ix_(*reversed(idx))]


def assemble(axes: Sequence[Axis], m_phys: np.ndarray, h: float, omega: float,
             pml: int, sigma0_delta: float = 60.0) -> sp.csr_matrix:
    """J-scaled PML Helmholtz operator on the grid spanned by ``axes`` (x first).

    ``m_phys`` is the squared slowness 1/c^2 on the physical cells.

    Stencil form: every interior face contributes the symmetric pair of
    off-diagonal entries, every face (boundary faces included: Dirichlet ghost)
    subtracts its coefficient from the diagonal of the cells it touches.
    """
    dim = len(axes)
    shape = tuple(ax.n for ax in reversed(axes))          # (nz,) ny, nx
    N = int(np.prod(shape))
    sc, sf = zip(*[axis_stretches(ax, h, pml, omega, sigma0_delta) for ax in axes])
    idx = np.arange(N).reshape(shape)
    rows, cols, vals = [], [], []
    diag = np.zeros(shape, dtype=np.complex128)

    def along(a, arr):
        """Reshape a per-axis 1D array so that it broadcasts along axis a."""
        s = [1] * dim
        s[dim - 1 - a] = arr.shape[0]
        return arr.reshape(s)

    for a in range(dim):
        # product of the other axes' centre stretches, broadcast on the grid
        other = np.ones(shape, dtype=np.complex128)
        for b in range(dim):
            if b != a:
                other = other * along(b, sc[b])
        ax_dim = dim - 1 - a                              # numpy axis of grid axis a
        # coefficient at the low face and the high face of every cell
        lo_face = other / along(a, sf[a][:-1]) / h ** 2
        hi_face = other / along(a, sf[a][1:]) / h ** 2
        diag -= lo_face + hi_face
        # off-diagonal pairs across interior faces: cell c and its +1 neighbour
        sl_lo = [slice(None)] * dim
        sl_hi = [slice(None)] * dim
        sl_lo[ax_dim] = slice(0, shape[ax_dim] - 1)
        sl_hi[ax_dim] = slice(1, shape[ax_dim])
        coef = hi_face[tuple(sl_lo)]
        i0 = idx[tuple(sl_lo)].ravel()
        i1 = idx[tuple(sl_hi)].ravel()
        c = coef.ravel()
        rows += [i0, i1]
        cols += [i1, i0]
        vals += [c, c]
    jac = np.ones(shape, dtype=np.complex128)
    for b in range(dim):
        jac = jac * along(b, sc[b])
    diag += omega ** 2 * medium_on(axes, m_phys, pml) * jac
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    M.sum_duplicates()
    return M


def jacobian(axes: Sequence[Axis], h: float, omega: float, pml: int,
             sigma0_delta: float = 60.0) -> np.ndarray:
    """J = prod_b s_b at the cell centres of the grid (shape reversed(n))."""
    dim = len(axes)
    shape = tuple(ax.n for ax in reversed(axes))
    jac = np.ones(shape, dtype=np.complex128)
    for b, ax in enumerate(axes):
        s, _ = axis_stretches(ax, h, pml, omega, sigma0_delta)
        sh = [1] * dim
        sh[dim - 1 - b] = ax.n
        jac = jac * s.reshape(sh)
    return jac


def slowness2(c_phys: np.ndarray) -> np.ndarray:
    """m = 1/c^2 on the physical cells."""
    return 1.0 / np.asarray(c_phys, dtype=np.float64) ** 2


def embed_physical(f_phys: np.ndarray, pml: int) -> np.ndarray:
    """Zero-pad a physical-cell array with ``pml`` cells on every side."""
    return np.pad(np.asarray(f_phys), pml)


def global_axes(n: Sequence[int], pml: int, h: float) -> List[Axis]:
    return [global_axis(k, pml, h) for k in n]
