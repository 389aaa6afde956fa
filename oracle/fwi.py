"""FWI data misfit and its gradient with respect to the squared slowness.

Paper: Remark 2 of Section 4 names full-waveform inversion (a forward and an
adjoint wavefield per shot, then the misfit gradient) as the multi-RHS use of
the method, but gives no formula.  The formulas below are derived from the
discrete system used everywhere else:

    M(m) u_s = f_s        (J-scaled PML operator, m = 1/c^2 on physical cells,
                           extended into the PML by index clamping)
    J(m) = 1/2 sum_s || P u_s - d_s ||^2          (P samples receiver cells)

M depends on m only through its diagonal omega^2 m_c J_c, so for the extended
medium  dJ/dm_c = -omega^2 Re( sum_s conj(lam_{s,c}) J_c u_{s,c} )  with the
adjoint field  M^H lam_s = P^T (P u_s - d_s).  M is complex symmetric, so
M^H = conj(M) and lam_s = conj( M^{-1} conj(P^T r_s) ).  The gradient on the
physical cells is the transpose of the clamp extension: every global cell adds
its value to the physical cell it was clamped to.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np
import scipy.sparse.linalg as spla

from .pml import assemble, embed_physical, global_axes, jacobian


class FWIOracle:
    def __init__(self, n, h, omega, pml, sources_phys: np.ndarray,
                 receivers: Tuple[np.ndarray, np.ndarray], sigma0_delta=60.0):
        self.n, self.h, self.omega, self.pml, self.s0 = tuple(n), h, omega, pml, sigma0_delta
        self.axes = global_axes(n, pml, h)
        self.gshape = tuple(ax.n for ax in reversed(self.axes))
        self.N = int(np.prod(self.gshape))
        self.F = np.stack([embed_physical(s, pml).ravel() for s in sources_phys], axis=1)
        iy, ix = receivers
        self.rec = (iy + pml) * self.gshape[1] + (ix + pml)
        self.J = jacobian(self.axes, h, omega, pml, sigma0_delta).ravel()
        # clamp map: global cell -> physical cell
        gy = np.clip(np.arange(self.gshape[0]) - pml, 0, n[1] - 1)
        gx = np.clip(np.arange(self.gshape[1]) - pml, 0, n[0] - 1)
        self.clamp = (gy[:, None] * n[0] + gx[None, :]).ravel()

    def operator(self, m_phys: np.ndarray):
        return assemble(self.axes, m_phys, self.h, self.omega, self.pml, self.s0).tocsc()

    def fields(self, m_phys: np.ndarray) -> np.ndarray:
        return spla.splu(self.operator(m_phys)).solve(self.F.astype(np.complex128))

    def misfit(self, m_phys: np.ndarray, d_obs: np.ndarray) -> float:
        U = self.fields(m_phys)
        res = U[self.rec, :] - d_obs
        return 0.5 * float(np.sum(np.abs(res) ** 2))

    def gradient(self, m_phys: np.ndarray, d_obs: np.ndarray) -> Tuple[float, np.ndarray]:
        lu = spla.splu(self.operator(m_phys))
        U = lu.solve(self.F.astype(np.complex128))
        res = U[self.rec, :] - d_obs
        PtR = np.zeros_like(U)
        PtR[self.rec, :] = res
        lam = np.conj(lu.solve(np.conj(PtR)))
        g_ext = -self.omega ** 2 * np.real(np.sum(np.conj(lam) * U, axis=1) * self.J)
        g = np.zeros(self.n[0] * self.n[1])
        np.add.at(g, self.clamp, g_ext)
        return 0.5 * float(np.sum(np.abs(res) ** 2)), g.reshape(self.n[1], self.n[0])

    def observed(self, m_phys: np.ndarray) -> np.ndarray:
        return self.fields(m_phys)[self.rec, :]
