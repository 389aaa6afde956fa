"""Flexible GMRES with the diagonal-sweeping DDM as right preconditioner.

Paper: Remark 1 of Section 4 (the DDM used as a preconditioner of a Krylov
solver, one preconditioner application = 2^n sweeps) and Section 5.2 (GMRES,
stopping at relative residual 1e-6).

Readings: right preconditioning in the flexible form (the preconditioned
directions Z are stored, so an inexact or lower-precision preconditioner can be
used), zero initial guess, modified Gram-Schmidt, restart after ``restart``
inner iterations from the current iterate; the relative residual is the true
2-norm residual ||b - M x|| / ||b|| of the J-scaled global system.
"""
from __future__ import annotations

from typing import Callable, List, Tuple

import numpy as np


def fgmres(matvec: Callable[[np.ndarray], np.ndarray],
           precond: Callable[[np.ndarray], np.ndarray],
           b: np.ndarray, tol: float = 1e-6, restart: int = 50,
           maxit: int = 200) -> Tuple[np.ndarray, int, List[float]]:
    """Solve M x = b for one right-hand side.

    Returns (x, total inner iterations, true relative residual after each restart cycle).
    """
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0:
        return x, 0, [0.0]
    history = []
    total = 0
    r = b.copy()
    while True:
        beta = np.linalg.norm(r)
        if beta / nb <= tol or total >= maxit:
            history.append(beta / nb)
            return x, total, history
        m = min(restart, maxit - total)
        V = np.zeros((b.size, m + 1), dtype=np.complex128)
        Z = np.zeros((b.size, m), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        V[:, 0] = r / beta
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        j_used = 0
        for j in range(m):
            Z[:, j] = precond(V[:, j])
            w = matvec(Z[:, j])
            for i in range(j + 1):                       # modified Gram-Schmidt
                H[i, j] = np.vdot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[:, j + 1] = w / H[j + 1, j]
            # complex Givens rotations G_i = [[conj(c_i), conj(s_i)], [-s_i, c_i]]
            for i in range(j):                           # apply earlier rotations
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, c = H[j, j], H[j + 1, j]                  # new rotation zeroing H[j+1, j]
            rho = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
            cs[j] = a / rho if rho else 1.0
            sn[j] = c / rho if rho else 0.0
            H[j, j] = rho
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            j_used = j + 1
            total += 1
            if abs(g[j + 1]) / nb <= tol:
                break
        y = np.linalg.solve(np.triu(H[:j_used, :j_used]), g[:j_used])
        x = x + Z[:, :j_used] @ y
        r = b - matvec(x)
        history.append(np.linalg.norm(r) / nb)


def ddm_iterate(matvec: Callable[[np.ndarray], np.ndarray],
                precond: Callable[[np.ndarray], np.ndarray],
                f: np.ndarray, iters: int) -> Tuple[np.ndarray, List[float]]:
    """The DDM as a stand-alone iterative solver (Section 5.2 runs the
    three-layer residual-decay test this way, without Krylov correction):
    x_0 = 0, x_{k+1} = x_k + precond(f - M x_k).

    Returns (x_iters, [||f - M x_k|| / ||f|| for k = 0..iters]).
    """
    f = np.asarray(f, dtype=np.complex128)
    nf = np.linalg.norm(f)
    x = np.zeros_like(f)
    r = f.copy()
    hist = [1.0 if nf > 0 else 0.0]
    for _ in range(iters):
        x = x + precond(r)
        r = f - matvec(x)
        hist.append(np.linalg.norm(r) / nf if nf > 0 else 0.0)
    return x, hist
