"""Direct solve of the constant-medium PML problem by separation of variables.

TEST INFRASTRUCTURE ONLY (see the package docstring).

In a constant medium the J-scaled operator of Section 2.1 (second-order
central differences, Section 5) is a Kronecker sum.  Along one axis let
D be the face-to-cell difference matrix with Dirichlet ghosts, s_c the
stretch at the cell centres and s_f at the faces; the 1D stiffness is
T = -D^T diag(1/s_f) D / h^2 and the 1D mass S = diag(s_c).  The operator
multiplied through by J = prod_b s_b is then

    2D:  S_y (x) T_x + T_y (x) S_x + kappa^2 S_y (x) S_x
    3D:  S_z S_y T_x + S_z T_y S_x + T_z S_y S_x + kappa^2 S_z S_y S_x

(Kronecker products, slowest axis first).  With the eigendecomposition
S_a^{-1} T_a = V_a diag(lam_a) V_a^{-1} of every axis, M = S (V (x) ...)
diag(sum lam + kappa^2) (V (x) ...)^{-1} where S is the Kronecker product of
the masses, so the solve is three (two) 1D transforms and a division.  It
shares nothing with the sparse LU (no sparse matrix, no factorisation of M),
which makes it an independent check of the global discrete solution.

The 1D PML operators are far from normal: the eigenvector bases lose a few
digits as the PML grows, so callers check the residual with the sparse
operator (``residual``) before trusting a solution.
"""
from __future__ import annotations

from typing import List, Sequence

import numpy as np

from .pml import axis_stretches, global_axes


def axis_operators(ax, h: float, pml: int, omega: float, sigma0_delta: float):
    """(T, s_c) of one axis: stiffness with Dirichlet ghosts, centre stretch."""
    sc, sf = axis_stretches(ax, h, pml, omega, sigma0_delta)
    m = ax.n
    D = np.zeros((m + 1, m))
    D[np.arange(m), np.arange(m)] = 1.0
    D[np.arange(1, m + 1), np.arange(m)] = -1.0
    T = -(D.T @ np.diag(1.0 / sf) @ D) / h ** 2
    return T, sc


def solve_constant(n: Sequence[int], h: float, omega: float, pml: int, c0: float,
                   f: np.ndarray, sigma0_delta: float = 60.0) -> np.ndarray:
    """u with M u = f on the global grid (physical n cells per axis plus pml
    on each side), medium c = c0 everywhere; f and u flat, x fastest."""
    axes = global_axes(n, pml, h)
    dim = len(axes)
    lam: List[np.ndarray] = []
    V: List[np.ndarray] = []
    Vinv: List[np.ndarray] = []
    S: List[np.ndarray] = []
    for ax in axes:
        T, sc = axis_operators(ax, h, pml, omega, sigma0_delta)
        l, P = np.linalg.eig(T / sc[:, None])
        lam.append(l)
        V.append(P)
        Vinv.append(np.linalg.inv(P))
        S.append(sc)
    shape = tuple(ax.n for ax in reversed(axes))          # slowest axis first
    G = f.reshape(shape).astype(np.complex128)
    # divide by the Kronecker product of the masses
    for a in range(dim):
        sh = [1] * dim
        sh[dim - 1 - a] = axes[a].n
        G = G / S[a].reshape(sh)
    # to the eigenbasis of every axis: apply V_a^{-1} along array axis dim-1-a
    for a in range(dim):
        G = np.moveaxis(np.tensordot(Vinv[a], G, axes=([1], [dim - 1 - a])), 0, dim - 1 - a)
    denom = np.full(shape, omega ** 2 / c0 ** 2, dtype=np.complex128)
    for a in range(dim):
        sh = [1] * dim
        sh[dim - 1 - a] = axes[a].n
        denom = denom + lam[a].reshape(sh)
    U = G / denom
    for a in range(dim):
        U = np.moveaxis(np.tensordot(V[a], U, axes=([1], [dim - 1 - a])), 0, dim - 1 - a)
    return U.ravel()


def residual(M, u: np.ndarray, f: np.ndarray) -> float:
    """||f - M u|| / ||f|| with a sparse operator M (the caller's check)."""
    return float(np.linalg.norm(f - M @ u) / np.linalg.norm(f))
