"""Checkerboard partition, extended subdomains, cutoffs and truncations.

Paper: Section 2.1 (the partition Omega_{i,j}, the extended subdomains
tilde Omega_{i,j} with tilde xi_1 = -inf, tilde xi_{N+1} = +inf, decomposed
sources f_{ij} = f chi_{Omega_ij}; the 3D analogue) and Section 2.2 (the 1D
cutoffs beta^{(1)}_{box,i}, beta^{(2)}_{tri,j}, their products beta_{box,tri;ij}
and beta_{0,0;ij}, the truncations chi_{box,tri;ij} over the half/quarter spaces
I^{(1)} x I^{(2)}, and the transfer operator Psi = -L(beta v) chi).

Readings (the paper leaves these open or is garbled):
  * own cells per axis come from ``numpy.array_split`` of the physical cells
    (larger parts first); a part on a global-boundary side also owns the PML
    cells on that side (tilde xi_1 = -inf);
  * a subdomain's local grid adds, on each interior side, ``d`` overlap cells
    (true medium, no damping) and then ``pml`` cells of local PML whose profile
    is measured from the outer face of the overlap (eq:PMLprofile); on a
    boundary side it keeps the global PML;
  * the medium inside the local PML is the medium clamped to the local
    undamped box;
  * cutoffs in index form: for a side whose neighbour's first own cell is
    ``e``, beta(e + m) = bhat(m/(d-1)) for 0 <= m <= d-1, beta = 1 before e and
    0 from e+d-1 on (mirrored on the low side); bhat(t) = 1 - (10t^3 - 15t^4 +
    6t^5), the C^2 quintic smoothstep (the paper only asks for a monotone C^2
    cutoff).  This keeps beta = 1 on the whole stencil of every cell before e,
    so the transfer identity of Lemma 2.1 holds exactly for the discrete
    operator;
  * the truncation on that side is the set of cells >= e (<= e-1 on the low
    side), tangential axes unrestricted;
  * beta_{0,0;ij} is the product of both cutoffs of every axis; the upper
    index i+1 printed in its definition is read as i (cut at xi_{i+1}).
"""
from __future__ import annotations

from dataclasses import dataclass
from itertools import product
from typing import Dict, List, Sequence, Tuple

import numpy as np

from .pml import Axis, global_axis


def bhat(t: np.ndarray) -> np.ndarray:
    """Monotone C^2 cutoff: 1 for t <= 0, 0 for t >= 1 (quintic smoothstep)."""
    t = np.clip(np.asarray(t, dtype=np.float64), 0.0, 1.0)
    return 1.0 - t ** 3 * (10.0 - 15.0 * t + 6.0 * t * t)


@dataclass(frozen=True)
class AxisPart:
    """Part ``p`` of ``P`` along one axis."""
    p: int
    P: int
    q0: int          # physical own range [q0, q1)
    q1: int
    o0: int          # own range in global array indices [o0, o1)
    o1: int
    local: Axis      # the extended subdomain's local grid along this axis


def axis_parts(n_phys: int, P: int, pml: int, d: int, h: float) -> List[AxisPart]:
    chunks = np.array_split(np.arange(n_phys), P)
    out = []
    for p, ch in enumerate(chunks):
        q0, q1 = int(ch[0]), int(ch[-1]) + 1
        if P > 1 and q1 - q0 < d:
            raise ValueError("every part must own at least d cells")
        o0 = 0 if p == 0 else q0 + pml
        o1 = n_phys + 2 * pml if p == P - 1 else q1 + pml
        g0 = 0 if p == 0 else q0 - d
        g1 = n_phys + 2 * pml if p == P - 1 else q1 + d + 2 * pml
        lo = 0.0 if p == 0 else (q0 - d) * h
        hi = n_phys * h if p == P - 1 else (q1 + d) * h
        clo = pml if p == 0 else q0 - d + pml
        chi = n_phys + pml - 1 if p == P - 1 else q1 + d + pml - 1
        out.append(AxisPart(p, P, q0, q1, o0, o1, Axis(g0, g1 - g0, lo, hi, clo, chi)))
    return out


def cutoff(part: AxisPart, comp: int, g: np.ndarray, d: int) -> np.ndarray:
    """beta^{(a)}_{comp, p} evaluated at global array indices ``g``."""
    g = np.asarray(g)
    if comp == 0:
        return np.ones(g.shape)
    if comp == 1:
        if part.p == part.P - 1:
            return np.ones(g.shape)
        e = part.o1
        return bhat((g - e) / (d - 1))
    if part.p == 0:
        return np.ones(g.shape)
    a = part.o0
    return bhat((a - 1 - g) / (d - 1))


def truncation(part: AxisPart, comp: int, g: np.ndarray) -> np.ndarray:
    """Indicator of I^{(a)}_{comp, p}: cells beyond the own range on that side."""
    g = np.asarray(g)
    if comp == 0:
        return np.ones(g.shape, dtype=bool)
    if comp == 1:
        return g >= part.o1
    return g < part.o0


def directions(dim: int) -> List[Tuple[int, ...]]:
    """All non-zero t in {-1,0,1}^dim, lexicographic with the x component first."""
    return [t for t in product((-1, 0, 1), repeat=dim) if any(t)]


class Partition:
    """The N_x x N_y (x N_z) checkerboard partition of a global grid."""

    def __init__(self, n: Sequence[int], parts: Sequence[int], pml: int, d: int, h: float):
        if d < 3:
            raise ValueError("overlap must be at least 3 cells")
        self.n, self.parts, self.pml, self.d, self.h = tuple(n), tuple(parts), pml, d, h
        self.dim = len(n)
        self.axis_parts = [axis_parts(n[a], parts[a], pml, d, h) for a in range(self.dim)]
        self.global_axes = [global_axis(n[a], pml, h) for a in range(self.dim)]
        self.subdomains = list(product(*[range(P) for P in parts]))

    def part(self, sub: Tuple[int, ...], a: int) -> AxisPart:
        return self.axis_parts[a][sub[a]]

    def exists(self, sub: Tuple[int, ...]) -> bool:
        return all(0 <= sub[a] < self.parts[a] for a in range(self.dim))

    def local_axes(self, sub) -> List[Axis]:
        return [self.part(sub, a).local for a in range(self.dim)]

    def own_mask(self, sub, axes: Sequence[Axis]) -> np.ndarray:
        """chi_{Omega_sub} on the grid of ``axes`` (shape reversed(n))."""
        m = np.ones((), dtype=bool)
        for a, ax in enumerate(axes):
            pa = self.part(sub, a)
            g = ax.cells
            ind = (g >= pa.o0) & (g < pa.o1)
            m = np.multiply.outer(ind, m) if m.ndim else ind
        return m

    def _outer(self, per_axis: List[np.ndarray]) -> np.ndarray:
        """Outer product of per-axis arrays (x first) in [.., y, x] layout."""
        out = per_axis[0]
        for arr in per_axis[1:]:
            out = np.multiply.outer(arr, out)
        return out

    def beta(self, sub, t: Tuple[int, ...], axes: Sequence[Axis]) -> np.ndarray:
        """beta_{t; sub} on the grid of ``axes``."""
        return self._outer([cutoff(self.part(sub, a), t[a], ax.cells, self.d)
                            for a, ax in enumerate(axes)])

    def beta00(self, sub, axes: Sequence[Axis]) -> np.ndarray:
        """beta_{0,..,0; sub}: both cutoffs of every axis."""
        return self._outer([cutoff(self.part(sub, a), -1, ax.cells, self.d) *
                            cutoff(self.part(sub, a), 1, ax.cells, self.d)
                            for a, ax in enumerate(axes)])

    def chi(self, sub, t: Tuple[int, ...], axes: Sequence[Axis]) -> np.ndarray:
        return self._outer([truncation(self.part(sub, a), t[a], ax.cells)
                            for a, ax in enumerate(axes)])
