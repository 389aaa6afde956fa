"""Diagonal sweeps: orders, transfer rules, Algorithms 3.1 (2D) and 4.1 (3D).

Paper: Section 3 (the 2^2 sweep directions in the order (+,+), (-,+), (+,-),
(-,-); the step of subdomain (i,j) in a sweep; Rule 3.1 "similar direction"
d1.d2 > 0; Rule 3.2 "opposite direction" for horizontal/vertical transfers;
Algorithm 3.1 and its assembly (eq:sumdiag2D)) and Section 4.1 (the order
(Sorder3D); similar direction in 3D: d1.d2 > 0 and d1(k) d2(k) >= 0; Rule 4.2
by projection onto the coordinate planes; Algorithm 4.1 and (eq:sumdiag3D)).

Two modes of the same algorithm:
  * ``real``  -- every local problem is the subdomain's own PML problem on its
                 extended local grid (the method as used in Section 5);
  * ``exact`` -- every local problem is replaced by the global PML problem
                 (global grid, global operator, cutoffs and truncations
                 evaluated on the global grid).  With the index-form cutoffs
                 the discrete source-transfer identity of Lemma 2.1 is exact,
                 so this mode reproduces the global solution up to rounding for
                 any medium; it is the discrete counterpart of Theorems 3.1 and
                 4.1 and is used to pin the scheduling, routing, transfer and
                 assembly logic.

Within a step the subdomains are independent; they are processed in
lexicographic order and incoming transfers are summed in the order they are
generated.
"""
from __future__ import annotations

from itertools import product
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse.linalg as spla

from .partition import Partition, directions
from .pml import assemble, global_axes

# --------------------------------------------------------------- orders and rules
ORDER_2D = [(1, 1), (-1, 1), (1, -1), (-1, -1)]
ORDER_3D = [(1, 1, 1), (-1, 1, 1), (1, -1, 1), (-1, -1, 1),
            (1, 1, -1), (-1, 1, -1), (1, -1, -1), (-1, -1, -1)]
# the other 3D order of Section 4.1: the L1 distance of each direction from the
# first one never decreases along the list
ORDER_3D_L1 = [(1, 1, 1), (-1, 1, 1), (1, -1, 1), (1, 1, -1),
               (-1, -1, 1), (-1, 1, -1), (1, -1, -1), (-1, -1, -1)]


def sweep_order(dim: int, variant: int = 0) -> List[Tuple[int, ...]]:
    """variant 0: (Sorder3D) (the 2D order in 3D, +z then -z); variant 1 (3D
    only): the L1-monotone order."""
    if dim == 2:
        if variant != 0:
            raise ValueError("2D has one sweep order")
        return ORDER_2D
    return ORDER_3D_L1 if variant == 1 else ORDER_3D


def similar(t: Sequence[int], D: Sequence[int]) -> bool:
    """Rule 3.1 (2D: t.D > 0) and Rule 4.1 (3D: t.D > 0 and t_k D_k >= 0)."""
    dot = sum(a * b for a, b in zip(t, D))
    if len(t) == 2:
        return dot > 0
    return dot > 0 and all(a * b >= 0 for a, b in zip(t, D))


def excluded(t: Sequence[int], D1: Sequence[int], D2: Sequence[int]) -> bool:
    """Rule 3.2 (2D) / Rule 4.2 (3D): a transfer made in sweep D1 is barred from
    sweep D2 if, in some coordinate plane, its projection has exactly one zero
    component and the projections of D1 and D2 are opposite.  In 2D the only
    plane is the xy-plane: an axial transfer is barred from the opposite sweep."""
    dim = len(t)
    planes = [(0, 1)] if dim == 2 else [(0, 1), (0, 2), (1, 2)]
    for a, b in planes:
        pt = (t[a], t[b])
        if sum(1 for c in pt if c == 0) != 1:
            continue
        if D1[a] == -D2[a] and D1[b] == -D2[b]:
            return True
    return False


def route(l: int, t: Sequence[int], dim: int, variant: int = 0) -> Optional[int]:
    """Smallest sweep l' >= l in which a transfer of direction t generated in
    sweep l may be used (Algorithm 3.1 / 4.1), or None (dropped)."""
    order = sweep_order(dim, variant)
    for lp in range(l, len(order)):
        if similar(t, order[lp]) and not excluded(t, order[l], order[lp]):
            return lp
    return None


def step_of(sub: Sequence[int], D: Sequence[int], parts: Sequence[int]) -> int:
    """1-based step of subdomain ``sub`` (0-based indices) in a sweep along D."""
    return sum((i if Dk > 0 else N - 1 - i) for i, Dk, N in zip(sub, D, parts)) + 1


def n_steps(parts: Sequence[int]) -> int:
    return sum(N - 1 for N in parts) + 1


def step_groups(D: Sequence[int], parts: Sequence[int]) -> List[List[Tuple[int, ...]]]:
    groups = [[] for _ in range(n_steps(parts))]
    for sub in product(*[range(N) for N in parts]):
        groups[step_of(sub, D, parts) - 1].append(sub)
    return groups


# ------------------------------------------------------------------------ the DDM
class LocalSpace:
    """The grid a subdomain's problem lives on, its operator and its factors."""

    def __init__(self, axes, M, lu):
        self.axes = axes
        self.shape = tuple(ax.n for ax in reversed(axes))
        self.N = int(np.prod(self.shape))
        self.M = M
        self.lu = lu

    def solve(self, r: np.ndarray) -> np.ndarray:
        return self.lu.solve(r)


class DiagonalSweepDDM:
    """Algorithm 3.1 / 4.1 as a linear map f -> u_DDM on the global grid.

    Vectors are (N, k) complex arrays, cell index with x fastest, one column
    per right-hand side.
    """

    def __init__(self, n, h, omega, pml, d, parts, m_phys, mode="real",
                 sigma0_delta=60.0, order_variant=0):
        if mode not in ("real", "exact"):
            raise ValueError(mode)
        self.mode = mode
        self.dim = len(n)
        self.part = Partition(n, parts, pml, d, h)
        self.gaxes = global_axes(n, pml, h)
        self.gshape = tuple(ax.n for ax in reversed(self.gaxes))
        self.N = int(np.prod(self.gshape))
        self.M = assemble(self.gaxes, m_phys, h, omega, pml, sigma0_delta).tocsc()
        self.variant = order_variant
        self.order = sweep_order(self.dim, order_variant)
        self.dirs = directions(self.dim)
        self.spaces: Dict[Tuple[int, ...], LocalSpace] = {}
        if mode == "exact":
            glu = spla.splu(self.M)
            for sub in self.part.subdomains:
                self.spaces[sub] = LocalSpace(self.gaxes, self.M, glu)
        else:
            for sub in self.part.subdomains:
                axes = self.part.local_axes(sub)
                Ml = assemble(axes, m_phys, h, omega, pml, sigma0_delta).tocsc()
                self.spaces[sub] = LocalSpace(axes, Ml, spla.splu(Ml))
        # per-subdomain cutoff / truncation tables on its own space
        self.beta00 = {s: self.part.beta00(s, self.spaces[s].axes).ravel()
                       for s in self.part.subdomains}
        self.own = {s: self.part.own_mask(s, self.spaces[s].axes).ravel()
                    for s in self.part.subdomains}

    # -- index maps between a space and the global grid ---------------------
    def _global_index(self, sp_: LocalSpace) -> np.ndarray:
        """Global flat index of every cell of a space (valid for cells that lie
        on the global grid; local PML cells map to the cell they overlay)."""
        idx = np.zeros((), dtype=np.int64)
        stride = 1
        for a, ax in enumerate(sp_.axes):
            g = ax.cells * stride
            idx = np.add.outer(g, idx) if idx.ndim else g
            stride *= self.gaxes[a].n
        return idx.ravel()

    def restrict_source(self, sub, f: np.ndarray) -> np.ndarray:
        """r^1_sub = f chi_{Omega_sub} on the subdomain's space."""
        sp_ = self.spaces[sub]
        gi = self._global_index(sp_)
        r = np.zeros((sp_.N, f.shape[1]), dtype=np.complex128)
        own = self.own[sub]
        r[own] = f[gi[own]]
        return r

    def transfer(self, sub, t, v: np.ndarray) -> Tuple[np.ndarray, Tuple[slice, ...]]:
        """Psi_{t; sub}(v) = -M_sub(beta_{t;sub} v) chi_{t;sub} on the sender's space.

        Returns the values on the truncation box (a sub-box of the sender's
        grid) together with the box in sender-local index slices."""
        sp_ = self.spaces[sub]
        k = v.shape[1]
        bt = self.part.beta(sub, t, sp_.axes).ravel()
        g = -(sp_.M @ (bt[:, None] * v))
        box = []
        for a, ax in enumerate(sp_.axes):
            pa = self.part.part(sub, a)
            cells = ax.cells
            if t[a] == 1:
                sel = np.nonzero(cells >= pa.o1)[0]
            elif t[a] == -1:
                sel = np.nonzero(cells < pa.o0)[0]
            else:
                sel = np.arange(ax.n)
            box.append(slice(int(sel[0]), int(sel[-1]) + 1))
        box_np = tuple(reversed(box))
        gv = g.reshape(sp_.shape + (k,))[box_np + (slice(None),)]
        return gv, box_np

    def _receiver_box(self, sub, nb, box_np) -> Tuple[slice, ...]:
        """Map a sender-local box to the receiver's space via global indices."""
        s_axes, r_axes = self.spaces[sub].axes, self.spaces[nb].axes
        out = []
        for a in range(self.dim):
            sl = box_np[self.dim - 1 - a]
            off = s_axes[a].g0 - r_axes[a].g0
            lo, hi = sl.start + off, sl.stop + off
            if lo < 0 or hi > r_axes[a].n:
                raise AssertionError("transfer box leaves the receiver's grid")
            out.append(slice(lo, hi))
        return tuple(reversed(out))

    def scatter(self, sub, v: np.ndarray, u: np.ndarray) -> None:
        """u_DDM += beta_{0;sub} v on the global grid."""
        sp_ = self.spaces[sub]
        gi = self._global_index(sp_)
        w = self.beta00[sub]
        nz = w != 0
        np.add.at(u, gi[nz], w[nz, None] * v[nz])

    def apply(self, f: np.ndarray, trace: Optional[dict] = None) -> np.ndarray:
        """u_DDM for the global (J-scaled) source(s) f, shape (N,) or (N, k)."""
        squeeze = f.ndim == 1
        f = f.reshape(self.N, -1).astype(np.complex128)
        k = f.shape[1]
        L = len(self.order)
        r = {(l, s): np.zeros((self.spaces[s].N, k), dtype=np.complex128)
             for l in range(L) for s in self.part.subdomains}
        for s in self.part.subdomains:
            r[(0, s)] += self.restrict_source(s, f)
        u = np.zeros((self.N, k), dtype=np.complex128)
        for l, D in enumerate(self.order):
            for step, group in enumerate(step_groups(D, self.part.parts), start=1):
                for sub in group:
                    rhs = r[(l, sub)]
                    v = self.spaces[sub].solve(rhs)
                    self.scatter(sub, v, u)
                    if trace is not None:
                        trace.setdefault("rhs_norm", {})[(l, step, sub)] = np.linalg.norm(rhs)
                    for t in self.dirs:
                        nb = tuple(i + ti for i, ti in zip(sub, t))
                        if not self.part.exists(nb):
                            continue
                        lp = route(l, t, self.dim, self.variant)
                        if lp is None:
                            continue
                        gv, box = self.transfer(sub, t, v)
                        rbox = self._receiver_box(sub, nb, box)
                        r[(lp, nb)].reshape(self.spaces[nb].shape + (k,))[rbox + (slice(None),)] += gv
                        if trace is not None:
                            trace.setdefault("transfer_norm", {})[(l, sub, t)] = np.linalg.norm(gv)
            if trace is not None:
                trace.setdefault("after_sweep", []).append(u.copy())
        return u[:, 0] if squeeze else u


def global_solve(M, f: np.ndarray) -> np.ndarray:
    """The global PML solution: sparse direct solve of the J-scaled system."""
    return spla.splu(M.tocsc()).solve(np.asarray(f, dtype=np.complex128))


class AdditiveDDM(DiagonalSweepDDM):
    """The additive overlapping DDM with source transfer (Section 2: Algorithm
    2.1 in 2D, 2.2 in 3D), the method the diagonal sweeps re-order.

    Step 1 solves every subdomain with its own source; at step s = 2..S
    (S = sum(N_a - 1) + 1) every subdomain solves with the transfers
    Psi_{t; sub - t}(u^{s - |t|_1}_{sub - t}) from all its neighbours, a
    neighbour at L1 distance |t|_1 contributing the solution of step
    s - |t|_1; u_DDM = sum over steps and subdomains of beta_{0; sub} u^s.
    Same local problems, cutoffs and transfers as the sweeps (both modes).
    """

    def apply(self, f: np.ndarray, trace: Optional[dict] = None) -> np.ndarray:
        squeeze = f.ndim == 1
        f = f.reshape(self.N, -1).astype(np.complex128)
        k = f.shape[1]
        S = n_steps(self.part.parts)
        u = np.zeros((self.N, k), dtype=np.complex128)
        sol: Dict[Tuple[int, Tuple[int, ...]], np.ndarray] = {}
        for s in range(1, S + 1):
            for sub in self.part.subdomains:
                if s == 1:
                    rhs = self.restrict_source(sub, f)
                else:
                    rhs = np.zeros((self.spaces[sub].N, k), dtype=np.complex128)
                    for t in self.dirs:
                        snd = tuple(i - ti for i, ti in zip(sub, t))
                        ss = s - sum(abs(ti) for ti in t)
                        if ss < 1 or not self.part.exists(snd):
                            continue
                        gv, box = self.transfer(snd, t, sol[(ss, snd)])
                        rbox = self._receiver_box(snd, sub, box)
                        rhs.reshape(self.spaces[sub].shape + (k,))[rbox + (slice(None),)] += gv
                v = self.spaces[sub].solve(rhs)
                sol[(s, sub)] = v
                self.scatter(sub, v, u)
            for key in [key for key in sol if key[0] <= s - self.dim]:
                del sol[key]                     # no later step reads them
        return u[:, 0] if squeeze else u
