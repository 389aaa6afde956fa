"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds only workload descriptions and random-input generators
(media, sources, receivers, perturbation directions).  It contains none of the
method's arithmetic: no stretching, no operator, no cutoff, no solve.  Both the
CPU oracle and the GPU path consume the arrays it returns, so a parity test
feeds both sides exactly the same bytes.

Conventions (shared by every consumer):
  * cell-centred grids, physical cell ``i`` of an axis sits at ``(i + 1/2) h``;
  * 2D arrays are indexed ``[iy, ix]`` (x fastest), 3D arrays ``[iz, iy, ix]``;
  * ``y`` is depth (``y = 0`` at the top surface).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np
from scipy.ndimage import gaussian_filter

__all__ = [
    "Workload", "WORKLOADS", "workload",
    "layered_medium", "grf_medium_3d", "constant_medium",
    "gaussian_source", "surface_gaussian_sources", "random_gaussian_sources_3d",
    "surface_receivers", "smooth_directions", "smooth_medium",
]


@dataclass(frozen=True)
class Workload:
    """One synthetic problem: grid, frequency, PML, partition and sources."""
    name: str
    n: Tuple[int, ...]            # physical cells per axis (x, y[, z])
    h: float                      # cell size
    omega: float                  # angular frequency
    pml: int                      # PML width in cells (global and local)
    overlap: int                  # overlap d in cells
    parts: Tuple[int, ...]        # subdomains per axis
    nrhs: int
    medium: str                   # "constant" | "layered" | "grf3d"
    sigma0_delta: float = 60.0    # sigma0 * (PML width) ; sigma = sigma0 (t/width)^2
    seed: int = 0
    note: str = ""
    restart: int = 30             # FGMRES restart length the benchmark uses
    solver: str = "auto"          # local solver the benchmark uses

    @property
    def dim(self) -> int:
        return len(self.n)


WORKLOADS = {
    # 2x2 constant medium, one centred Gaussian, four sweeps, no Krylov.
    "c1": Workload("c1", (128, 128), 1.0 / 128, 2 * np.pi * 8, 16, 8, (2, 2), 1, "constant"),
    # 8x8 layered medium, 16 surface shots, GMRES to 1e-6.  Nested dissection:
    # its subdomains span few enough wavelengths (7) for well-conditioned
    # separator blocks, and it solves faster than the cyclic reduction here.
    "c2": Workload("c2", (1024, 1024), 1.0 / 1024, 2 * np.pi * 40, 20, 10, (8, 8), 16, "layered",
                   solver="nd"),
    # 16x16 uneven partition, 128 surface shots.  FGMRES(10): it converges in 8-9
    # iterations, and the shorter basis lets one batch hold more of the 128 RHS
    # (fewer passes over the factors).  Nested dissection, as for c2.
    "c3": Workload("c3", (2050, 1990), 1.0 / 2048, 2 * np.pi * 60, 20, 10, (16, 16), 128, "layered",
                   restart=10, solver="nd"),
    # 3D at half the resolution and frequency (80^3, 4x4x4).
    "c4r": Workload("c4r", (80, 80, 80), 1.0 / 80, 2 * np.pi * 6, 8, 4, (4, 4, 4), 32, "grf3d"),
    # 3D as stated.  FGMRES(8): it converges in 4 iterations, and the FP64 Krylov
    # vectors of all 32 right-hand sides at restart 30 (65 vectors of 5.45M
    # cells each) would not fit beside the factors, splitting the solve into
    # four batches that each stream every factor.
    "c4": Workload("c4", (160, 160, 160), 1.0 / 160, 2 * np.pi * 12, 8, 4, (4, 4, 4), 32, "grf3d",
                   restart=8),
    # FWI gradient workload, 64 shots and 128 receivers.
    "c5": Workload("c5", (512, 512), 1.0 / 512, 2 * np.pi * 20, 20, 10, (8, 8), 64, "layered"),
}


def workload(name: str, **overrides) -> Workload:
    w = WORKLOADS[name]
    return replace(w, **overrides) if overrides else w


# --------------------------------------------------------------------------- media
def constant_medium(n: Tuple[int, ...], c: float = 1.0) -> np.ndarray:
    return np.full(tuple(reversed(n)), float(c))


def layered_medium(nx: int, ny: int, seed: int = 0, n_interfaces: int = 5,
                   vmin: float = 1.5, vmax: float = 4.5, noise: float = 0.05,
                   corr_cells: float = 20.0) -> np.ndarray:
    """Layered wave speed c[iy, ix].

    ``n_interfaces`` depths drawn uniformly in (0, 1) (as a fraction of the
    domain height) and sorted; layer speeds ``linspace(vmin, vmax)`` increase
    with depth.  The result is multiplied by ``1 + noise * g`` where ``g`` is
    white noise smoothed by a Gaussian of ``corr_cells`` cells (reflecting
    boundaries) and renormalised to unit standard deviation.
    """
    rng = np.random.default_rng(seed)
    depths = np.sort(rng.uniform(0.0, 1.0, n_interfaces))
    speeds = np.linspace(vmin, vmax, n_interfaces + 1)
    frac = (np.arange(ny) + 0.5) / ny
    layer = np.searchsorted(depths, frac)
    c = np.repeat(speeds[layer][:, None], nx, axis=1)
    if noise:
        g = gaussian_filter(np.random.default_rng(seed + 1).standard_normal((ny, nx)),
                            corr_cells, mode="reflect")
        g = (g - g.mean()) / g.std()
        c = c * (1.0 + noise * g)
    return np.ascontiguousarray(c)


def three_layer_medium(nx: int, ny: int, speeds=(1.0, 2.0, 1.0),
                       cuts=(0.25, 0.75)) -> np.ndarray:
    """Three horizontal layers on [0,1]^2 (y = depth as a fraction of the domain),
    speeds top to bottom, interfaces at the depth fractions ``cuts``; (ny, nx)."""
    y = (np.arange(ny) + 0.5) / ny
    col = np.where(y < cuts[0], speeds[0], np.where(y < cuts[1], speeds[1], speeds[2]))
    return np.repeat(col[:, None], nx, axis=1).astype(np.float64)


def point_source(nx: int, ny: int, h: float, pml: int, x: float, y: float) -> np.ndarray:
    """Unit-mass discrete delta (1/h^2 in the cell holding (x, y)) on the global
    grid with the PML, shape (ny + 2 pml, nx + 2 pml), complex128."""
    f = np.zeros((ny + 2 * pml, nx + 2 * pml), np.complex128)
    f[pml + int(y / h), pml + int(x / h)] = 1.0 / h ** 2
    return f


def grf_medium_3d(n: int, seed: int = 0, mean: float = 2.0, std: float = 0.2,
                  corr_cells: float = 16.0) -> np.ndarray:
    """Smooth Gaussian random field c[iz, iy, ix] with the given mean and std."""
    g = gaussian_filter(np.random.default_rng(seed).standard_normal((n, n, n)),
                        corr_cells, mode="reflect")
    g = (g - g.mean()) / g.std()
    return np.ascontiguousarray(mean + std * g)


def smooth_medium(c: np.ndarray, cells: float) -> np.ndarray:
    """Gaussian smoothing of a medium (the FWI starting model)."""
    return np.ascontiguousarray(gaussian_filter(c, cells, mode="reflect"))


def medium_for(w: Workload) -> np.ndarray:
    if w.medium == "constant":
        return constant_medium(w.n, 1.0)
    if w.medium == "layered":
        return layered_medium(w.n[0], w.n[1], seed=w.seed)
    if w.medium == "grf3d":
        return grf_medium_3d(w.n[0], seed=w.seed)
    raise ValueError(w.medium)


# ------------------------------------------------------------------------- sources
def _centres(n: int, h: float) -> np.ndarray:
    return (np.arange(n) + 0.5) * h


def gaussian_source(n: Tuple[int, ...], h: float, centre, width: float) -> np.ndarray:
    """exp(-|x - centre|^2 / (2 width^2)) sampled at the physical cell centres."""
    axes = [_centres(k, h) for k in n]
    r2 = 0.0
    for a, x in enumerate(axes):
        shape = [1] * len(n)
        shape[len(n) - 1 - a] = n[a]
        r2 = r2 + ((x - centre[a]) ** 2).reshape(shape)
    return np.ascontiguousarray(np.exp(-r2 / (2.0 * width * width)))


def surface_gaussian_sources(nx: int, ny: int, h: float, nsrc: int, depth: float = 0.05,
                             width_cells: float = 2.0) -> np.ndarray:
    """``nsrc`` Gaussians at depth ``depth``, x uniformly spaced: (nsrc, ny, nx)."""
    L = nx * h
    xs = (np.arange(nsrc) + 0.5) / nsrc * L
    return np.stack([gaussian_source((nx, ny), h, (x, depth), width_cells * h) for x in xs])


def random_gaussian_sources_3d(n: int, h: float, nsrc: int, seed: int = 2,
                               width_cells: float = 2.0) -> np.ndarray:
    L = n * h
    pos = np.random.default_rng(seed).uniform(0.1 * L, 0.9 * L, (nsrc, 3))
    return np.stack([gaussian_source((n, n, n), h, p, width_cells * h) for p in pos])


def surface_receivers(nx: int, ny: int, h: float, nrec: int, depth: float = 0.05):
    """Receiver cells (iy, ix) at the cell row nearest ``depth``, x uniform."""
    iy = int(np.clip(round(depth / h - 0.5), 0, ny - 1))
    xs = (np.arange(nrec) + 0.5) / nrec * nx * h
    ix = np.clip(np.round(xs / h - 0.5).astype(int), 0, nx - 1)
    return np.full(nrec, iy, dtype=np.int64), ix.astype(np.int64)


def smooth_directions(nx: int, ny: int, count: int, seed: int = 100,
                      cells: float = 16.0) -> np.ndarray:
    """``count`` smooth unit-norm perturbation fields (count, ny, nx), seeds seed..seed+count-1."""
    out = []
    for k in range(count):
        g = gaussian_filter(np.random.default_rng(seed + k).standard_normal((ny, nx)),
                            cells, mode="reflect")
        out.append(g / np.linalg.norm(g))
    return np.stack(out)


def sources_for(w: Workload, nrhs: Optional[int] = None) -> np.ndarray:
    """The workload's source batch on physical cells, shape (nrhs, *reversed(n))."""
    k = w.nrhs if nrhs is None else nrhs
    if w.name == "c1" or (w.medium == "constant" and w.dim == 2):
        src = gaussian_source(w.n, w.h, tuple(0.5 * m * w.h for m in w.n), 2 * w.h)
        return np.repeat(src[None], k, axis=0)
    if w.dim == 2:
        return surface_gaussian_sources(w.n[0], w.n[1], w.h, k)
    return random_gaussian_sources_3d(w.n[0], w.h, k)
