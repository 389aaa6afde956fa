"""Free-space solutions for the normalised Gaussian sources of the paper's
constant-medium accuracy tests (Section 5.1, Tables 1 and 2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The source centred at x0 is  f = (a/pi)^(dim/2) exp(-a |x - x0|^2)  with
a = (4 kappa / pi)^2, which integrates to one; the paper writes it as
16 kappa^2/pi^3 exp(...) in 2D and 64 kappa^3/pi^(9/2) exp(...) in 3D.
The discrete operator everywhere else solves  Delta u + kappa^2 u = f  (the
J-scaled PML equation with J = 1 on physical cells), so the free-space
solution is  u = -(G * f)  with the outgoing fundamental solution G of
Delta + kappa^2 (Delta G + kappa^2 G = -delta, time dependence exp(-i omega t)):

    2D:  G(r) = (i/4) H0^(1)(kappa r)        3D:  G(r) = exp(i kappa r) / (4 pi r).

For a radially symmetric source the convolution is one-dimensional.  The
angular mean of G(|x - y|) over the circle (sphere) |y - x0| = rho is, with
r< = min(r, rho) and r> = max(r, rho) (Graf's addition theorem in 2D, the
spherical-wave expansion in 3D):

    2D:  (i/4) J0(kappa r<) H0(kappa r>)
    3D:  sin(kappa r<) exp(i kappa r>) / (4 pi kappa r< r>)

so that, with A and B the inner and outer radial integrals,

    2D:  (G*f)(r) = (i pi / 2) [ H0(kappa r) int_0^r rho f J0(kappa rho) drho
                                + J0(kappa r) int_r^inf rho f H0(kappa rho) drho ]
    3D:  (G*f)(r) = 1/(kappa r) [ exp(i kappa r) int_0^r rho f sin(kappa rho) drho
                                 + sin(kappa r) int_r^inf rho f exp(i kappa rho) drho ].

Beyond the numerical support of f (f < 1e-20 f(0)) the outer integral
vanishes and the inner one is the Fourier transform of f at kappa,
exp(-kappa^2 / (4a)), which gives the closed forms

    2D:  u = -(i/4) H0(kappa r) exp(-kappa^2/(4a))
    3D:  u = -exp(i kappa r) / (4 pi r) exp(-kappa^2/(4a)).

Inside, both radial integrals are cumulative trapezoid sums on a fine radial
grid (second order in its spacing) and the solution is interpolated linearly
between its nodes.
"""
from __future__ import annotations

import numpy as np
from scipy import special


def gaussian_width(kappa: float) -> float:
    """a = (4 kappa / pi)^2 of the paper's sources."""
    return (4.0 * kappa / np.pi) ** 2


def gaussian_source(kappa: float, dim: int, r: np.ndarray) -> np.ndarray:
    a = gaussian_width(kappa)
    return (a / np.pi) ** (dim / 2) * np.exp(-a * np.asarray(r, dtype=float) ** 2)


def support_radius(kappa: float) -> float:
    """Radius beyond which f < 1e-20 f(0) (exp(-46) = 1.1e-20)."""
    return float(np.sqrt(46.0 / gaussian_width(kappa)))


def _far(kappa: float, dim: int, r: np.ndarray) -> np.ndarray:
    damp = np.exp(-kappa ** 2 / (4.0 * gaussian_width(kappa)))
    if dim == 2:
        return -0.25j * special.hankel1(0, kappa * r) * damp
    return -np.exp(1j * kappa * r) / (4.0 * np.pi * r) * damp


def _cumtrapz(y: np.ndarray, dx: float) -> np.ndarray:
    out = np.zeros_like(y)
    out[1:] = np.cumsum(0.5 * (y[1:] + y[:-1])) * dx
    return out


def _near_table(kappa: float, dim: int, nodes: int):
    R = support_radius(kappa)
    rho = np.linspace(0.0, R, nodes)
    d = rho[1] - rho[0]
    f = gaussian_source(kappa, dim, rho)
    kr = kappa * rho
    if dim == 2:
        j0 = special.j0(kr)
        y0 = np.zeros_like(rho)
        y0[1:] = special.y0(kr[1:])
        h0 = j0 + 1j * y0
        inner = _cumtrapz(rho * f * j0, d)
        g_out = rho * f * h0                   # rho Y0(kappa rho) -> 0 at rho = 0
        outer = _cumtrapz(g_out[::-1], d)[::-1]
        gf = np.empty(nodes, dtype=complex)
        gf[1:] = 0.5j * np.pi * (h0[1:] * inner[1:] + j0[1:] * outer[1:])
        gf[0] = 0.5j * np.pi * outer[0]        # H0 A -> 0 as rho -> 0
    else:
        inner = _cumtrapz(rho * f * np.sin(kr), d)
        outer = _cumtrapz((rho * f * np.exp(1j * kr))[::-1], d)[::-1]
        gf = np.empty(nodes, dtype=complex)
        gf[1:] = (np.exp(1j * kr[1:]) * inner[1:] + np.sin(kr[1:]) * outer[1:]) / kr[1:]
        gf[0] = outer[0]                       # sin(kr)/(kr) -> 1, A/(kr) -> 0
    return rho, -gf


def free_space(kappa: float, dim: int, r: np.ndarray, nodes: int = 400001) -> np.ndarray:
    """u(r) = -(G * f)(r) for the paper's Gaussian source, at distances r >= 0."""
    r = np.asarray(r, dtype=float)
    out = np.empty(r.shape, dtype=complex)
    R = support_radius(kappa)
    far = r >= R
    out[far] = _far(kappa, dim, r[far])
    if np.any(~far):
        rho, u = _near_table(kappa, dim, nodes)
        out[~far] = np.interp(r[~far], rho, u.real) + 1j * np.interp(r[~far], rho, u.imag)
    return out


def l2_error(u_phys: np.ndarray, h: float, x0, kappa: float) -> float:
    """Absolute L2 norm over the physical cells, sqrt(sum |u_h - u|^2 h^dim), of
    the difference between a cell-centred grid function (array axes reversed:
    (y, x) or (z, y, x)) and the free-space solution; cell i of an axis has its
    centre at (i + 1/2) h."""
    dim = u_phys.ndim
    centres = [(np.arange(s) + 0.5) * h for s in u_phys.shape]      # slowest axis first
    coords = np.meshgrid(*centres, indexing="ij")
    r = np.sqrt(sum((c - x0[dim - 1 - k]) ** 2 for k, c in enumerate(coords)))
    e = u_phys - free_space(kappa, dim, r)
    return float(np.sqrt(np.sum(np.abs(e) ** 2) * h ** dim))
