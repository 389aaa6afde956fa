"""Pins for the oracle's FWI misfit gradient (oracle.fwi).

The adjoint gradient is derived, not printed, so it is pinned against what the
calculus fixes: central finite differences of the misfit itself along smooth
directions, and the second-order Taylor remainder.
"""
import numpy as np
import pytest

from oracle.fwi import FWIOracle
from oracle.pml import slowness2
import synth


def _setup(N=40, pml=8):
    n, h, om = (N, N), 1.0 / N, 2 * np.pi * 3
    c_true = synth.layered_medium(N, N, seed=0)
    c0 = synth.smooth_medium(c_true, 4.0)
    src = synth.surface_gaussian_sources(N, N, h, 4)
    rec = synth.surface_receivers(N, N, h, 12)
    fw = FWIOracle(n, h, om, pml, src, rec)
    d_obs = fw.observed(slowness2(c_true))
    return fw, slowness2(c0), d_obs


def test_gradient_matches_central_differences():
    fw, m0, d = _setup()
    J0, g = fw.gradient(m0, d)
    dirs = synth.smooth_directions(40, 40, 3, seed=100, cells=4.0)
    for p in dirs:
        eps = 1e-4 * np.linalg.norm(m0) / np.linalg.norm(p)
        fd = (fw.misfit(m0 + eps * p, d) - fw.misfit(m0 - eps * p, d)) / (2 * eps)
        ad = float(np.sum(g * p))
        assert abs(fd - ad) / abs(ad) < 1e-6, (fd, ad)


def test_taylor_remainder_is_second_order():
    fw, m0, d = _setup(32, 6)
    J0, g = fw.gradient(m0, d)
    p = synth.smooth_directions(32, 32, 1, seed=104, cells=3.0)[0]
    base = 1e-2 * np.linalg.norm(m0) / np.linalg.norm(p)
    rem = []
    for k in range(4):
        eps = base / 2 ** k
        rem.append(abs(fw.misfit(m0 + eps * p, d) - J0 - eps * np.sum(g * p)))
    rates = np.log2(np.array(rem[:-1]) / np.array(rem[1:]))
    assert np.all(rates > 1.8), rates
