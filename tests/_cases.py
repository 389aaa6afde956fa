"""Shared seeded cases for the GPU parity tests (inputs only; both sides get the same arrays)."""
import numpy as np

import synth
from oracle.pml import embed_physical, slowness2


def medium(kind, n, seed=0):
    if kind == "const":
        return np.ones(tuple(reversed(n)))
    if kind == "layered":
        return synth.layered_medium(n[0], n[1], seed=seed)
    if kind == "grf3d":
        return synth.grf_medium_3d(n[0], seed=seed) if len(set(n)) == 1 else \
            2.0 + 0.2 * np.random.default_rng(seed).standard_normal(tuple(reversed(n)))
    if kind == "random":
        return 1.0 + 0.5 * np.random.default_rng(seed).random(tuple(reversed(n)))
    raise ValueError(kind)


def sources(n, h, pml, k, seed=1):
    """k seeded sources on physical cells (Gaussians + noise), embedded: (k, *gshape)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(k):
        centre = tuple(rng.uniform(0.2, 0.8) * m * h for m in n)
        f = synth.gaussian_source(n, h, centre, 2 * h) + 0.1 * rng.standard_normal(tuple(reversed(n)))
        out.append(embed_physical(f.astype(complex) * np.exp(1j * rng.uniform(0, 2 * np.pi)), pml))
    return np.stack(out)


def rel(a, b):
    """Relative 2-norm error over the whole array."""
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def elem(a, b):
    """Element-wise error max |a - b| / max |b|: a local error (a PML strip, a
    transfer box, a corner subdomain) that the 2-norm would average away."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def close(a, b, tol, what=""):
    """Assert both the relative 2-norm and the element-wise error below tol."""
    e2, ei = rel(a, b), elem(a, b)
    if what:
        print(f"{what}: rel {e2:.2e} elementwise {ei:.2e} (bound {tol:.0e})", flush=True)
    assert e2 < tol and ei < tol, (what, e2, ei, tol)
    return e2


def sub_tuple(sid, parts):
    """GPU subdomain index (x part fastest) -> oracle tuple."""
    out = []
    for P in parts:
        out.append(sid % P)
        sid //= P
    return tuple(out)


__all__ = ["medium", "sources", "rel", "elem", "close", "sub_tuple", "slowness2", "embed_physical"]
