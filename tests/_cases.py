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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sub_tuple(sid, parts):
    """GPU subdomain index (x part fastest) -> oracle tuple."""
    out = []
    for P in parts:
        out.append(sid % P)
        sid //= P
    return tuple(out)


__all__ = ["medium", "sources", "rel", "sub_tuple", "slowness2", "embed_physical"]
