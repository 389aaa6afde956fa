"""Write table2_oracle.json: the oracle's L2 errors for Table 2's rows (Section 5.1).

Calls only ``oracle/``: the discrete global solution of Table 2's constant-medium
problem (kappa/2pi = 10, physical box [-3/8, 3/8]^3 inside the unit cube, PML
to the cube's faces) with the source as printed -- unit mass,
64 kappa^3 / pi^(9/2) exp(-(4 kappa/pi)^2 |x - x0|^2) -- by the separable solver,
its residual under the sparse operator, and its L2 error against the
free-space solution over the physical cells.

Usage: python tests/golden/make_table2_oracle.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.analytic import gaussian_source, l2_error   # noqa: E402
from oracle.pml import assemble, global_axes            # noqa: E402
from oracle.separable import residual, solve_constant   # noqa: E402


def table2_problem(tab, mesh):
    """Grid, PML and source of one row (the same construction the GPU test uses)."""
    dim = len(tab["source_centre"])
    kappa = 2 * np.pi * tab["kappa_over_2pi"]
    h = 1.0 / mesh
    n = int(round(2 * tab["l"] / h))
    pml = (mesh - n) // 2
    x0 = [c + tab["l"] for c in tab["source_centre"]]
    c = (np.arange(n) + 0.5) * h
    coords = np.meshgrid(*([c] * dim), indexing="ij")
    r = np.sqrt(sum((g - x0[dim - 1 - k]) ** 2 for k, g in enumerate(coords)))
    f = np.pad(gaussian_source(kappa, dim, r), pml).astype(np.complex128)
    return dim, kappa, h, n, pml, x0, f


def main():
    tab = json.load(open(os.path.join(HERE, "accuracy_tables.json")))["table2_3d"]
    out = {"citation": "Section 5.1, Table 2 (3D constant medium, kappa/2pi = 10): the oracle's "
                       "discrete solution (separable direct solve) with the unit-mass source as "
                       "printed; L2 error over the physical cells against the free-space solution",
           "rows": {}}
    for mesh in (80, 96, 128, 160):
        dim, kappa, h, n, pml, x0, f = table2_problem(tab, mesh)
        u = solve_constant((n,) * dim, h, kappa, pml, 1.0, f.ravel())
        M = assemble(global_axes((n,) * dim, pml, h), np.ones((n,) * dim), h, kappa, pml)
        res = residual(M, u, f.ravel())
        sl = (slice(pml, pml + n),) * dim
        e = l2_error(u.reshape(f.shape)[sl], h, x0, kappa)
        printed = [r[2] for r in tab["rows"] if r[0] == mesh][0]
        print(f"{mesh}^3: n={n} pml={pml} residual {res:.1e} L2 error {e:.6e} "
              f"(printed {printed}, ratio {e / printed:.4f})", flush=True)
        out["rows"][str(mesh)] = {"l2_error": e, "residual": res, "printed": printed}
    with open(os.path.join(HERE, "table2_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=2)


if __name__ == "__main__":
    main()
