"""Plain FP64 CPU oracle for the diagonal-sweeping source-transfer DDM.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the
HIP library (no kernels, headers, tables, constants or pre/post-processing);
the only common inputs are the seeded arrays produced by ``synth``.

Everything here is complex128 numpy/scipy, written to be checked against the
paper by eye:

  * :mod:`oracle.pml`       -- grid, complex stretching, J-scaled 5/7-point operator
                                (Section 2.1, eq. (eq:sigma), (eq:PML), (eq:PMLprofile))
  * :mod:`oracle.partition` -- checkerboard partition, extended subdomains,
                                index-form cutoffs and truncations (Section 2.2)
  * :mod:`oracle.sweep`     -- sweep orders, Rules 3.1/3.2/4.1/4.2, Algorithms 3.1/4.1,
                                and the additive DDM it re-orders (Algorithms 2.1/2.2)
  * :mod:`oracle.krylov`    -- flexible GMRES with the DDM as right preconditioner
                                (Remark 1 of Section 4, Section 5.2)
  * :mod:`oracle.analytic`  -- free-space solutions of the Gaussian sources of the
                                constant-medium accuracy tests (Section 5.1,
                                Tables 1 and 2) and the L2 error against them
  * :mod:`oracle.fwi`       -- misfit and adjoint gradient w.r.t. 1/c^2
                                (Remark 2 of Section 4 motivates it; no formula in
                                the paper, so the adjoint is derived from the
                                discrete system)

Readings of points the paper leaves open are listed in each module header and
collected in the design notes of the repository.
"""
