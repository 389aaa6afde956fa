"""Host-side checks of the C-ABI library (no GPU calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "dsweep.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    return sorted(set(re.findall(r"\b(dsd_[a-z_0-9]+)\s*\(", hdr)))


def test_library_loads_and_exports_every_declared_symbol():
    from paper_2002_05327_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    # the binding declares exactly the header's entry points
    assert set(_lib.EXPORTS) == set(names)


def test_strerror_without_gpu():
    from paper_2002_05327_amd import _lib
    lib = _lib.load()
    assert lib.dsd_strerror(-4).decode().startswith("singular")
    assert lib.dsd_strerror(1).decode().startswith("tolerance")


def test_oracle_is_not_imported_by_the_product():
    pkg = os.path.join(ROOT, "paper_2002_05327_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", txt, re.M), fn
                assert "oracle/" not in txt, fn


def _params(**kw):
    from paper_2002_05327_amd import _lib
    p = _lib.Params()
    p.dim, p.h, p.pml, p.overlap, p.sigma0_delta = 2, 1 / 64, 8, 4, 60.0
    p.n[0], p.n[1], p.n[2] = 64, 64, 1
    p.parts[0], p.parts[1], p.parts[2] = 2, 2, 1
    p.precision, p.max_rhs = 2, 1
    for k, v in kw.items():
        if k in ("n", "parts"):
            for a, x in enumerate(v):
                getattr(p, k)[a] = x
        else:
            setattr(p, k, v)
    return p


@pytest.mark.parametrize("bad", [dict(dim=4), dict(overlap=2), dict(pml=-1), dict(h=0.0),
                                 dict(precision=7), dict(local_solver=5), dict(schedule=3),
                                 dict(dense_top=-2), dict(sweep_order=1),
                                 dict(parts=(65, 2, 1)), dict(n=(0, 64, 1)), "omega"])
def test_plan_create_rejects_bad_parameters_without_gpu(bad):
    """Parameter validation answers DSD_EINVAL with a message before any device
    work (so it runs without a GPU); the medium pointer is never read."""
    from paper_2002_05327_amd import _lib
    lib = _lib.load()
    p = _params() if bad == "omega" else _params(**bad)
    omega = 0.0 if bad == "omega" else 2 * 3.141592653589793 * 4
    h = ctypes.c_void_p()
    rc = lib.dsd_plan_create(ctypes.byref(p), omega, ctypes.c_void_p(16), None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert lib.dsd_last_error_detail().decode()


def test_entry_points_reject_a_null_plan_without_gpu():
    from paper_2002_05327_amd import _lib
    lib = _lib.load()
    one = ctypes.c_void_p(16)
    assert lib.dsd_sweep_apply(None, one, one, 1, None) == -1
    assert lib.dsd_apply_operator(None, one, one, 1, None) == -1
    assert lib.dsd_ddm_iterate(None, one, one, 1, 1, (ctypes.c_double * 2)(), None) == -1
    assert lib.dsd_timing_flops(None, (ctypes.c_double * 1)()) == -1


def test_bench_band_work_matches_the_stated_c2_figures():
    """bench.py's algorithmic bytes (band LU factor once per RHS block plus the
    vectors, over the 2^dim * N_sub local solves of one application) reproduce
    the C2 figures the measurement is defined by: 26.0 GB of complex64 factor
    stream per RHS block and 0.28 GB of vectors per RHS; 2.59e10 flops per RHS.
    Local grids come from the oracle's partition."""
    import bench
    import synth
    from oracle.partition import Partition
    w = synth.workload("c2")
    part = Partition(w.n, w.parts, w.pml, w.overlap, w.h)

    class FakePlan:
        def subdomain_grid(self, sid):
            sub = (sid % w.parts[0], sid // w.parts[0])
            return tuple(ax.n for ax in part.local_axes(sub)), (0, 0)

    b1, f1 = bench.band_work(FakePlan(), w, 1, 8)
    b2, f2 = bench.band_work(FakePlan(), w, 2, 8)
    vec = b2 - b1
    fac = b1 - vec
    assert abs(fac / 26.0e9 - 1) < 0.01 and abs(vec / 0.28e9 - 1) < 0.03
    assert abs(f1 / 2.59e10 - 1) < 0.01 and f2 == 2 * f1


def test_noalloc_scratch_size_matches_the_header():
    from paper_2002_05327_amd import _lib
    hdr = open(os.path.join(ROOT, "include", "dsweep.h")).read()
    m = re.search(r"#define DSD_NOALLOC_SCRATCH_BYTES \((\d+)LL << (\d+)\)", hdr)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.NOALLOC_SCRATCH_BYTES
