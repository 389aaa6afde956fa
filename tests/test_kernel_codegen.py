"""Code-generation checks of the nested-dissection solve kernels (CPU: hipcc
cross-compiles gfx950 device assembly here).

The solve kernels are latency-bound launches whose speed depends on two
properties of the generated code that no numerical test sees:

* no private (scratch) memory: a conditional between two complex lvalues
  selects an address and keeps whole arrays in scratch (the complex128
  forward and dense-top kernels once spilled 160 bytes per lane that way);
* no flat loads: a load through a pointer selected between a global array and
  LDS or a private value compiles to a flat load, whose wait also covers every
  global load in flight.

The device assembly of nd.hip is built with the library's own flags and every
instance of the level and dense-top kernels for 8 right-hand sides per
workgroup (the default group) is checked for both properties.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def nd_asm(tmp_path_factory):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    from paper_2002_05327_amd.build import CSRC, HIPCC_FLAGS
    flags = [f for f in HIPCC_FLAGS if f != "-fPIC"]
    out = str(tmp_path_factory.mktemp("asm") / "nd.s")
    subprocess.run([HIPCC, *flags, "--cuda-device-only", "-S", os.path.join(CSRC, "nd.hip"),
                    "-o", out], check=True, capture_output=True)
    return open(out).read()


def _kernels(asm, pattern):
    """(name, body, private segment size) of every kernel whose mangled name
    matches pattern."""
    starts = [(m.start(), m.group(1)) for m in re.finditer(r"\n(_ZN3dsd[A-Za-z0-9_]+):", asm)]
    out = []
    for k, (pos, name) in enumerate(starts):
        if not re.search(pattern, name):
            continue
        end = starts[k + 1][0] if k + 1 < len(starts) else len(asm)
        body = asm[pos:end]
        m = re.search(r"\.amdhsa_kernel " + re.escape(name) + r"\s.*?\.amdhsa_private_segment_fixed_size (\d+)",
                      asm, re.S)
        out.append((name, body, int(m.group(1)) if m else None))
    return out


@pytest.mark.parametrize("kernel", ["k_nd_lvl_fwd", "k_nd_lvl_bwd", "k_nd_top"])
@pytest.mark.parametrize("prec", ["f", "d"])
def test_solve_kernels_use_no_scratch_and_no_flat_loads(nd_asm, kernel, prec):
    found = _kernels(nd_asm, rf"^_ZN3dsd\d+{kernel}I{prec}Li8E")
    assert found, f"{kernel}<{prec}, 8> not in the device assembly"
    for name, body, scratch in found:
        print(name[:60], "private segment", scratch, "flat loads", body.count("flat_load"))
        assert scratch == 0, f"{name}: {scratch} bytes of scratch per lane"
        assert "flat_load" not in body, f"{name}: flat loads"
