"""The solve-phase kernels keep their working data in registers (CPU, from the device assembly
hipcc writes for gfx950 with the library's own flags): no kernel of the PCG / V-cycle / panel /
fused paths uses scratch memory or spills registers.  A kernel whose per-lane arrays fall out of
registers (an out-of-line helper, a loop the compiler does not unroll) streams them through
memory on every launch; the dense tail product did once, at 1.6x its time."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2011_13325_amd import build as B

SOLVE_SOURCES = ["kernels.hip", "coarse.hip", "panel.hip", "fused.hip"]
# setup kernels that keep small dense matrices per thread (pseudo-inverses, P_s rows, criteria)
SETUP_KERNELS = re.compile(r"k_diag_pinv|k_ps_numeric|k_mu_b|k_mu_g|k_coarse_[ME]|k_gj_|k_dense_assemble")


def _kernels(src):
    try:
        hipcc = B._hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.s")
        cmd = [hipcc, *[f for f in B.HIP_FLAGS if f != "-fPIC"], *B.FILE_FLAGS.get(src, []),
               "--cuda-device-only", "-S", "-o", out, os.path.join(B.CSRC, src)]
        subprocess.run(cmd, check=True, capture_output=True, timeout=600)
        text = open(out).read()
    meta = text[text.index("amdhsa.kernels:"):]
    ks = []
    for block in re.split(r"\n  - ", meta)[1:]:
        name = re.search(r"\.name:\s+(\S+)", block)
        priv = re.search(r"\.private_segment_fixed_size:\s+(\d+)", block)
        spill = re.search(r"\.vgpr_spill_count:\s+(\d+)", block)
        if name and priv:
            ks.append((name.group(1), int(priv.group(1)), int(spill.group(1)) if spill else 0))
    return ks


@pytest.mark.parametrize("src", SOLVE_SOURCES)
def test_solve_kernels_use_no_scratch(src):
    ks = [k for k in _kernels(src) if not SETUP_KERNELS.search(k[0])]
    assert ks, src
    bad = [k for k in ks if k[1] or k[2]]
    assert not bad, bad
