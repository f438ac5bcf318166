"""Host logic of bench.py, on the CPU: the one-GPU rule, the Lanczos condition-number estimate
from CG coefficients, and the machine-read lines of the committed counter summary."""
import hashlib
import json
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


class _Coefficients:
    """Stands in for the binding: eamg_solve_coefficients returns given CG coefficients."""

    def __init__(self, alpha, beta):
        self.a, self.b = alpha, beta

    def eamg_solve_coefficients(self, h):
        return self.a, self.b


class _Hierarchy:
    h = None


def _cg_coefficients(lam, iters, seed=0):
    """alpha_k, beta_k of plain CG on diag(lam) (beta_1 = 0, as the library reports them)."""
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(lam.size)
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rho = r @ r
    alpha, beta = [], [0.0]
    for k in range(iters):
        q = lam * p
        a = rho / (p @ q)
        alpha.append(a)
        x += a * p
        r -= a * q
        rho_new = r @ r
        if k + 1 < iters:
            beta.append(rho_new / rho)
        p = r + (rho_new / rho) * p
        rho = rho_new
    return alpha, beta


def test_lanczos_condition_number_from_cg_coefficients():
    # the tridiagonal matrix built from CG's alpha, beta is the Lanczos matrix of the operator:
    # its extreme eigenvalues converge to the operator's, so kappa = 100 / 1 is recovered
    lam = np.linspace(1.0, 100.0, 200)
    a, b = _cg_coefficients(lam, 60)
    k = bench._kappa(_Coefficients(a, b), _Hierarchy())
    assert k["kappa"] == pytest.approx(100.0, rel=1e-3)
    assert k["lambda_min"] == pytest.approx(1.0, rel=1e-3)
    assert k["lambda_max"] == pytest.approx(100.0, rel=1e-3)
    s = np.sqrt(k["kappa"])
    assert k["cg_factor"] == pytest.approx((s - 1) / (s + 1), abs=1e-4)
    # a short run sees an inner part of the spectrum only: the estimate is a lower bound
    a, b = _cg_coefficients(lam, 4)
    assert bench._kappa(_Coefficients(a, b), _Hierarchy())["kappa"] < 100.0


def test_traffic_line_follows_the_measured_source():
    path = os.path.join(ROOT, "profiles", "traffic_k_gs_color_cube128.md")
    txt = open(path).read()
    kernel = re.search(r"^traffic_kernel: (.+)$", txt, re.M).group(1).strip()
    value = float(re.search(r"^traffic_bytes_per_launch: (\d+)$", txt, re.M).group(1))
    sha = re.search(r"^kernels_hip_sha256: ([0-9a-f]+)$", txt, re.M).group(1)
    src = open(os.path.join(ROOT, "paper_2011_13325_amd", "csrc", "kernels.hip"), "rb").read()
    current = hashlib.sha256(src).hexdigest() == sha
    assert bench._traffic(kernel) == (value if current else None)
    assert bench._traffic("k_not_measured<float>") is None
