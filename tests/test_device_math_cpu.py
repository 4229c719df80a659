"""The solver's device math on the host (compiled with hipcc for the CPU):
the FP32 sin/cos of the circle map against libm, and the banded Cholesky
factorisation and solve against a dense numpy solve on block-banded
symmetric positive definite matrices of every order and block size."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2301_06399_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    hipcc = shutil.which("hipcc")
    if hipcc is None:
        pytest.skip("hipcc not found")
    exe = str(tmp_path_factory.mktemp("devmath") / "device_math_check")
    subprocess.run([hipcc, "-O2", "-std=c++17", "--offload-arch=gfx950", "-I", CSRC,
                    os.path.join(HERE, "device_math_check.hip"), "-o", exe], check=True, capture_output=True)
    return exe


def test_sincos32_accuracy(harness):
    """Within 2e-7 of sin and cos (about one FP32 ulp at 1) wherever the
    reduction's products are exact (|a| < 6400), and still close beyond."""
    for amax, bar in ((3.2, 1.2e-7), (100.0, 2e-7), (6000.0, 2e-7)):
        out = subprocess.run([harness, "sincos", str(amax), "400000"], check=True, capture_output=True, text=True)
        assert float(out.stdout) <= bar, (amax, out.stdout)


def _band_pattern(n, b):
    m = n * b
    mask = np.zeros((m, m), bool)
    for i in range(m):
        for j in range(m):
            mask[i, j] = abs(i // b - j // b) <= 2
    return mask


def test_band_cholesky_matches_dense_solve(harness):
    rng = np.random.default_rng(7)
    lines, cases = [], []
    for b in (2, 3):
        for n in range(1, 6):
            m = n * b
            mask = _band_pattern(n, b)
            for trial in range(6):
                # J^T J of a block-tridiagonal J plus a damping term: the
                # shape of the normal equations the solver factors
                J = rng.normal(size=(m, m)) * (np.abs(np.subtract.outer(np.arange(m) // b, np.arange(m) // b)) <= 1)
                A = J.T @ J + (10.0 ** rng.uniform(-6, 0)) * np.diag(rng.uniform(0.5, 2.0, m))
                assert not A[~mask].any()
                g = rng.normal(size=m)
                packed = [A[i, j] for i in range(m) for j in range(i + 1)]
                lines.append(f"{n} {b}\n" + " ".join(f"{v:.17g}" for v in packed) + "\n" +
                             " ".join(f"{v:.17g}" for v in -g))
                cases.append((A, g))
    # a matrix that is not positive definite is refused
    A = -np.eye(2)
    lines.append("1 2\n" + " ".join(f"{A[i, j]:.17g}" for i in range(2) for j in range(i + 1)) + "\n1 1")
    out = subprocess.run([harness, "band"], input="\n".join(lines) + "\n", check=True, capture_output=True,
                         text=True).stdout.split("\n")
    for (A, g), line in zip(cases, out):
        v = np.array([float(t) for t in line.split()])
        assert v[0] == 1
        x, dec = v[1:-1], v[-1]
        ref = np.linalg.solve(A, -g)
        assert np.linalg.norm(x - ref) <= 1e-9 * np.linalg.norm(ref) * max(1.0, np.linalg.cond(A) * 1e-6)
        assert abs(dec - (-g @ ref)) <= 1e-9 * abs(g @ ref) * max(1.0, np.linalg.cond(A) * 1e-6)
    assert out[len(cases)].split()[0] == "0"
