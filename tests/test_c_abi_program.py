"""The C ABI from a plain C program (tests/c_abi/potential_demo.c): the header compiles as C99
with gcc and the program links against libnlf.so (CPU); on the GPU the program's potential
matches the FP64 oracle element by element and the closed form of Example 2.2 at the origin."""
import os
import subprocess

import numpy as np
import pytest

from oracle import potential as op

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_abi", "potential_demo.c")
PKG = os.path.join(ROOT, "paper_1410_3584_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _compile(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libnlf.so")):
        pytest.fail("libnlf.so is not built (run `python -m paper_1410_3584_amd.build`)")
    exe = str(tmp_path / "potential_demo")
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROCM, "include"), "-I", os.path.join(ROOT, "include"), SRC, "-o", exe,
           "-L", PKG, "-lnlf", "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath," + PKG, "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    subprocess.run(cmd, check=True)
    return exe


def test_c_program_compiles_and_links(tmp_path):
    assert os.path.exists(_compile(tmp_path))


@pytest.mark.gpu
def test_c_program_potential_matches_oracle(tmp_path):
    print("[c abi program] 2D Coulomb 64^2 on [-8,8)^2, FP64", flush=True)
    exe = _compile(tmp_path)
    out = tmp_path / "u.bin"
    res = subprocess.run([exe, str(out)], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    u = np.fromfile(out, dtype=np.float64).reshape(64, 64)
    n, L = (64, 64), (8.0, 8.0)
    xs, _ = op.grid_axes(n, L)
    X, Y = np.meshgrid(xs[0], xs[1], indexing="ij")
    want = op.potential(np.exp(-(X * X + Y * Y)), n, L, op.COULOMB2D)
    assert np.max(np.abs(u - want)) <= 1e-10 * np.max(np.abs(want))
    # Example 2.2 with sigma = 1: u(0) = int_0^inf e^{-r^2} dr = sqrt(pi)/2
    assert abs(u[32, 32] - 0.5 * np.sqrt(np.pi)) <= 1e-10
    assert "u(0)" in res.stdout
