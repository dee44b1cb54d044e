"""The coarse-system assembly (host code, csrc/coarse_csr.h) against its
definition, the sum over elements of P_e^T A_e P_e on the free nodes formed
densely element by element (CPU only; built with AddressSanitizer and
UndefinedBehaviorSanitizer).  Cases: Dirichlet and Neumann boxes of trilinear
elements, permuted node ids, a collapsed element (two local points on one
node), no free nodes at all, and a nonpositive diagonal reported at its row.
The CSR must hold exactly the touched (row, column) pairs, columns ascending,
with values bit-identical to the element-by-element sums."""
import os
import shutil
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2104_05829_amd", "csrc")
DRIVER = os.path.join(ROOT, "tests", "sanitize", "coarse_csr_driver.cpp")


def test_coarse_assembly_matches_dense_definition(tmp_path):
    import pytest
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(DRIVER):
        pytest.skip("g++ or the driver source not available")
    exe = str(tmp_path / "coarse_csr_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, DRIVER, "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr[-4000:]
    assert res.stdout.count("ok case") == 6, res.stdout
