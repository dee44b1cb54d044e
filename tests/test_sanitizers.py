"""Host code under sanitizers (CPU only).

* The oracle's C loops (oracle/sem_oracle.c), built with AddressSanitizer and
  UndefinedBehaviorSanitizer, driven through every entry point on small
  deformed boxes (tests/sanitize/oracle_driver.c).
* The library's host-side Schwarz construction (csrc/schwarz.hip, threaded
  over element ranges and a parallel sort) and GLL construction (csrc/gll.cpp),
  built from the library's sources with ThreadSanitizer and, separately, with
  AddressSanitizer + UndefinedBehaviorSanitizer on the host pass only
  (tests/sanitize/setup_driver.cpp).  The driver also checks that the
  construction with 1 and with 16 host threads is bit-identical.

No device code runs.  The builds need gcc, hipcc and ROCm's clang++."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2104_05829_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANGXX = "/opt/rocm/lib/llvm/bin/clang++"
HIP_FLAGS = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, env=None, timeout=900):
    res = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    assert res.returncode == 0, f"{' '.join(cmd)}\nrc={res.returncode}\n{res.stdout}\n{res.stderr[-4000:]}"
    return res


def test_oracle_under_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_asan")
    _run(["gcc", "-std=gnu11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-fast-math", "-ffp-contract=off", os.path.join(ROOT, "oracle", "sem_oracle.c"),
          os.path.join(SAN, "oracle_driver.c"), "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
    out = _run([exe], env=env).stdout
    assert out.count("oracle N=") == 4, out


def _build_setup_driver(tmp_path, kind):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)):
        pytest.skip("hipcc / ROCm clang++ not found")
    san = "thread" if kind == "tsan" else "address,undefined"
    host = ["-Xarch_host", f"-fsanitize={san}"]
    if kind != "tsan":
        host += ["-Xarch_host", "-fno-sanitize-recover=all"]
    objs = []
    for src in ("schwarz.hip", "gll.cpp"):
        o = str(tmp_path / f"{src}.{kind}.o")
        _run([HIPCC] + HIP_FLAGS + host + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    drv = str(tmp_path / f"driver.{kind}.o")
    _run([CLANGXX, "-O1", "-g", "-std=c++17", f"-fsanitize={san}", "-c",
          os.path.join(SAN, "setup_driver.cpp"), "-o", drv])
    exe = str(tmp_path / f"setup_{kind}")
    _run([CLANGXX, f"-fsanitize={san}", drv] + objs +
         ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    return exe


def test_schwarz_setup_under_tsan(tmp_path):
    exe = _build_setup_driver(tmp_path, "tsan")
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:exitcode=66")
    # 12 x 12 x 8 elements: 16 threads over element ranges and the sort
    for args in (["3", "12", "12", "8"], ["7", "8", "8", "8"]):
        out = _run([exe] + args, env=env)
        assert "bit-identical" in out.stdout and "ThreadSanitizer" not in out.stderr, out.stderr[-2000:]


def test_schwarz_setup_under_asan_ubsan(tmp_path):
    exe = _build_setup_driver(tmp_path, "asan")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    for args in (["2", "5", "4", "3"], ["3", "12", "12", "8"]):
        out = _run([exe] + args, env=env)
        assert "bit-identical" in out.stdout, out.stdout
