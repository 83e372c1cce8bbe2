"""The host-side numerics of the library and the FP64 oracle under
AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

tests/sanitize/host_numerics.cpp drives the library's host code (quadrature
and velocity tables, the zeta table, per-shell equilibrium coefficients, the
Landau and quantum-statistics frames) over every supported order, shell and
angle count; tests/sanitize/oracle_driver.c drives the oracle (quadratures,
equilibria, frames, short runs with every boundary condition and statistics).
Both are built with g++ / gcc, -fsanitize=address,undefined and
-fno-sanitize-recover=all, so any out-of-bounds access, use after free,
leak or undefined operation fails the run.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1"]


def _run(exe, env_extra=None):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", OMP_NUM_THREADS="2")
    env.update(env_extra or {})
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert r.stdout.startswith("ok"), out[-4000:]
    return r.stdout.strip()


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_library_host_numerics_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_numerics")
    subprocess.check_call(["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + SAN +
                          [os.path.join(ROOT, "tests", "sanitize", "host_numerics.cpp"),
                           os.path.join(ROOT, "paper_2011_06856_amd", "csrc", "quadrature.cpp"), "-o", exe],
                          stderr=subprocess.DEVNULL)
    print(_run(exe))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    subprocess.check_call(["gcc", "-std=c11", "-fopenmp"] + SAN +
                          [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "rlbm_oracle.c"), "-lm", "-o", exe])
    print(_run(exe))
