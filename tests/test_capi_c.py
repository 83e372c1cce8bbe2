"""The C ABI from plain C: tests/capi_c/step_from_c.c includes include/rlbm.h,
links librlbm.so and drives a whole run (quadrature, fields, steps, moments)
with no Python or torch in its process.

- CPU: the header and the program compile as strict C99 with warnings as
  errors, and the program links against the built library when it is there.
- GPU: the program's fields and charges after the steps equal the FP64 oracle's
  on the same seeded inputs: 1e-12 in FP64 (tile and push kernels), 1e-4 in
  FP32, relative L-inf per field and the flow as a vector (tests/fieldcheck.py).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O
import workloads as W
from fieldcheck import check_fields, say

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "capi_c", "step_from_c.c")
INC = os.path.join(ROOT, "include")
PKG = os.path.join(ROOT, "paper_2011_06856_amd")
LIB = os.path.join(PKG, "librlbm.so")
CFLAGS = ["-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-O1", "-I", INC]


def _cc():
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    return cc


def _build(tmp_path):
    exe = str(tmp_path / "step_from_c")
    subprocess.run([_cc()] + CFLAGS + [SRC, "-o", exe, "-L", PKG, "-lrlbm", "-Wl,-rpath," + PKG],
                   check=True, capture_output=True, text=True)
    return exe


def test_header_and_program_compile_as_c99(tmp_path):
    obj = str(tmp_path / "step_from_c.o")
    r = subprocess.run([_cc()] + CFLAGS + ["-c", SRC, "-o", obj], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    if os.path.exists(LIB):
        _build(tmp_path)


def _run_c(exe, tmp_path, Np, K, N, nx, ny, fld, tau, dt, steps, prec, bcx=0, bcy=0):
    n, T, ux, uy = fld
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    with open(inp, "wb") as f:
        f.write(np.array([Np, K, N, nx, ny, steps, prec, bcx, bcy], dtype=np.int32).tobytes())
        f.write(np.array([tau, dt], dtype=np.float64).tobytes())
        for a in (n, T, ux, uy):
            f.write(np.ascontiguousarray(a, dtype=np.float64).reshape(ny, nx).tobytes())
    r = subprocess.run([exe, inp, out], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    raw = open(out, "rb").read()
    status = int(np.frombuffer(raw[:4], dtype=np.int32)[0])
    vals = np.frombuffer(raw[4:], dtype=np.float64)
    S = nx * ny
    assert vals.size == 4 * S + 4
    fields = tuple(vals[k * S:(k + 1) * S].reshape(ny, nx) for k in range(4))
    return status, fields, vals[4 * S:]


CASES = [
    # name, Np, K, N, nx, ny, kind, tau, dt, steps, precision, tol
    ("tile_fp64", 3, 16, 2, 70, 9, "quadrant", 2.0, 0.7, 40, 0, 1e-12),
    ("push_fp64", 4, 96, 3, 70, 9, "disc", 2.0, 0.7, 20, 0, 1e-12),
    ("tile_fp32", 3, 16, 2, 70, 9, "quadrant", 2.0, 0.7, 40, 1, 1e-4),
]


@pytest.mark.gpu
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_c_program_matches_the_oracle(case, tmp_path):
    name, Np, K, N, nx, ny, kind, tau, dt, steps, prec, tol = case
    if not os.path.exists(LIB):
        raise FileNotFoundError("librlbm.so is not built: " + LIB)
    exe = _build(tmp_path)
    if kind == "quadrant":
        fld = W.quadrant(nx, ny, seed=nx + ny)
    else:
        fld = W.disc(nx, ny, min(nx, ny) / 4, seed=nx)
    say("case C caller %s %dx%d Np=%d K=%d N=%d steps=%d" % (name, nx, ny, Np, K, N, steps))
    status, got, ch = _run_c(exe, tmp_path, Np, K, N, nx, ny, fld, tau, dt, steps, prec)
    assert status == 0, status
    q = O.Quadrature(Np, K, N)
    sim = O.Sim(q, nx, ny, *fld, tau=tau, dt=dt)
    sim.step(steps)
    check_fields(got, sim.fields(), tol, "c_caller_" + name)
    np.testing.assert_allclose(ch, sim.charges(), rtol=max(tol, 1e-12), atol=1e-12)
