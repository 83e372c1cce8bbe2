"""CPU tests of the C ABI: exported symbols, argument checks and the host-side
tables of the GPU library (no device call), compared with the oracle."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
R = pytest.importorskip("paper_2011_06856_amd.rlbm")


def _lib_or_skip():
    try:
        return R.lib()
    except ImportError as e:  # built by __graft_entry__.build()
        pytest.skip(str(e))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "rlbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rlbm_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    L = _lib_or_skip()
    names = declared_symbols()
    assert len(names) >= 17
    bound = {n for n, _, _ in R.SIGNATURES}
    for n in names:
        assert hasattr(L, n), n
        assert n in bound, n


def test_quadrature_matches_oracle():
    _lib_or_skip()
    for Np, K, N in [(3, 32, 3), (4, 64, 3), (6, 256, 5), (4, 24, 3), (5, 11, 4)]:
        s = R.Solver(Np, K, N)
        p, th, w = s.quadrature()
        q = O.Quadrature(Np, K, N)
        np.testing.assert_allclose(p, q.p, rtol=1e-14)
        np.testing.assert_allclose(th, q.theta, rtol=1e-15, atol=1e-15)
        np.testing.assert_allclose(w, q.w, rtol=1e-13)


@pytest.mark.parametrize("Np,K,N", [(3, 32, 3), (4, 64, 3), (6, 256, 5), (3, 5, 2), (5, 16, 4), (8, 20, 7), (4, 9, 1)])
def test_host_equilibrium_matches_oracle(Np, K, N):
    """Polar-Laguerre closed form (library) vs Cholesky-monomial tensor route (oracle)."""
    _lib_or_skip()
    s = R.Solver(Np, K, N)
    q = O.Quadrature(Np, K, N)
    rng = np.random.default_rng(Np * 100 + K)
    for trial in range(5):
        n, T = rng.uniform(0.1, 2.0), rng.uniform(0.5, 1.6)
        ux, uy = rng.uniform(-0.7, 0.7, size=2)
        a, b = s.host_feq(n, T, ux, uy), q.feq(n, T, ux, uy)
        np.testing.assert_allclose(a, b, rtol=0, atol=2e-13 * np.abs(b).max())


def test_host_landau_matches_oracle_bisection():
    _lib_or_skip()
    q = O.Quadrature(4, 32, 3)
    rng = np.random.default_rng(4)
    for trial in range(50):
        f = q.feq(rng.uniform(0.2, 1.5), rng.uniform(0.6, 1.4), *rng.uniform(-0.6, 0.6, 2))
        f = f * (1 + 0.3 * rng.uniform(-1, 1, size=q.nvel))
        m = q.moments(f)
        a, ok_a = R.host_landau(m)
        b, ok_b = O.landau(m)
        assert ok_a and ok_b
        np.testing.assert_allclose(a, b, rtol=2e-14, atol=2e-15)
    _, ok = R.host_landau(np.zeros(9))
    assert not ok


def test_invalid_arguments_are_rejected_without_a_device():
    _lib_or_skip()
    L = R.lib()
    h = ctypes.c_void_p()
    assert L.rlbm_init_quadrature(None, 4, 64, 3, 1) == R.RLBM_EINVAL
    assert L.rlbm_init_quadrature(ctypes.byref(h), 4, 6, 3, 1) == R.RLBM_EINVAL      # K < 2N+1
    assert L.rlbm_init_quadrature(ctypes.byref(h), 2, 64, 3, 1) == R.RLBM_EINVAL     # Np too small
    assert L.rlbm_init_quadrature(ctypes.byref(h), 4, 64, 0, 1) == R.RLBM_EINVAL
    assert L.rlbm_init_quadrature(ctypes.byref(h), 4, 64, 8, 1) == R.RLBM_EINVAL
    assert L.rlbm_init_quadrature(ctypes.byref(h), 4, 64, 3, 1) == R.RLBM_OK
    # batch calls on a null handle
    iv = ctypes.c_int()
    assert L.rlbm_batch_set_push_bands(None, 2) == R.RLBM_EINVAL
    assert L.rlbm_batch_get_push_bands(None, ctypes.byref(iv)) == R.RLBM_EINVAL
    assert L.rlbm_batch_set_mode(None, 0) == R.RLBM_EINVAL
    assert L.rlbm_batch_step(None, 1) == R.RLBM_EINVAL
    nx, ny = 4, 3
    n = np.ones(nx * ny)
    T = np.ones(nx * ny)
    bad_n = n.copy()
    bad_n[5] = -1.0
    nan_T = T.copy()
    nan_T[2] = math.nan

    def init(nn, TT, tau=1.0, dt=1.0, bc=0, prec=1):
        return L.rlbm_init_fields(h, nx, ny, R._p(nn), R._p(TT), None, None, tau, dt, bc, 0, prec, None, None)

    assert init(bad_n, T) == R.RLBM_EINVAL
    assert init(n, nan_T) == R.RLBM_EINVAL
    assert init(n, T, tau=0.0) == R.RLBM_EINVAL
    assert init(n, T, tau=math.nan) == R.RLBM_EINVAL
    assert init(n, T, dt=1.5) == R.RLBM_EINVAL
    assert init(n, T, bc=7) == R.RLBM_EINVAL
    h7 = ctypes.c_void_p()
    assert L.rlbm_init_quadrature(ctypes.byref(h7), 3, 7, 2, 1) == R.RLBM_OK
    assert L.rlbm_init_fields(h7, nx, ny, R._p(n), R._p(T), None, None, 1.0, 1.0, 2, 0, 1, None, None) == \
        R.RLBM_EINVAL                                                       # wall with an odd angle count
    assert b"even" in L.rlbm_last_error(h7)
    assert L.rlbm_destroy(h7) == R.RLBM_OK
    assert init(n, T, prec=9) == R.RLBM_EINVAL
    assert L.rlbm_step(h, 1) == R.RLBM_ESTATE
    assert b"before" in L.rlbm_last_error(h)
    assert L.rlbm_moments(h, None, None, None, None, None) == R.RLBM_ESTATE
    b = ctypes.c_size_t()
    assert L.rlbm_workspace_bytes(h, 1024, 1024, 1, ctypes.byref(b)) == R.RLBM_OK
    # two buffers of 256 + 1 planes, four FP64 field planes, and the push
    # kernel's two partial-sum buffers (3 row slots x 8 moments per site)
    assert b.value >= (2 * 257 * 4 + 4 * 8 + 2 * 3 * 8 * 4) * 1024 * 1024
    assert L.rlbm_workspace_bytes(h, 1024, 1024, 5, ctypes.byref(b)) == R.RLBM_EINVAL   # no such precision
    # bfloat16 deviations: two buffers of 256 + 1 planes of 2 bytes, and two
    # buffers of 4 shells x 7 FP32 equilibrium coefficients per site
    assert L.rlbm_workspace_bytes(h, 1024, 1024, R.RLBM_BF16DEV, ctypes.byref(b)) == R.RLBM_OK
    assert b.value >= (2 * 257 * 2 + 2 * 4 * 7 * 4 + 4 * 8 + 2 * 3 * 8 * 4) * 1024 * 1024
    assert L.rlbm_set_waves(h, 17) == R.RLBM_EINVAL
    assert L.rlbm_destroy(h) == R.RLBM_OK


def test_failed_initialisation_leaves_no_fields():
    """A call of rlbm_init_fields that passes the argument checks and then
    fails (here: no device) leaves the context without fields, so that a step
    or a moments call is refused instead of running on freed tables."""
    _lib_or_skip()
    L = R.lib()
    h = ctypes.c_void_p()
    assert L.rlbm_init_quadrature(ctypes.byref(h), 3, 8, 2, 1) == R.RLBM_OK
    n = np.ones(6)
    rc = L.rlbm_init_fields(h, 3, 2, R._p(n), R._p(n), None, None, 1.0, 1.0, 0, 0, 1, None, None)
    if rc == R.RLBM_OK:
        L.rlbm_destroy(h)
        pytest.skip("a device is present: the initialisation succeeded")
    assert rc == R.RLBM_EDEVICE
    assert L.rlbm_step(h, 1) == R.RLBM_ESTATE
    assert L.rlbm_moments(h, None, None, None, None, None) == R.RLBM_ESTATE
    assert L.rlbm_destroy(h) == R.RLBM_OK


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: without the built library every entry raises."""
    monkeypatch.setattr(R, "_L", None)
    monkeypatch.setattr(R, "SO_PATH", str(tmp_path / "librlbm.so"))
    with pytest.raises(ImportError, match="not built"):
        R.lib()
    with pytest.raises(ImportError, match="not built"):
        R.Solver(4, 16, 3)


@pytest.mark.parametrize("stat,name", [(1, "fd"), (2, "be")])
def test_host_quantum_equilibrium_matches_oracle(stat, name):
    """The library's own radial integrals and fugacity solve (host code of
    the kernels' device functions) against the oracle's, on the discrete
    truncated equilibrium of Fermi-Dirac and Bose-Einstein statistics."""
    _lib_or_skip()
    rng = np.random.default_rng(30 + stat)
    for (Np, K, N) in [(4, 64, 3), (6, 32, 5), (3, 12, 2)]:
        s = R.Solver(Np, K, N).set_statistics(name)
        q = O.Quadrature(Np, K, N)
        for trial in range(6):
            n, T = rng.uniform(0.1, 1.5), rng.uniform(0.6, 1.6)
            ux, uy = rng.uniform(-0.7, 0.7, size=2)
            if stat == 2 and n / T ** 2 >= 1.6:
                continue
            got = s.host_feq(n, T, ux, uy)
            exp = q.feq(n, T, ux, uy, stat=stat)
            np.testing.assert_allclose(got, exp, rtol=1e-12, atol=1e-13 * np.abs(exp).max())
    s = R.Solver(3, 12, 2).set_statistics("be")
    with pytest.raises(R.RlbmError):
        s.host_feq(2.0, 1.0)                     # above Bose-Einstein condensation
