"""Closed forms the oracle is checked against (test infrastructure only).

* The free-streaming (tau -> inf) solution of the 1D shock tube for a massless
  gas in 2+1 dimensions (Appendix A).
* The Landau-frame solution of a (1+1)-dimensional energy-momentum tensor.
* The relative L2 error of Eq. rel_err.
"""
import numpy as np


def _i012(w):
    """i_0, i_1, i_2 of Appendix A for |w| <= 1."""
    w = np.clip(w, -1.0, 1.0)
    ac = np.arccos(w)
    sq = np.sqrt(1.0 - w * w)
    return 2 * np.pi - 2 * ac, -2 * sq, np.pi - w * sq - ac


def free_streaming_tube(w, nL, TL, nR, TR):
    """Moments of the free-streaming shock tube at self-similar w = x/t.

    Returns N^0, N^x, T^00, T^0x, T^xx, T^yy (N^y = T^0y = T^xy = 0).  The
    pressure is P = nT.  The T^00 line of Appendix A prints P_L as its constant
    term; on the light cone T^00 = T^xx + T^yy must hold and the unperturbed
    left state (w < -1) has T^00 = eps_L = 2 P_L, so the constant is 2 P_L.
    The other five lines are used as printed.
    """
    w = np.asarray(w, dtype=np.float64)
    PL, PR = nL * TL, nR * TR
    i0, i1, i2 = _i012(w)
    N0 = nL + i0 * (nR - nL) / (2 * np.pi)
    Nx = i1 * (nR - nL) / (2 * np.pi)
    T00 = 2 * PL + i0 * (PR - PL) / np.pi
    T0x = i1 * (PR - PL) / np.pi
    Txx = PL + i2 * (PR - PL) / np.pi
    Tyy = PL + (i0 - i2) * (PR - PL) / np.pi
    # unperturbed regions
    left, right = w < -1, w > 1
    N0 = np.where(left, nL, np.where(right, nR, N0))
    Nx = np.where(left | right, 0.0, Nx)
    T00 = np.where(left, 2 * PL, np.where(right, 2 * PR, T00))
    T0x = np.where(left | right, 0.0, T0x)
    Txx = np.where(left, PL, np.where(right, PR, Txx))
    Tyy = np.where(left, PL, np.where(right, PR, Tyy))
    return N0, Nx, T00, T0x, Txx, Tyy


def landau_1d(N0, Nx, T00, T0x, Txx):
    """Landau frame of a (1+1)D tensor: eps, beta, n (largest root of the 2x2 pencil)."""
    eps = 0.5 * ((T00 - Txx) + np.sqrt((T00 + Txx) ** 2 - 4 * T0x ** 2))
    beta = T0x / (eps + Txx)
    gamma = 1.0 / np.sqrt(1.0 - beta ** 2)
    n = gamma * (N0 - beta * Nx)
    return eps, beta, n


def rel_l2(a, ref):
    """Eq. rel_err: ||a - ref||_2 / ||ref||_2."""
    a, ref = np.asarray(a, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(a - ref) / np.linalg.norm(ref))
