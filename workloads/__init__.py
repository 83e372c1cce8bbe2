"""Seeded synthetic inputs for the relativistic lattice Boltzmann solver.

This module is shared by the GPU path's tests and benchmark and by the oracle's
tests.  It holds none of the method's arithmetic: it only produces initial
macroscopic fields (n, T, U^x, U^y on a [ny][nx] grid) and the run parameters
of the shock-wave workloads.  The paper uses synthetic Riemann problems only
(the 1D tube of Sec. 3.1 and the 2D quadrant problem of Sec. 3.2); no public
dataset is involved.

Random numbers come from a counter-based generator so that every language
produces the same stream: u(seed, k) = (SplitMix64(seed * 2^32 + k) >> 11) * 2^-53,
SplitMix64 as published by Steele, Lea and Flood (2014).
"""
import math

import numpy as np

_M64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 finaliser of the counter x (numpy uint64 array or int)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(seed, k):
    """u(seed, k) in [0, 1) for integer counter(s) k."""
    k = np.asarray(k, dtype=np.uint64)
    base = np.uint64((int(seed) << 32) & _M64)
    with np.errstate(over="ignore"):
        z = splitmix64(base + k)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _grid(nx, ny):
    return np.zeros((ny, nx))


def tube(nx, ny=1, nL=1.0, TL=1.0, nR=0.125, TR=0.75):
    """1D shock tube at rest: cell i is on the left iff i < nx/2."""
    n, T = _grid(nx, ny), _grid(nx, ny)
    left = (np.arange(nx) < nx / 2)[None, :]
    n[:] = np.where(left, nL, nR)
    T[:] = np.where(left, TL, TR)
    return n, T, _grid(nx, ny), _grid(nx, ny)


def disc(nx, ny, R, n_in=1.0, T_in=1.5, n_out=0.5, T_out=1.0, noise=0.01, seed=0):
    """Circular shock at rest: a disc of radius R at the grid centre, with
    n <- n (1 + noise (2u - 1)) per site (counter = site index y*nx + x)."""
    x = np.arange(nx) + 0.5 - nx / 2
    y = np.arange(ny) + 0.5 - ny / 2
    inside = (x[None, :] ** 2 + y[:, None] ** 2) < R * R
    n = np.where(inside, n_in, n_out).astype(np.float64)
    T = np.where(inside, T_in, T_out).astype(np.float64)
    if noise:
        u = uniform(seed, np.arange(nx * ny)).reshape(ny, nx)
        n = n * (1.0 + noise * (2.0 * u - 1.0))
    return n, T, _grid(nx, ny), _grid(nx, ny)


def quadrant(nx, ny, seed=0):
    """Four quadrants at rest, quadrant q = [x >= nx/2] + 2 [y >= ny/2], with
    n_q = 0.25 + 0.75 u(seed, 2q) and T_q = 0.5 + u(seed, 2q + 1)."""
    qx = (np.arange(nx) >= nx / 2).astype(int)
    qy = (np.arange(ny) >= ny / 2).astype(int)
    qi = qx[None, :] + 2 * qy[:, None]
    nq = 0.25 + 0.75 * uniform(seed, 2 * np.arange(4))
    Tq = 0.5 + uniform(seed, 2 * np.arange(4) + 1)
    return nq[qi], Tq[qi], _grid(nx, ny), _grid(nx, ny)


def paper_quadrant(nx, ny):
    """The 2D initial state of Sec. 3.2 (quadrants with (n, T, beta_x, beta_y)),
    returned with U^i = gamma beta^i."""
    table = {  # (x>0, y>0): n, T, bx, by
        (0, 0): (0.5, 1.0, 0.0, 0.0),
        (1, 0): (0.5, 2.0, 0.0, 0.1),
        (0, 1): (0.5, 2.0, 0.1, 0.0),
        (1, 1): (1.0, 1.0, 0.0, 0.0),
    }
    n, T, ux, uy = (_grid(nx, ny) for _ in range(4))
    for (qx, qy), (nn, TT, bx, by) in table.items():
        mx = (np.arange(nx) >= nx / 2) == bool(qx)
        my = (np.arange(ny) >= ny / 2) == bool(qy)
        m = my[:, None] & mx[None, :]
        g = 1.0 / math.sqrt(1.0 - bx * bx - by * by)
        n[m], T[m], ux[m], uy[m] = nn, TT, g * bx, g * by
    return n, T, ux, uy


def tau_of(Kn, L):
    """Kn = c tau / L with L the side in lattice cells (Sec. 3.1)."""
    return Kn * L


def dt_of(tau):
    """Time step: 1 (CFL 1 along the axes), halved relaxation time where tau < 2
    so that the explicit relaxation factor stays below one."""
    return min(1.0, tau / 2.0)


# --------------------------------------------------------------------------
# The shock-wave workloads (grid, quadrature, initial state, steps).
# --------------------------------------------------------------------------

def tube_1d(nx=1000):
    """Tube: nx x 1, Np=3 x K=32 (96 velocities), order 3, FP64, clamp in x,
    left n=1 T=1, right n=0.125 T=0.75, Kn=0.05, 500 steps."""
    tau = tau_of(0.05, nx)
    return dict(name="tube1d_%dx1_np3_k32" % nx, nx=nx, ny=1, Np=3, K=32, N=3, precision="f64",
                tau=tau, dt=dt_of(tau), bcx=1, bcy=0, steps=500, fields=tube(nx, 1))


def circular_shock(side=1024, Kn=0.01, seed=0, steps=2000):
    """Circular shock: side^2 periodic, Np=4 x K=64 (256 velocities), order 3,
    FP32; disc radius side/8 (128 at 1024) n=1 T=1.5 inside, n=0.5 T=1
    outside, 1% seeded noise on n."""
    tau = tau_of(Kn, side)
    return dict(name="circular_shock_%d_np4_k64_kn%g" % (side, Kn), nx=side, ny=side, Np=4, K=64,
                N=3, precision="f32", tau=tau, dt=dt_of(tau), bcx=0, bcy=0, steps=steps,
                fields=disc(side, side, side / 8, seed=seed))


def quadrant_shock(side=2048, Np=6, K=256, Kn=10.0, seed=0, steps=1000, precision="f32"):
    """High-Kn quadrant Riemann problem: side^2 periodic, Np=6 x K=256 (1536
    velocities), order 5."""
    tau = tau_of(Kn, side)
    return dict(name="quadrant_%d_np%d_k%d_kn%g" % (side, Np, K, Kn), nx=side, ny=side, Np=Np, K=K,
                N=Np - 1, precision=precision, tau=tau, dt=dt_of(tau), bcx=0, bcy=0,
                steps=steps, fields=quadrant(side, side, seed))


def batch_problems(count=48, seed=0, steps=1000):
    """Independent shock problems of uneven size: side from {128,256,512,1024},
    Kn = 10^(-3 + 4u), K from {48,64,96,128}, Np=4, disc (radius side/8) or
    quadrant state, FP32.  Counters: 8*i + {0..4} for problem i."""
    sides, Ks = (128, 256, 512, 1024), (48, 64, 96, 128)
    out = []
    for i in range(count):
        u = uniform(seed, 8 * i + np.arange(5))
        side = sides[min(3, int(4 * u[0]))]
        Kn = 10.0 ** (-3.0 + 4.0 * u[1])
        K = Ks[min(3, int(4 * u[2]))]
        tau = tau_of(Kn, side)
        if u[3] < 0.5:
            fld = disc(side, side, side / 8, seed=seed * 1000 + i)
        else:
            fld = quadrant(side, side, seed * 1000 + i)
        out.append(dict(name="batch%d_%d_k%d" % (i, side, K), nx=side, ny=side, Np=4, K=K, N=3,
                        precision="f32", tau=tau, dt=dt_of(tau), Kn=Kn, bcx=0, bcy=0,
                        steps=steps, fields=fld))
    return out


def random_shock(side, seed):
    """Random disc or quadrant state for the learned correction's data:
    counters 0..3 of ``seed`` pick the kind, Kn = 10^(-1 + 2u), and the disc
    radius side/8 .. side/4."""
    u = uniform(seed, np.arange(4))
    Kn = 10.0 ** (-1.0 + 2.0 * u[0])
    if u[1] < 0.5:
        R = side / 8 + u[2] * side / 8
        fld = disc(side, side, R, seed=seed)
    else:
        fld = quadrant(side, side, seed)
    return Kn, fld
