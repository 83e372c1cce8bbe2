"""The locality that tests/test_gpu_fullsize.py relies on, checked on the
oracle alone: after t steps a site of a periodic grid equals the centre of a
block of half-width t + 1 (t would do) cut around it (wrapped) and stepped
with clamped edges (Eq. interpolation reads only upwind neighbours; the collision is
local)."""
import numpy as np

import oracle as O
import workloads as W

from test_gpu_fullsize import HALF, STEPS, block


def test_block_centre_equals_full_periodic_run():
    nx, ny = 40, 28
    q = O.Quadrature(4, 12, 3)
    fld = W.disc(nx, ny, 6.0, seed=2)
    tau = 3.0
    full = O.Sim(q, nx, ny, *fld, tau=tau, dt=1.0)
    full.step(STEPS)
    ref = full.fields()
    w = 2 * HALF + 1
    for (x, y) in [(0, 0), (nx - 1, ny - 1), (14, 20), (26, 8), (20, 14)]:
        sub = [block(np.broadcast_to(f, (ny, nx)), x, y, HALF) for f in fld]
        sim = O.Sim(q, w, w, *sub, tau=tau, dt=1.0, bcx=1, bcy=1)
        sim.step(STEPS)
        got = [f[HALF, HALF] for f in sim.fields()]
        for g, r in zip(got, ref):
            assert abs(g - r[y, x]) <= 1e-13 * max(1.0, abs(r[y, x])), (x, y, g, r[y, x])


def test_block_of_half_width_t_minus_one_is_not_enough():
    """The cone is tight: with half-width t - 1 the clamped edge reaches the
    centre (half-width t is the least that works; the GPU test takes t + 1)."""
    nx, ny = 40, 28
    q = O.Quadrature(4, 12, 3)
    fld = W.disc(nx, ny, 6.0, seed=2)
    full = O.Sim(q, nx, ny, *fld, tau=3.0, dt=1.0)
    full.step(STEPS)
    ref = full.fields()
    h = STEPS - 1
    x, y = 14, 14   # on the disc edge, where the state varies
    sub = [block(np.broadcast_to(f, (ny, nx)), x, y, h) for f in fld]
    sim = O.Sim(q, 2 * h + 1, 2 * h + 1, *sub, tau=3.0, dt=1.0, bcx=1, bcy=1)
    sim.step(STEPS)
    got = sim.fields()[0][h, h]
    assert abs(got - ref[0][y, x]) > 1e-9
