"""GPU parity of the wall and fixed boundaries (tile kernel) against the FP64
oracle: relative L-inf <= 1e-12 with FP64 populations, <= 1e-4 with FP32 after
1000 steps (tests/fieldcheck.py); conservation at walls; kernel choice."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from fieldcheck import check_fields, say

pytestmark = pytest.mark.gpu
PER, CLAMP, WALL, FIXED = 0, 1, 2, 3


def _rlbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_06856_amd import rlbm
    rlbm.lib()
    return rlbm


CASES = [
    # label, Np, K, N, nx, ny, fields, tau, dt, steps, bcx, bcy, waves
    ("walls_moving", 4, 16, 3, 200, 37, "paper_quadrant", 6.0, 1.0, 80, WALL, WALL, 0),
    ("walls_free_streaming", 3, 24, 2, 90, 21, "disc", np.inf, 1.0, 120, WALL, WALL, 3),
    ("fixed_both", 4, 16, 3, 130, 19, "quadrant", 3.0, 1.0, 60, FIXED, FIXED, 0),
    ("wall_x_fixed_y", 4, 20, 3, 70, 33, "paper_quadrant", 2.0, 1.0, 50, WALL, FIXED, 2),
    ("fixed_x_periodic_y", 3, 32, 3, 150, 1, "tube", 15.0, 1.0, 140, FIXED, PER, 0),
    ("periodic_x_wall_y", 4, 16, 3, 66, 25, "disc", 4.0, 0.8, 50, PER, WALL, 1),
    ("tiny_walls", 3, 6, 2, 5, 3, "quadrant", 2.0, 1.0, 20, WALL, WALL, 0),
]


def _fields(kind, nx, ny):
    if kind == "tube":
        return W.tube(nx, ny)
    if kind == "paper_quadrant":
        return W.paper_quadrant(nx, ny)
    if kind == "quadrant":
        return W.quadrant(nx, ny, seed=nx + ny)
    return W.disc(nx, ny, min(nx, ny) / 4, seed=nx)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_boundaries_fp64_match_oracle(case):
    rl = _rlbm()
    label, Np, K, N, nx, ny, kind, tau, dt, steps, bcx, bcy, waves = case
    fld = _fields(kind, nx, ny)
    say("case boundaries_fp64 %s" % label)
    s = rl.Solver(Np, K, N).init_fields(nx, ny, *fld, tau=tau, dt=dt, bcx=bcx, bcy=bcy, precision="f64")
    assert s.get_kernel() == "tile"
    if waves:
        s.set_waves(waves)
    ch0 = s.moments()[4]
    s.step(steps)
    n, eps, ux, uy, ch = s.moments()
    sim = O.Sim(O.Quadrature(Np, K, N), nx, ny, *fld, tau=tau, dt=dt, bcx=bcx, bcy=bcy)
    sim.step(steps)
    check_fields((n, eps, ux, uy), sim.fields(), 1e-12, label)
    if bcx in (PER, WALL) and bcy in (PER, WALL):   # walls keep mass and energy
        np.testing.assert_allclose(ch[:2], ch0[:2], rtol=1e-12)


@pytest.mark.slow
def test_walls_fp32_match_oracle_after_1000_steps():
    """FP32, Np=4 x K=64 (256 velocities), the circular shock in a closed box
    of 320 x 24 cells (walls on both axes, interior tiles in the middle
    rows), Kn = 0.01 and 1, 1000 steps: the waves reflect many times."""
    rl = _rlbm()
    nx, ny = 320, 24
    for Kn in (0.01, 1.0):
        tau = W.tau_of(Kn, nx)
        fld = W.disc(nx, ny, ny / 3, seed=13)
        say("case walls_fp32_1000 Kn=%g" % Kn)
        s = rl.Solver(4, 64, 3).init_fields(nx, ny, *fld, tau=tau, dt=W.dt_of(tau), bcx=WALL, bcy=WALL,
                                            precision="f32")
        s.step(1000)
        got = s.moments()[:4]
        sim = O.Sim(O.Quadrature(4, 64, 3), nx, ny, *fld, tau=tau, dt=W.dt_of(tau), bcx=WALL, bcy=WALL)
        sim.step(1000)
        check_fields(got, sim.fields(), 1e-4, "walls_fp32_1000_kn%g" % Kn)


def test_boundaries_choose_the_tile_kernel():
    rl = _rlbm()
    fld = W.quadrant(40, 8, seed=1)
    s = rl.Solver(6, 256, 5).init_fields(40, 8, *fld, tau=2.0, bcx=WALL, precision="f32")
    assert s.get_kernel() == "tile"            # 1536 velocities would take the push kernel
    with pytest.raises(rl.RlbmError):
        s.set_kernel("push")
    with pytest.raises(rl.RlbmError):          # no reversed velocity for an odd angle count
        rl.Solver(3, 7, 2).init_fields(8, 8, *W.quadrant(8, 8), tau=2.0, bcx=WALL, precision="f64")
    p = dict(Np=4, K=16, N=3, nx=64, ny=8, fields=W.quadrant(64, 8), tau=2.0, dt=1.0, bcx=WALL, bcy=0)
    with pytest.raises(rl.RlbmError):
        rl.Batch([p], precision="f32")
