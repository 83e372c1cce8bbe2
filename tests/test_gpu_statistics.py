"""GPU parity of the Fermi-Dirac and Bose-Einstein equilibria (Eq. feq_dist
with epsilon = +1, -1; tile kernel) against the FP64 oracle: relative L-inf
<= 1e-12 with FP64 populations, <= 1e-4 with FP32 after 1000 steps
(tests/fieldcheck.py); conservation; rest states; kernel choice."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from fieldcheck import check_fields, say

pytestmark = pytest.mark.gpu
STATS = {"fd": 1, "be": 2}


def _rlbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_06856_amd import rlbm
    rlbm.lib()
    return rlbm


CASES = [
    # label, stat, Np, K, N, nx, ny, fields, tau, dt, steps, bcx, bcy, waves
    ("fd_moving", "fd", 4, 16, 3, 200, 37, "paper_quadrant", 6.0, 1.0, 60, 0, 0, 0),
    ("be_moving", "be", 4, 16, 3, 200, 37, "paper_quadrant", 6.0, 1.0, 60, 0, 0, 0),
    ("fd_order5", "fd", 6, 32, 5, 70, 20, "quadrant", 3.0, 1.0, 40, 0, 0, 2),
    ("be_order5_tau_small", "be", 6, 32, 5, 70, 20, "quadrant", 0.8, 0.4, 40, 0, 0, 0),
    ("fd_walls", "fd", 4, 20, 3, 90, 21, "disc", 4.0, 1.0, 80, 2, 2, 3),
    ("be_tube_fixed", "be", 3, 32, 3, 150, 1, "tube", 15.0, 1.0, 140, 3, 0, 0),
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
def test_quantum_statistics_fp64_match_oracle(case):
    rl = _rlbm()
    label, stat, Np, K, N, nx, ny, kind, tau, dt, steps, bcx, bcy, waves = case
    fld = _fields(kind, nx, ny)
    say("case statistics_fp64 %s" % label)
    s = rl.Solver(Np, K, N).set_statistics(stat)
    s.init_fields(nx, ny, *fld, tau=tau, dt=dt, bcx=bcx, bcy=bcy, precision="f64")
    assert s.get_kernel() == "tile"
    if waves:
        s.set_waves(waves)
    ch0 = s.moments()[4]
    s.step(steps)
    n, eps, ux, uy, ch = s.moments()
    sim = O.Sim(O.Quadrature(Np, K, N), nx, ny, *fld, tau=tau, dt=dt, bcx=bcx, bcy=bcy, stat=STATS[stat])
    sim.step(steps)
    assert sim.nonphys() == 0
    check_fields((n, eps, ux, uy), sim.fields(), 1e-12, label)
    if bcx in (0, 2) and bcy in (0, 2):
        np.testing.assert_allclose(ch[:2], ch0[:2], rtol=1e-12)


@pytest.mark.slow
@pytest.mark.timeout(400)
def test_fermi_dirac_fp32_matches_oracle_after_1000_steps():
    """FP32, Np=4 x K=64, the circular shock on a 256 x 16 periodic grid
    (interior tiles), Fermi-Dirac statistics, Kn = 1, 1000 steps."""
    rl = _rlbm()
    nx, ny = 256, 16
    tau = W.tau_of(1.0, nx)
    fld = W.disc(nx, ny, ny / 3, seed=17)
    say("case fd_fp32_1000")
    s = rl.Solver(4, 64, 3).set_statistics("fd")
    s.init_fields(nx, ny, *fld, tau=tau, dt=W.dt_of(tau), precision="f32")
    s.step(1000)
    got = s.moments()[:4]
    sim = O.Sim(O.Quadrature(4, 64, 3), nx, ny, *fld, tau=tau, dt=W.dt_of(tau), stat=1)
    sim.step(1000)
    check_fields(got, sim.fields(), 1e-4, "fd_fp32_1000")


@pytest.mark.parametrize("stat", ["fd", "be"])
def test_uniform_rest_state_stays_with_quantum_statistics(stat):
    rl = _rlbm()
    s = rl.Solver(4, 32, 3).set_statistics(stat)
    s.init_fields(64, 8, 0.7, 1.3, tau=2.0, precision="f64")
    f0 = s.get_populations()
    s.step(25)
    np.testing.assert_allclose(s.get_populations(), f0, rtol=1e-12, atol=1e-16)


def test_quantum_statistics_choose_the_tile_kernel_and_check_condensation():
    rl = _rlbm()
    fld = W.quadrant(40, 8, seed=1)
    s = rl.Solver(6, 256, 5).set_statistics("fd")
    s.init_fields(40, 8, *fld, tau=2.0, precision="f32")
    assert s.get_kernel() == "tile"
    with pytest.raises(rl.RlbmError):
        s.set_kernel("push")
    b = rl.Solver(3, 16, 2).set_statistics("be")
    with pytest.raises(rl.RlbmError):                     # n / T^2 = 2 > zeta(2)
        b.init_fields(8, 8, 2.0, 1.0, tau=2.0, precision="f64")
    b.init_fields(8, 8, 1.0, 1.0, tau=2.0, precision="f64")
    b.step(3)
