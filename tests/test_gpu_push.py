"""GPU parity of the push kernel (next-step moments pushed as partial sums)
against the FP64 oracle and against the tile kernel, and the bookkeeping of
its partial sums when the populations change outside a step.

Tolerances as in test_gpu_parity: relative L-inf per field <= 1e-12 for FP64,
<= 1e-4 for FP32 after 1000 steps; the flow as a vector (tests/fieldcheck.py).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from fieldcheck import check_fields, say

pytestmark = pytest.mark.gpu


def _rlbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_06856_amd import rlbm
    rlbm.lib()
    return rlbm


def check(got, exp, tol, label):
    check_fields(got, exp, tol, label)


def gpu(rl, kernel, Np, K, N, nx, ny, fld, tau, dt, steps, prec="f64", bcx=0, bcy=0):
    s = rl.Solver(Np, K, N).init_fields(nx, ny, *fld, tau=tau, dt=dt, bcx=bcx, bcy=bcy, precision=prec)
    s.set_kernel(kernel)
    s.step(steps)
    return s.moments()[:4], s


def oracle(Np, K, N, nx, ny, fld, tau, dt, steps, bcx=0, bcy=0):
    sim = O.Sim(O.Quadrature(Np, K, N), nx, ny, *fld, tau=tau, dt=dt, bcx=bcx, bcy=bcy)
    sim.step(steps)
    return sim.fields()


CASES = [
    # (label, Np, K, N, nx, ny, fields, tau, dt, steps, bcx, bcy)
    ("tube_clamp", 3, 32, 3, 300, 1, "tube", 15.0, 1.0, 120, 1, 0),
    ("ragged_moving", 4, 16, 3, 200, 37, "paper_quadrant", 6.0, 1.0, 60, 0, 0),
    ("order5_clamp_y", 6, 40, 5, 130, 9, "quadrant", 0.7, 0.35, 30, 0, 1),
    ("order7", 8, 30, 7, 70, 20, "disc", 3.0, 1.0, 25, 0, 0),
    ("tiny", 3, 12, 2, 5, 3, "quadrant", 2.0, 1.0, 15, 0, 0),
    ("free_streaming", 3, 24, 2, 90, 31, "disc", np.inf, 1.0, 40, 0, 0),
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
def test_push_fp64_matches_oracle(case):
    rl = _rlbm()
    label, Np, K, N, nx, ny, kind, tau, dt, steps, bcx, bcy = case
    fld = _fields(kind, nx, ny)
    say("case push_fp64 %s" % label)
    got, _ = gpu(rl, "push", Np, K, N, nx, ny, fld, tau, dt, steps, bcx=bcx, bcy=bcy)
    exp = oracle(Np, K, N, nx, ny, fld, tau, dt, steps, bcx=bcx, bcy=bcy)
    check(got, exp, 1e-12, "push_" + label)
    tile, _ = gpu(rl, "tile", Np, K, N, nx, ny, fld, tau, dt, steps, bcx=bcx, bcy=bcy)
    check(got, tile, 1e-12, "push_vs_tile_" + label)


def test_auto_choice_by_velocity_count():
    rl = _rlbm()
    fld = W.quadrant(40, 8, seed=1)
    small = rl.Solver(4, 64, 3).init_fields(40, 8, *fld, tau=2.0, precision="f32")
    large = rl.Solver(6, 256, 5).init_fields(40, 8, *fld, tau=2.0, precision="f32")
    assert small.get_kernel() == "tile" and large.get_kernel() == "push"
    large.set_kernel("tile")
    assert large.get_kernel() == "tile"
    with pytest.raises(KeyError):
        large.set_kernel("other")


def test_checkpoint_resume_is_bitwise_with_push():
    """Partial sums rebuilt from restored populations equal those a step
    pushes, so a resumed run continues bitwise."""
    rl = _rlbm()
    nx, ny = 96, 40
    fld = W.disc(nx, ny, 9.0, seed=5)
    for prec in ("f64", "f32"):
        a = rl.Solver(4, 32, 3).init_fields(nx, ny, *fld, tau=4.0, precision=prec).set_kernel("push")
        a.step(30)
        b = rl.Solver(4, 32, 3).init_fields(nx, ny, *fld, tau=4.0, precision=prec).set_kernel("push")
        b.step(15)
        ck = b.get_populations()
        c = rl.Solver(4, 32, 3).init_fields(nx, ny, *fld, tau=4.0, precision=prec).set_kernel("push")
        c.step(3)                      # partial sums of another state, to be discarded
        c.set_populations(ck)
        c.step(15)
        assert np.array_equal(c.get_populations(), a.get_populations()), prec


def test_partial_sums_follow_external_changes():
    """After the populations change outside a step (stress injection,
    resampling, switching kernels), the push kernel's moments are those of
    the new populations: it matches the tile kernel run on the same state."""
    import torch
    rl = _rlbm()
    nx, ny = 64, 30
    fld = W.quadrant(nx, ny, seed=9)
    runs = {}
    for kern in ("push", "tile"):
        s = rl.Solver(4, 24, 3).init_fields(nx, ny, *fld, tau=3.0, precision="f64").set_kernel(kern)
        s.step(5)
        d = torch.full((nx * ny, 3), 0.01, device="cuda")
        d[:, 1] = -0.004
        rl.add_stress(s, d)
        s.step(4)
        fine = rl.Solver(4, 48, 3).init_fields(nx, ny, *fld, tau=3.0, precision="f64")
        fine.step(2)
        rl.resample(fine, s)
        s.step(4)
        s.set_kernel("tile" if kern == "push" else "push")
        s.step(3)
        s.set_kernel(kern)
        s.step(3)
        runs[kern] = s.moments()[:4]
    check(runs["push"], runs["tile"], 1e-12, "push_after_external_changes")


def test_push_fp32_matches_oracle_after_1000_steps():
    """FP32 populations, Np=4 x K=192 (768 velocities, where the automatic
    choice is the push kernel), 1000 steps, Kn = 0.01 and 1, on a 200 x 16
    periodic grid: four tile columns (the middle two on the interior load
    path, partial sums crossing every tile edge through the halo) and four
    4-row work-group bands."""
    rl = _rlbm()
    nx, ny = 200, 16
    for Kn in (0.01, 1.0):
        tau = W.tau_of(Kn, nx)
        fld = W.disc(nx, ny, ny / 3, seed=11)
        say("case push_fp32_1000 Kn=%g" % Kn)
        args = (4, 192, 3, nx, ny, fld, tau, W.dt_of(tau), 1000)
        got, s = gpu(rl, "auto", *args, prec="f32")
        assert s.get_kernel() == "push"
        exp = oracle(*args)
        check(got, exp, 1e-4, "push_fp32_1000_kn%g" % Kn)


@pytest.mark.timeout(400)
def test_precision_form_quadrature_fp32_matches_oracle_after_1000_steps():
    """The precision form's quadrature and order (Np=6 x K=256 = 1536
    velocities, order 5, Kn = 10) with FP32 populations on the push kernel,
    1000 steps of the quadrant problem on a 136 x 24 periodic grid (one
    interior tile column), against the FP64 oracle at the 1e-4 tolerance."""
    rl = _rlbm()
    nx, ny = 136, 24
    tau = W.tau_of(10.0, nx)
    fld = W.quadrant(nx, ny, seed=0)
    say("case precision_quadrature_fp32_1000 %dx%d" % (nx, ny))
    args = (6, 256, 5, nx, ny, fld, tau, W.dt_of(tau), 1000)
    got, s = gpu(rl, "auto", *args, prec="f32")
    assert s.get_kernel() == "push"
    exp = oracle(*args)
    check(got, exp, 1e-4, "precision_quadrature_fp32_1000")


def test_precision_form_full_size_fp32_against_fp64():
    """The quadrant problem at full size (2048^2, Np=6 x K=256 = 1536
    velocities, order 5, Kn = 10), 100 steps: FP32 against FP64 (both on the
    push kernel the automatic choice selects), and global conservation."""
    import torch
    rl = _rlbm()
    cfg = W.quadrant_shock(2048, steps=100)
    say("case precision_full 2048^2 x 1536, 100 steps")
    res = {}
    for prec in ("f32", "f64"):
        s = rl.Solver(cfg["Np"], cfg["K"], cfg["N"]).init_fields(cfg["nx"], cfg["ny"], *cfg["fields"], tau=cfg["tau"],
                                                                dt=cfg["dt"], precision=prec)
        assert s.get_kernel() == "push"
        ch0 = s.moments()[4]
        s.step(100)
        res[prec] = s.moments()
        del s
        torch.cuda.empty_cache()
        ch = res[prec][4]
        tol = 1e-12 if prec == "f64" else 1e-5
        assert abs(ch[0] - ch0[0]) <= tol * ch0[0] and abs(ch[1] - ch0[1]) <= tol * ch0[1], (prec, ch, ch0)
    check(res["f32"][:4], res["f64"][:4], 1e-5, "precision_full")
