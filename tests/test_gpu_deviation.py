"""GPU parity of the deviation storage against the FP64 oracle.

Deviation storage keeps g = f - F per site and velocity, with F the truncated
equilibrium of the site's last collision (Sec. 2.2, Eq.
mj-feq-expansion-truncated) held as per-shell harmonic coefficients.  The
step rebuilds the equilibrium at the four upwind corners of Eq.
interpolation from those coefficients, so the representation changes the
arithmetic, not the method:

  - F64DEV (g and coefficients in FP64) must match the oracle to the FP64
    tolerance of every parity test, relative L-inf <= 1e-12 per field (the
    flow as a vector, tests/fieldcheck.py), and its reconstructed populations
    g + F must match the oracle's populations;
  - F32DEV must match it to 1e-4 after 1000 steps, the FP32 tolerance;
  - BF16DEV rounds g to bfloat16 every step, the one departure from F32DEV.
    Its error against the oracle is reported per field and bounded as
    derived in test_precision_form_quadrature_deviation_after_1000_steps.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from fieldcheck import check_fields, field_errors, say

pytestmark = pytest.mark.gpu


def _rlbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_06856_amd import rlbm
    rlbm.lib()
    return rlbm


def gpu(rl, Np, K, N, nx, ny, fld, tau, dt, steps, prec, bcx=0, bcy=0):
    s = rl.Solver(Np, K, N).init_fields(nx, ny, *fld, tau=tau, dt=dt, bcx=bcx, bcy=bcy, precision=prec)
    assert s.get_kernel() == "push"
    s.step(steps)
    return s.moments()[:4], s


def oracle_sim(Np, K, N, nx, ny, fld, tau, dt, steps, bcx=0, bcy=0):
    sim = O.Sim(O.Quadrature(Np, K, N), nx, ny, *fld, tau=tau, dt=dt, bcx=bcx, bcy=bcy)
    sim.step(steps)
    return sim


def _fields(kind, nx, ny):
    if kind == "tube":
        return W.tube(nx, ny)
    if kind == "paper_quadrant":
        return W.paper_quadrant(nx, ny)
    if kind == "quadrant":
        return W.quadrant(nx, ny, seed=nx + ny)
    return W.disc(nx, ny, min(nx, ny) / 4, seed=nx)


def nmax_of(N):
    return 3 if N <= 3 else (5 if N <= 5 else 7)


def reconstruct(s, raw):
    """Populations f = g + F of a deviation checkpoint (FP64 storage):
    deviations [nvel][ny][nx], then coefficients [Np][2 Nm + 1][ny][nx] with
    F_v = sum_t C[shell][t] w_v {1, cos m th, sin m th}_t."""
    nv, S = s.nvel, s.nx * s.ny
    nt = 2 * nmax_of(s.N) + 1
    vals = raw.view(np.float64)
    g = vals[:nv * S].reshape(nv, S)
    C = vals[nv * S:].reshape(s.Np, nt, S)
    p, th, w = s.quadrature()
    f = g.copy()
    for v in range(nv):
        i = v // s.K
        h = [1.0]
        for m in range(1, nmax_of(s.N) + 1):
            h += [math.cos(m * th[v]), math.sin(m * th[v])]
        f[v] += w[v] * np.tensordot(np.array(h), C[i], axes=1)
    return f.reshape(nv, s.ny, s.nx)


CASES = [
    # (label, Np, K, N, nx, ny, fields, tau, dt, steps, bcx, bcy)
    ("tube_clamp", 3, 32, 3, 300, 1, "tube", 15.0, 1.0, 120, 1, 0),
    ("ragged_moving", 4, 16, 3, 200, 37, "paper_quadrant", 6.0, 1.0, 60, 0, 0),
    ("order5_clamp_y", 6, 40, 5, 130, 9, "quadrant", 0.7, 0.35, 30, 0, 1),
    ("order4_clamp_xy", 5, 20, 4, 66, 6, "quadrant", 2.0, 1.0, 20, 1, 1),
    ("order7", 8, 30, 7, 70, 20, "disc", 3.0, 1.0, 25, 0, 0),
    ("tiny", 3, 12, 2, 5, 3, "quadrant", 2.0, 1.0, 15, 0, 0),
    ("free_streaming", 3, 24, 2, 90, 31, "disc", np.inf, 1.0, 40, 0, 0),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_f64dev_matches_oracle(case):
    rl = _rlbm()
    label, Np, K, N, nx, ny, kind, tau, dt, steps, bcx, bcy = case
    fld = _fields(kind, nx, ny)
    say("case f64dev %s" % label)
    got, s = gpu(rl, Np, K, N, nx, ny, fld, tau, dt, steps, "f64dev", bcx=bcx, bcy=bcy)
    sim = oracle_sim(Np, K, N, nx, ny, fld, tau, dt, steps, bcx=bcx, bcy=bcy)
    check_fields(got, sim.fields(), 1e-12, "f64dev_" + label)
    f = reconstruct(s, s.get_populations())
    fo = sim.get_f()
    err = np.abs(f - fo).max() / np.abs(fo).max()
    say("f64dev_%s populations rel Linf %.3e" % (label, err))
    assert err <= 1e-12, err


def test_initial_state_is_the_equilibrium():
    """Zero steps: the fields of the stored state are the initial fields (f =
    F exactly; the coefficients are FP32 in BF16DEV / F32DEV)."""
    rl = _rlbm()
    nx, ny = 70, 9
    fld = W.paper_quadrant(nx, ny)
    n, T, ux, uy = fld
    exp = (n, 2.0 * n * T, ux, uy)
    for prec, tol in (("f64dev", 1e-13), ("f32dev", 1e-6), ("bf16dev", 1e-6)):
        s = rl.Solver(4, 20, 3).init_fields(nx, ny, *fld, tau=3.0, precision=prec)
        check_fields(s.moments()[:4], exp, tol, "init_" + prec)


def test_f32dev_matches_oracle_after_1000_steps():
    """F32DEV, Np=4 x K=192 (768 velocities), 1000 steps, Kn = 0.01 and 1, on a
    200 x 16 periodic grid: four tile columns (two on the interior load path,
    coefficients and partial sums crossing every tile edge) and four 4-row
    work-group bands."""
    rl = _rlbm()
    nx, ny = 200, 16
    for Kn in (0.01, 1.0):
        tau = W.tau_of(Kn, nx)
        fld = W.disc(nx, ny, ny / 3, seed=11)
        say("case f32dev_1000 Kn=%g" % Kn)
        args = (4, 192, 3, nx, ny, fld, tau, W.dt_of(tau), 1000)
        got, _ = gpu(rl, *args, "f32dev")
        exp = oracle_sim(*args).fields()
        check_fields(got, exp, 1e-4, "f32dev_1000_kn%g" % Kn)


@pytest.mark.timeout(600)
def test_precision_form_quadrature_deviation_after_1000_steps():
    """The precision form's quadrature and order (Np=6 x K=256 = 1536
    velocities, order 5, Kn = 10), quadrant problem on a 136 x 24 periodic
    grid, 1000 steps, against the FP64 oracle.

    F32DEV: the FP32 tolerance, 1e-4.

    BF16DEV: rounding g stochastically to bfloat16 (8 significant bits)
    errs by less than one ulp, at most 2^-7 |g|, with zero mean and a
    standard deviation of at most half an ulp, 2^-8 |g|, independently
    between velocities, sites and steps.  A moment M = sum_v P(v) f_v then
    takes per step an error of standard deviation at most 2^-8 ||P g||_2,
    and after n steps sqrt(n) times that.  With |g| at most |f| and P of one
    sign over a shell, ||P g||_2 / |M| is at most about 1 / sqrt(K) (a
    shell's K velocities share |P|): 1/16 here.  So the relative field error
    has a standard deviation below 2^-8 sqrt(1000) / 16 = 7.7e-3, and the
    largest of the 3264 sites stays below 4 of those: 3.1e-2, asserted on n
    and eps as 3e-2.  The flow U^i ~ T^0i / (eps + P) = T^0i / (1.5 eps)
    takes the error of T^0i, bounded relative to T^00 = eps by the same
    3e-2: |dU| stays below 2e-2 in units of c, asserted (this flow is slow,
    ~1e-3 c, so the error relative to its own size is reported, not
    bounded).  The global charges follow the same law over the 3264 sites:
    their drift stays below 4 x 7.7e-3 / sqrt(3264) = 5.4e-4.  Round to
    nearest would be biased here (it drops every per-step change smaller
    than half an ulp): on this problem it gave errors of 4.4e-4 (n),
    7.1e-4 (eps), 3.3e-4 (|dU|) and a drift of 1.7e-4 in N^0, against
    1.1e-4, 1.7e-4, 7.7e-5 and 2.5e-6 with stochastic rounding."""
    rl = _rlbm()
    nx, ny = 136, 24
    tau = W.tau_of(10.0, nx)
    fld = W.quadrant(nx, ny, seed=0)
    args = (6, 256, 5, nx, ny, fld, tau, W.dt_of(tau), 1000)
    say("case precision_quadrature_deviation_1000 %dx%d" % (nx, ny))
    sim0 = O.Sim(O.Quadrature(6, 256, 5), nx, ny, *fld, tau=tau, dt=W.dt_of(tau))
    ch0 = sim0.charges()
    exp = oracle_sim(*args).fields()
    got, _ = gpu(rl, *args, "f32dev")
    check_fields(got, exp, 1e-4, "precision_quadrature_f32dev_1000")
    s = rl.Solver(6, 256, 5).init_fields(nx, ny, *fld, tau=tau, dt=W.dt_of(tau), precision="bf16dev")
    s.step(1000)
    n, eps, ux, uy, ch = s.moments()
    e_n, e_eps, e_u = field_errors((n, eps, ux, uy), exp)
    du = float(np.hypot(ux - exp[2], uy - exp[3]).max())
    drift = [abs(ch[k] - ch0[k]) / abs(ch0[k]) for k in (0, 1)]
    say("precision_quadrature_bf16dev_1000 n=%.3e eps=%.3e |du|=%.3e c (flow-relative %.3e), charge drift "
        "N0 %.3e T00 %.3e" % (e_n, e_eps, du, e_u, drift[0], drift[1]))
    assert e_n <= 3e-2 and e_eps <= 3e-2 and du <= 2e-2, (e_n, e_eps, du)
    assert max(drift) <= 5.4e-4, drift
    assert e_n > 0.0   # the rounding is there: BF16DEV is not silently another storage


BF16_CASES = [
    # (Np, K, N): 5 to 11 velocities per segment (padded to a load batch),
    # one case per order class
    (4, 20, 3),
    (6, 40, 5),
    (8, 44, 7),
]


@pytest.mark.parametrize("Np,K,N", BF16_CASES, ids=["order%d" % c[2] for c in BF16_CASES])
def test_bf16dev_within_the_rounding_bound_at_every_order(Np, K, N):
    """BF16DEV on ragged segments and at every order class (each its own
    kernel instance, with its own register allocation): 30 steps stay within
    the stochastic-rounding bound derived in
    test_precision_form_quadrature_deviation_after_1000_steps, 4 x 2^-8
    sqrt(steps) / sqrt(K), against F64DEV (which equals the oracle to
    1e-12)."""
    rl = _rlbm()
    nx, ny, steps = 150, 9, 30
    fld = W.quadrant(nx, ny, seed=3)
    tau = 1.5
    say("case bf16dev_orders Np=%d K=%d N=%d %dx%d" % (Np, K, N, nx, ny))
    ref, _ = gpu(rl, Np, K, N, nx, ny, fld, tau, 1.0, steps, "f64dev")
    got, _ = gpu(rl, Np, K, N, nx, ny, fld, tau, 1.0, steps, "bf16dev")
    e_n, e_eps, _ = field_errors(got, ref)
    du = float(np.hypot(got[2] - ref[2], got[3] - ref[3]).max())
    bound = 4 * 2.0 ** -8 * math.sqrt(steps) / math.sqrt(K)
    say("bf16dev_orders N=%d n=%.3e eps=%.3e |du|=%.3e bound %.3e" % (N, e_n, e_eps, du, bound))
    assert e_n <= bound and e_eps <= bound and du <= bound, (e_n, e_eps, du, bound)
    assert e_n > 0.0


def test_checkpoint_resume_is_bitwise():
    """A run resumed from a checkpoint of (deviations, coefficients)
    continues bit for bit: the partial sums rebuilt from the restored state
    equal those a step pushes."""
    rl = _rlbm()
    nx, ny = 96, 40
    fld = W.disc(nx, ny, 9.0, seed=5)
    for prec in ("bf16dev", "f32dev", "f64dev"):
        a = rl.Solver(4, 32, 3).init_fields(nx, ny, *fld, tau=4.0, precision=prec)
        a.step(30)
        b = rl.Solver(4, 32, 3).init_fields(nx, ny, *fld, tau=4.0, precision=prec)
        b.step(15)
        ck = b.get_populations()
        c = rl.Solver(4, 32, 3).init_fields(nx, ny, *fld, tau=4.0, precision=prec)
        c.step(3)                      # partial sums of another state, to be discarded
        c.set_populations(ck)
        c.step(15)
        assert np.array_equal(c.get_populations(), a.get_populations()), prec


def test_moments_device_matches_moments():
    import torch
    rl = _rlbm()
    nx, ny = 80, 12
    fld = W.paper_quadrant(nx, ny)
    s = rl.Solver(4, 24, 3).init_fields(nx, ny, *fld, tau=5.0, precision="bf16dev")
    s.step(20)
    n, eps, ux, uy, ch = s.moments()
    d = torch.zeros(4 * nx * ny, dtype=torch.float64, device="cuda")
    dc = torch.zeros(4, dtype=torch.float64, device="cuda")
    s.moments_device(d, dc)
    torch.cuda.synchronize()
    got = d.cpu().numpy().reshape(4, ny, nx)
    for a, b in zip(got, (n, eps, ux, uy)):
        assert np.array_equal(a, b)
    assert np.allclose(dc.cpu().numpy(), ch, rtol=1e-14, atol=0)


def test_unsupported_combinations_are_rejected():
    rl = _rlbm()
    nx, ny = 40, 8
    fld = W.quadrant(nx, ny, seed=2)
    for bc in (2, 3):   # wall, fixed
        with pytest.raises(rl.RlbmError):
            rl.Solver(4, 16, 3).init_fields(nx, ny, *fld, tau=2.0, bcx=bc, precision="bf16dev")
    with pytest.raises(rl.RlbmError):
        rl.Solver(4, 16, 3).set_statistics("fd").init_fields(nx, ny, *fld, tau=2.0, precision="bf16dev")
    s = rl.Solver(4, 16, 3).init_fields(nx, ny, *fld, tau=2.0, precision="bf16dev")
    with pytest.raises(rl.RlbmError):
        s.set_kernel("tile")
    assert s.get_kernel() == "push"
    s.step(2)
    assert np.isfinite(s.moments()[0]).all()
