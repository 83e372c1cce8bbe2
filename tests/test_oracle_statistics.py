"""Pins of the oracle's Fermi-Dirac and Bose-Einstein equilibria (Eq.
feq_dist with epsilon = +1, -1; the paper notes its quadratures apply to
them unchanged).  The readings are stated in the oracle: normalisation
1/(2 pi), radial integrals G_k(z) = -Li_{k+1}(-z) (FD), Li_{k+1}(z) (BE),
rank-k moments = Maxwell-Juttner ones times G_k / G_1.  The references are
mpmath's polylogarithm, direct numerical integration of the distributions,
closed forms and conservation laws."""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle as O

FD, BE = 1, 2
ETA = np.diag([1.0, -1.0, -1.0])


@pytest.mark.parametrize("stat", [FD, BE])
def test_radial_integrals_match_mpmath_polylog(stat):
    zs = [1e-6, 0.01, 0.3, 0.5, 0.51, 0.9, 0.99, 0.999999, 1.0]
    if stat == FD:
        zs += [1.0001, 1.5, 2.7, 7.5, 40.0, 3e3, 1e8]
    mp.mp.dps = 30
    for z in zs:
        for k in range(9):
            if stat == BE and z == 1.0 and k == 0:
                continue            # Li_1(1) diverges
            s = k + 1
            ref = -mp.polylog(s, -z) if stat == FD else mp.polylog(s, z)
            got = O.qs_G(k, z, stat)
            assert abs(got - float(ref)) <= 2e-15 * abs(float(ref)), (stat, z, k, got, float(ref))


def test_radial_integrals_match_direct_integration():
    mp.mp.dps = 25
    for stat, eps in ((FD, 1), (BE, -1)):
        for z in (0.2, 0.8, 3.0):
            if stat == BE and z > 1:
                continue
            for k in (0, 1, 2, 5):
                f = lambda x: x ** k / (mp.exp(x) / z + eps)
                ref = mp.quad(f, [0, 1, 5, 20, mp.inf]) / mp.factorial(k)
                assert abs(O.qs_G(k, z, stat) - float(ref)) <= 1e-14 * float(ref), (stat, z, k)


def test_radial_integral_closed_forms_and_classical_limit():
    z = 0.37
    assert abs(O.qs_G(0, z, FD) - math.log1p(z)) < 1e-16
    assert abs(O.qs_G(0, z, BE) + math.log1p(-z)) < 1e-16
    zeta = {2: math.pi ** 2 / 6, 4: math.pi ** 4 / 90, 6: math.pi ** 6 / 945}
    for s, zv in zeta.items():
        assert abs(O.qs_G(s - 1, 1.0, BE) - zv) < 1e-15 * zv
        assert abs(O.qs_G(s - 1, 1.0, FD) - (1 - 2.0 ** (1 - s)) * zv) < 1e-15 * zv
    for stat in (FD, BE):   # z -> 0: both statistics become Maxwell-Juttner (G_k -> z)
        for k in range(6):
            assert abs(O.qs_G(k, 1e-9, stat) / 1e-9 - 1) < 1e-9


def _integrated_moments(stat, z, T, U):
    """N^mu and T^{mu nu} of f = (1/2pi) / (z^-1 exp(U.p/T) +- 1) by direct
    numerical integration over p (d^2p/p^0 = dp dtheta for massless p),
    adaptive Gauss-Kronrod in both variables (scipy)."""
    from scipy import integrate
    eps = 1.0 if stat == FD else -1.0

    def radial(th, k):
        A = U[0] - U[1] * math.cos(th) - U[2] * math.sin(th)
        def f(p):   # p^k / (z^-1 e^(A p / T) + eps), written without overflow
            t = math.exp(-A * p / T)
            return p ** k * z * t / (1.0 + eps * z * t)
        return integrate.quad(f, 0, np.inf,
                              epsabs=0, epsrel=1e-13, limit=200)[0]

    def ang(g, k):
        return integrate.quad(lambda th: g(th) * radial(th, k), 0, 2 * math.pi, epsabs=0, epsrel=1e-13,
                              limit=200)[0] / (2 * math.pi)

    e = (lambda th: 1.0, math.cos, math.sin)
    N = np.array([ang(e[mu], 1) for mu in range(3)])
    Tm = np.zeros((3, 3))
    for mu in range(3):
        for nu in range(mu, 3):
            Tm[mu, nu] = Tm[nu, mu] = ang(lambda th, mu=mu, nu=nu: e[mu](th) * e[nu](th), 2)
    return N, Tm


@pytest.mark.slow
@pytest.mark.parametrize("stat", [FD, BE])
def test_discrete_equilibrium_reproduces_the_integrated_distribution(stat):
    """The discrete truncated equilibrium (order 3, an exact quadrature) of
    the quantum statistics at a moving frame carries N^mu and T^{mu nu} of
    the actual distribution, integrated directly: a check of the moment
    factors and of the fugacity solve together."""
    n, T, ux, uy = 0.8, 1.1, 0.3, -0.2
    q = O.Quadrature(4, 64, 3)
    m = q.moments(q.feq(n, T, ux, uy, stat=stat))
    # fugacity from n = T^2 G_1(z), by mpmath, independently
    mp.mp.dps = 30
    G1 = (lambda z: -mp.polylog(2, -z)) if stat == FD else (lambda z: mp.polylog(2, z))
    z = float(mp.findroot(lambda z: G1(z) - n / T ** 2, 0.5))
    U = [math.sqrt(1 + ux * ux + uy * uy), ux, uy]
    Nref, Tref = _integrated_moments(stat, z, T, U)
    np.testing.assert_allclose(m[:3], Nref, rtol=1e-12, atol=1e-13)
    got_T = np.array([[m[3], m[4], m[5]], [m[4], m[6], m[7]], [m[5], m[7], m[8]]])
    np.testing.assert_allclose(got_T, Tref, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(m[:3], n * np.array(U), rtol=1e-12)   # N^mu = n U^mu


@pytest.mark.parametrize("stat", [FD, BE])
def test_frame_recovers_the_state_of_an_equilibrium(stat):
    q = O.Quadrature(4, 64, 3)
    rng = np.random.default_rng(4 + stat)
    for trial in range(10):
        n, T = rng.uniform(0.2, 1.2), rng.uniform(0.7, 1.5)
        ux, uy = rng.uniform(-0.6, 0.6, size=2)
        out, ok = O.qs_landau(q.moments(q.feq(n, T, ux, uy, stat=stat)), stat)
        assert ok
        np.testing.assert_allclose(out[[0, 2, 3, 4]], [n, ux, uy, T], rtol=1e-12, atol=1e-13)
        # eps = 2 n T G_2 / G_1 (P = eps / 2 for the massless gas)
        assert abs(out[1] - 2 * n * T * out[7]) < 1e-12 * out[1]


def test_bose_einstein_has_no_equilibrium_above_condensation():
    q = O.Quadrature(3, 16, 2)
    with pytest.raises(ValueError):
        q.feq(2.0, 1.0, stat=BE)            # n / T^2 = 2 > zeta(2)
    with pytest.raises(ValueError):
        O.Sim(q, 4, 4, 2.0, 1.0, tau=1.0, stat=BE)
    q.feq(2.0, 1.0, stat=FD)                # Fermi-Dirac has one at any n / T^2


@pytest.mark.parametrize("stat", [FD, BE])
def test_collision_conserves_charges_and_rest_state_stays(stat):
    q = O.Quadrature(4, 24, 3)
    sim = O.Sim(q, 10, 8, 0.7, 1.3, tau=2.0, dt=1.0, stat=stat)
    f0 = sim.get_f()
    sim.step(20)
    np.testing.assert_allclose(sim.get_f(), f0, rtol=1e-12, atol=1e-15)
    nx, ny = 30, 20
    u = np.random.default_rng(9).uniform(0, 1, size=(2, ny, nx))
    sim = O.Sim(q, nx, ny, 0.4 + 0.5 * u[0], 0.8 + 0.5 * u[1], tau=3.0, dt=1.0, stat=stat)
    c0 = sim.charges()
    sim.step(60)
    assert sim.nonphys() == 0
    np.testing.assert_allclose(sim.charges(), c0, rtol=1e-12, atol=1e-12)


def test_quantum_statistics_differ_from_maxwell_juttner_and_each_other():
    """Same (n, T): FD populations sit below, BE above the Maxwell-Juttner
    ones at low momentum (Pauli blocking / Bose enhancement)."""
    q = O.Quadrature(4, 16, 3)
    f = {s: q.feq(0.8, 1.0, stat=s) for s in (0, FD, BE)}
    m = {s: q.moments(f[s]) for s in f}
    assert m[FD][3] > m[0][3] > m[BE][3]     # eps = 2nT phi_2: larger for fermions at equal n, T
