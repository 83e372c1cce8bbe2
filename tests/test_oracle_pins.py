"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None retypes the oracle's formulas:
the references are library routines (numpy's Gauss-Laguerre rule), textbook
identities (k! moments, orthogonality of harmonics), the paper's own relations
(equation of state, Landau decomposition, free-streaming solution of
Appendix A), independent numerical integration, and an arbitrary-precision
brute force on a tiny lattice.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ETA = np.diag([1.0, -1.0, -1.0])

CONFIG_QUADS = [(3, 32, 3), (4, 64, 3), (6, 256, 5), (4, 24, 3), (4, 384, 3),
                (4, 48, 3), (4, 96, 3), (4, 128, 3)]


def four_velocity(ux, uy):
    return np.array([math.sqrt(1 + ux * ux + uy * uy), ux, uy])


# --- Sec. 2.3: radial Gauss-Laguerre rule --------------------------------------------------

@pytest.mark.parametrize("Np", [1, 2, 3, 4, 5, 6, 8])
def test_shells_match_numpy_gauss_laguerre(Np):
    q = O.Quadrature(Np, 5, 0)
    x, wx = np.polynomial.laguerre.laggauss(Np)
    p = q.p.reshape(Np, 5)[:, 0]
    wr = q.w.reshape(Np, 5).sum(axis=1) / (2 * np.pi)
    np.testing.assert_allclose(p, x, rtol=1e-13)
    np.testing.assert_allclose(wr, wx, rtol=1e-12)


@pytest.mark.parametrize("Np", [2, 3, 4, 6])
def test_radial_rule_exact_to_degree_2Np_minus_1(Np):
    q = O.Quadrature(Np, 1, 0)
    for k in range(2 * Np):
        s = np.sum(q.w * q.p ** k) / (2 * np.pi)
        assert abs(s - math.factorial(k)) <= 1e-12 * math.factorial(k), k
    s = np.sum(q.w * q.p ** (2 * Np)) / (2 * np.pi)
    assert abs(s - math.factorial(2 * Np)) > 1e-6 * math.factorial(2 * Np)


@pytest.mark.parametrize("Np,K", [(3, 32), (4, 12), (4, 24), (6, 256)])
def test_angular_rule_exact_below_K(Np, K):
    q = O.Quadrature(Np, K, 3)
    th = q.theta.reshape(Np, K)
    for i in range(Np):
        for m in range(-K + 1, K):
            s = np.sum(np.exp(1j * m * th[i]))
            assert abs(s - (K if m == 0 else 0)) < 1e-11, (i, m)
        assert abs(abs(np.sum(np.exp(1j * K * th[i]))) - K) < 1e-9
    # rotated shells: offset i/Np of the angular spacing
    np.testing.assert_allclose(th[:, 0], np.arange(Np) / Np * 2 * np.pi / K, atol=1e-15)
    np.testing.assert_allclose(np.sum(q.w), 2 * np.pi, rtol=1e-14)
    np.testing.assert_allclose(np.hypot(q.cth, q.sth), 1.0, rtol=1e-15)


def test_paper_stencil_counts():
    g = json.load(open(os.path.join(HERE, "golden", "paper_states.json")))
    s = g["stencil_fig1"]
    assert O.Quadrature(s["order"] + 1, s["K"], s["order"]).nvel == s["N_pop"]
    for N, npop in g["product_rule"]["cases"]:
        assert O.Quadrature(N + 1, 2 * N + 1, N, rotate=False).nvel == npop


def test_paper_initial_states_obey_eos():
    """The printed initial states satisfy P = nT (eps = 2P = 2nT)."""
    g = json.load(open(os.path.join(HERE, "golden", "paper_states.json")))
    for side in ("left", "right"):
        st = g["tube_1d"][side]
        assert abs(st["P"] - st["n"] * st["T"]) < 1e-12
    for k, st in g["quadrant_2d"].items():
        if k.startswith("_"):
            continue
        assert abs(st["P"] - st["n"] * st["T"]) < 1e-12


# --- Eq. mj-orthogonal-conditions: orthonormality of the basis on the nodes -----------------

@pytest.mark.parametrize("Np,K,N", [(4, 64, 3), (3, 5, 2), (6, 256, 5), (4, 7, 3), (2, 3, 1)])
def test_basis_orthonormal_on_exact_quadratures(Np, K, N):
    q = O.Quadrature(Np, K, N)
    J, _ = q.basis()
    G = (J * q.w) @ J.T
    np.testing.assert_allclose(G, np.eye(q.nb), atol=1e-12)


def test_basis_not_orthonormal_when_radial_rule_too_short():
    """Np = N shells cannot integrate degree 2N radially (N+1 shells needed)."""
    q = O.Quadrature(3, 32, 3)
    J, _ = q.basis()
    G = (J * q.w) @ J.T
    assert np.abs(G - np.eye(q.nb)).max() > 0.1


def test_basis_spans_light_cone_polynomials():
    """The (N+1)^2 basis functions are independent and each is a polynomial of
    degree <= N: a rich enough rule reproduces any such polynomial exactly."""
    q = O.Quadrature(6, 40, 4)
    J, ex = q.basis()
    assert np.linalg.matrix_rank(J) == q.nb == 25
    rng = np.random.default_rng(1)
    c = rng.normal(size=(3,))
    poly = 1 + c[0] * q.p * q.cth + c[1] * q.p ** 2 * q.sth * q.cth + c[2] * q.p ** 4 * q.cth ** 3 * q.sth
    coef = (J * q.w) @ poly
    np.testing.assert_allclose(coef @ J, poly, rtol=0, atol=1e-9 * np.abs(poly).max())


# --- Sec. 2.1: Maxwell-Juttner moments --------------------------------------------------------

def _numeric_mj_moment(idx, n, T, U, M=2048):
    """int f_eq p^idx dtheta dp with the radial integral done analytically,
    int_0^inf p^k e^{-pA/T} dp = k! (T/A)^{k+1}, and a periodic trapezoid in angle."""
    th = 2 * np.pi * np.arange(M) / M
    comps = [np.ones(M), np.cos(th), np.sin(th)]
    k = len(idx)
    prod = np.ones(M)
    for i in idx:
        prod = prod * comps[i]
    A = U[0] - U[1] * np.cos(th) - U[2] * np.sin(th)
    rad = math.factorial(k) * (T / A) ** (k + 1)
    return n / (2 * np.pi * T * T) * np.sum(prod * rad) * 2 * np.pi / M


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5])
def test_mj_moment_tensor_matches_numerical_integration(k):
    rng = np.random.default_rng(k)
    for trial in range(6):
        n, T = rng.uniform(0.2, 2.0), rng.uniform(0.4, 2.0)
        ux, uy = rng.uniform(-0.8, 0.8, size=2)
        U = four_velocity(ux, uy)
        idx = rng.integers(0, 3, size=k)
        ref = _numeric_mj_moment(idx, n, T, U)
        got = O.mj_moment(idx, n, T, ux, uy)
        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (k, idx, got, ref)


def test_mj_low_moments_are_the_ideal_fluid():
    """N^mu = n U^mu and T^{mu nu} = (eps + P) U U - P eta with eps = 2P = 2nT
    (Eq. ll-decomp without dissipative terms, and the ideal EOS)."""
    n, T, ux, uy = 0.8, 1.3, 0.4, -0.25
    U = four_velocity(ux, uy)
    for a in range(3):
        assert abs(O.mj_moment([a], n, T, ux, uy) - n * U[a]) < 1e-14
        for b in range(3):
            P = n * T
            ref = 3 * P * U[a] * U[b] - P * ETA[a, b]
            assert abs(O.mj_moment([a, b], n, T, ux, uy) - ref) < 1e-13


# --- Eq. mj-feq-expansion-truncated: the discrete equilibrium ---------------------------------

@pytest.mark.parametrize("Np,K,N", CONFIG_QUADS)
def test_discrete_feq_reproduces_Nmu_Tmunu(Np, K, N):
    q = O.Quadrature(Np, K, N)
    rng = np.random.default_rng(Np * 1000 + K)
    for trial in range(4):
        n, T = rng.uniform(0.2, 1.5), rng.uniform(0.5, 1.5)
        ux, uy = rng.uniform(-0.5, 0.5, size=2)
        U = four_velocity(ux, uy)
        m = q.moments(q.feq(n, T, ux, uy))
        np.testing.assert_allclose(m[:3], n * U, rtol=1e-12, atol=1e-13)
        Tm = n * T * (3 * np.outer(U, U) - ETA)
        np.testing.assert_allclose(m[3:], Tm[np.triu_indices(3)], rtol=1e-12, atol=1e-13)


def _disc_rank_k(q, f, idx):
    comps = [q.p, q.p * q.cth, q.p * q.sth]
    prod = np.ones(q.nvel)
    for i in idx:
        prod = prod * comps[i]
    return np.sum(prod * f)


def test_rank3_exactness_depends_on_angular_order():
    """Rank-k moments of the discrete f_eq are exact when k + N <= K - 1
    (angular) and k + N <= 2Np - 1 (radial); N = 3, Np = 4: K = 7 exact, K = 6 not."""
    n, T, ux, uy = 0.9, 1.1, 0.35, 0.2
    idx = [1, 1, 2]
    ref = O.mj_moment(idx, n, T, ux, uy)
    q7 = O.Quadrature(4, 7, 3)
    assert abs(_disc_rank_k(q7, q7.feq(n, T, ux, uy), idx) - ref) < 1e-12
    q6 = O.Quadrature(4, 6, 3)
    assert abs(_disc_rank_k(q6, q6.feq(n, T, ux, uy), idx) - ref) > 1e-6


def test_feq_at_rest_with_weighting_temperature():
    """At rest with T = T0 = 1 the equilibrium equals n omega / (2 pi): f_v = w_v n / (2 pi)."""
    q = O.Quadrature(4, 64, 3)
    np.testing.assert_allclose(q.feq(0.7, 1.0), q.w * 0.7 / (2 * np.pi), rtol=1e-13)


def test_feq_is_not_clamped():
    """Far from T0 the truncated expansion goes negative; it is used as is."""
    q = O.Quadrature(4, 64, 3)
    f = q.feq(1.0, 0.5) / q.w
    assert f.min() < -0.1 * f.max()


# --- Landau frame (eigenvalue problem of Sec. 2.2, EOS eps = 2nT) -----------------------------

def test_landau_recovers_equilibrium_fields():
    q = O.Quadrature(4, 64, 3)
    rng = np.random.default_rng(7)
    for trial in range(20):
        n, T = rng.uniform(0.1, 2.0), rng.uniform(0.5, 1.5)
        ux, uy = rng.uniform(-1.0, 1.0, size=2)
        m = q.moments(q.feq(n, T, ux, uy))
        out, ok = O.landau(m)
        assert ok
        np.testing.assert_allclose(out[:5], [n, 2 * n * T, ux, uy, T], rtol=1e-12, atol=1e-13)
        # eigenvalues of T^mu_nu: (2nT, -nT, -nT)
        Tm = np.array([[m[3], m[4], m[5]], [m[4], m[6], m[7]], [m[5], m[7], m[8]]])
        ev = np.sort(np.linalg.eigvals(Tm @ ETA).real)
        np.testing.assert_allclose(ev, [-n * T, -n * T, 2 * n * T], rtol=1e-11, atol=1e-12)


def test_landau_on_non_equilibrium_states():
    """eps U = T U_lower for states with shear and heat flux; U.U = 1."""
    q = O.Quadrature(4, 32, 3)
    rng = np.random.default_rng(3)
    for trial in range(20):
        f = q.feq(rng.uniform(0.5, 1), rng.uniform(0.7, 1.2), *rng.uniform(-0.4, 0.4, 2))
        f = f * (1 + 0.2 * rng.uniform(-1, 1, size=q.nvel))
        m = q.moments(f)
        out, ok = O.landau(m)
        assert ok
        n, eps, ux, uy, T, U0 = out
        U = np.array([U0, ux, uy])
        Tm = np.array([[m[3], m[4], m[5]], [m[4], m[6], m[7]], [m[5], m[7], m[8]]])
        np.testing.assert_allclose(Tm @ ETA @ U, eps * U, rtol=1e-12, atol=1e-13)
        assert abs(U @ ETA @ U - 1) < 1e-13
        assert abs(n - U @ ETA @ m[:3]) < 1e-13
        ev = np.linalg.eigvals(Tm @ ETA).real
        assert abs(eps - ev.max()) < 1e-12 * eps


def test_landau_1d_closed_form_agrees():
    N0, Nx, T00, T0x, Txx = 1.2, 0.3, 2.5, 0.6, 1.0
    Tyy = T00 - Txx
    eps, beta, n = O.landau_1d(N0, Nx, T00, T0x, Txx)
    out, ok = O.landau([N0, Nx, 0, T00, T0x, 0, Txx, 0, Tyy])
    assert ok
    g = 1 / math.sqrt(1 - beta * beta)
    np.testing.assert_allclose([out[1], out[2], out[0]], [eps, g * beta, n], rtol=1e-13)


def test_landau_flags_non_physical_state():
    out, ok = O.landau([0, 0, 0, 0, 0, 0, 0, 0, 0])
    assert not ok
    out, ok = O.landau([1, 0, 0, 1, 2, 0, 0.5, 0, 0.5])   # |T^0x| > T^00: no timelike vector
    assert not ok


# --- Eq. ll-decomp: shear stress of the Landau-Lifshitz decomposition (site_stats) ----------

def _boost(ux, uy):
    """Lorentz boost Lambda^mu_nu taking the rest frame to four-velocity U."""
    U = four_velocity(ux, uy)
    g = U[0]
    L = np.eye(3)
    L[0, 0] = g
    L[0, 1:] = L[1:, 0] = U[1:]
    u2 = ux * ux + uy * uy
    if u2 > 0:
        L[1:, 1:] += (g - 1.0) * np.outer(U[1:], U[1:]) / u2
    return L


def test_site_stats_shear_vanishes_for_equilibria():
    """f = f_eq(n, T, U) is an ideal fluid, T = (eps + P) U U - P eta: its
    shear stress is zero, at rest and moving (Eq. ll-decomp)."""
    q = O.Quadrature(4, 64, 3)
    rng = np.random.default_rng(11)
    for trial in range(12):
        n, T = rng.uniform(0.2, 2.0), rng.uniform(0.5, 1.5)
        ux, uy = (0.0, 0.0) if trial == 0 else rng.uniform(-0.8, 0.8, size=2)
        st = O.site_stats(q.moments(q.feq(n, T, ux, uy)))
        np.testing.assert_allclose(st[:4], [n, 2 * n * T, ux, uy], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(st[4:], 0.0, atol=1e-12 * n * T)


def test_site_stats_recovers_a_prescribed_shear_stress():
    """Build T^{mu nu} = (eps + P) U U - P eta + pi from a traceless spatial
    shear stress given in the rest frame and boosted to U (so that pi U = 0),
    with N^mu = n U^mu; the decomposition must return n, eps, U and the lab
    frame's pi^{ij}.  A wrong enthalpy, pressure sign or index order fails
    for moving frames."""
    rng = np.random.default_rng(5)
    for trial in range(16):
        n, eps = rng.uniform(0.3, 2.0), rng.uniform(0.5, 3.0)
        ux, uy = rng.uniform(-0.7, 0.7, size=2)
        a, b = rng.uniform(-0.1, 0.1, size=2) * eps
        pi_rest = np.array([[0.0, 0.0, 0.0], [0.0, a, b], [0.0, b, -a]])
        L = _boost(ux, uy)
        pi = L @ pi_rest @ L.T
        U = four_velocity(ux, uy)
        P = eps / 2.0
        Tmn = (eps + P) * np.outer(U, U) - P * np.linalg.inv(ETA) + pi
        assert np.allclose(pi @ ETA @ U, 0.0, atol=1e-14)             # orthogonal to U
        assert abs(np.trace(ETA @ pi)) < 1e-14                          # traceless
        N = n * U
        mom = [N[0], N[1], N[2], Tmn[0, 0], Tmn[0, 1], Tmn[0, 2], Tmn[1, 1], Tmn[1, 2], Tmn[2, 2]]
        st = O.site_stats(mom)
        assert st is not None
        np.testing.assert_allclose(st[:4], [n, eps, ux, uy], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(st[4:], [pi[1, 1], pi[1, 2], pi[2, 2]], atol=1e-12 * eps)


# --- Eq. collision: conservation, equilibrium, relaxation rate --------------------------------

def test_collision_conserves_charges_per_site():
    """On a 1x1 periodic lattice streaming is the identity, so one step is one
    collision: N^0, T^00, T^0x, T^0y are conserved and the shear relaxes."""
    q = O.Quadrature(4, 32, 3)
    rng = np.random.default_rng(11)
    for trial in range(5):
        sim = O.Sim(q, 1, 1, 0.8, 1.1, 0.2, -0.1, tau=3.0, dt=1.0)
        f = sim.get_f() * (1 + 0.3 * rng.uniform(-1, 1, size=(q.nvel, 1, 1)))
        sim.set_f(f)
        m0 = sim.moments()[:, 0, 0]
        sim.step(1)
        m1 = sim.moments()[:, 0, 0]
        for k in (0, 3, 4, 5):
            assert abs(m1[k] - m0[k]) < 1e-14 * max(1, abs(m0[k])), k
        assert np.abs(m1[6] - m0[6]) > 1e-6


def test_relaxation_rate_at_rest():
    """A shear perturbation w_v cos(2 theta_v) carries no N^mu or T^{0 mu}, so
    the fluid stays at rest, f_eq is unchanged and, with p.U / p^0 = 1,
    f - f_eq decays exactly as (1 - dt/tau)^t (Eq. discrete-rbe)."""
    q = O.Quadrature(4, 32, 3)
    tau, dt = 5.0, 1.0
    sim = O.Sim(q, 1, 1, 1.0, 1.0, tau=tau, dt=dt)
    feq = sim.get_f()
    delta = 0.05 * (q.w * np.cos(2 * q.theta)).reshape(q.nvel, 1, 1)
    sim.set_f(feq + delta)
    for t in range(1, 6):
        sim.step(1)
        np.testing.assert_allclose(sim.get_f() - feq, delta * (1 - dt / tau) ** t, atol=1e-15)


def test_uniform_fluid_at_rest_stays_at_rest():
    q = O.Quadrature(4, 32, 3)
    sim = O.Sim(q, 6, 5, 0.7, 1.3, tau=2.0, dt=1.0)
    f0 = sim.get_f()
    sim.step(20)
    np.testing.assert_allclose(sim.get_f(), f0, rtol=1e-13, atol=1e-16)
    n, eps, ux, uy = sim.fields()
    assert np.abs(ux).max() < 1e-14 and np.abs(uy).max() < 1e-14
    np.testing.assert_allclose(n, 0.7, rtol=1e-13)
    np.testing.assert_allclose(eps, 2 * 0.7 * 1.3, rtol=1e-13)


def test_global_charges_conserved_on_periodic_grid():
    q = O.Quadrature(4, 16, 3)
    fld = W.disc(24, 20, 5.0, seed=2)
    sim = O.Sim(q, 24, 20, *fld, tau=3.0, dt=1.0)
    c0 = sim.charges()
    sim.step(100)
    c1 = sim.charges()
    np.testing.assert_allclose(c1[:2], c0[:2], rtol=1e-12)
    assert np.abs(c1[2:]).max() < 1e-11
    assert sim.nonphys() == 0


# --- Eq. streaming / Eq. interpolation ----------------------------------------------------------

def test_stream_only_is_binomial_tensor_product():
    """t steps of bilinear upwind streaming equal a tensor product of binomial
    distributions of the shifts: weights C(t,k) a^k (1-a)^(t-k) per axis."""
    q = O.Quadrature(2, 5, 1)
    nx, ny, t = 9, 7, 4
    rng = np.random.default_rng(5)
    sim = O.Sim(q, nx, ny, 1.0, 1.0)
    f0 = rng.uniform(0.1, 1.0, size=(q.nvel, ny, nx))
    sim.set_f(f0)
    sim.stream(t)
    got = sim.get_f()
    for v in range(q.nvel):
        ax, ay = abs(q.cth[v]), abs(q.sth[v])
        sx = 1 if q.cth[v] >= 0 else -1
        sy = 1 if q.sth[v] >= 0 else -1
        ref = np.zeros((ny, nx))
        for k in range(t + 1):
            for l in range(t + 1):
                wgt = math.comb(t, k) * ax ** k * (1 - ax) ** (t - k) * math.comb(t, l) * ay ** l * (1 - ay) ** (t - l)
                ref += wgt * np.roll(np.roll(f0[v], k * sx, axis=1), l * sy, axis=0)
        np.testing.assert_allclose(got[v], ref, rtol=1e-13)


def test_stream_axis_velocity_is_exact_shift_and_mass_conserved():
    q = O.Quadrature(3, 8, 2)
    nx, ny = 11, 6
    rng = np.random.default_rng(9)
    sim = O.Sim(q, nx, ny, 1.0, 1.0)
    f0 = rng.uniform(size=(q.nvel, ny, nx))
    sim.set_f(f0)
    sim.stream(3)
    f = sim.get_f()
    # v = 0: shell 0, theta = 0 -> shift by +3 cells in x exactly
    np.testing.assert_allclose(f[0], np.roll(f0[0], 3, axis=1), rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(f.sum(axis=(1, 2)), f0.sum(axis=(1, 2)), rtol=1e-13)


def test_clamp_boundary_keeps_uniform_state():
    q = O.Quadrature(3, 32, 3)
    sim = O.Sim(q, 10, 1, 0.4, 0.9, tau=np.inf, dt=1.0, bcx=1, bcy=0)
    f0 = sim.get_f()
    sim.step(5)
    np.testing.assert_allclose(sim.get_f(), f0, rtol=1e-14)


# --- Appendix A: free streaming of the shock tube -----------------------------------------------

def test_closed_form_reduces_to_the_initial_states_outside_the_fan():
    nL, TL, nR, TR = 1.5, 1.5, 0.1, 0.5
    N0, Nx, T00, T0x, Txx, Tyy = O.free_streaming_tube(np.array([-1.0, 1.0]), nL, TL, nR, TR)
    # w = -1: nothing from the right has arrived; w = +1: everything has
    np.testing.assert_allclose([N0[0], T00[0], Txx[0], Tyy[0]], [nL, 2 * nL * TL, nL * TL, nL * TL], rtol=1e-14)
    np.testing.assert_allclose([N0[1], T00[1], Txx[1], Tyy[1]], [nR, 2 * nR * TR, nR * TR, nR * TR], rtol=1e-14)
    w = np.linspace(-1, 1, 41)
    N0, Nx, T00, T0x, Txx, Tyy = O.free_streaming_tube(w, nL, TL, nR, TR)
    np.testing.assert_allclose(T00, Txx + Tyy, rtol=1e-14)


def test_closed_form_matches_direct_integration_of_the_distribution():
    """Appendix A's integrals redone numerically from f = f_L + theta(w - v_x)(f_R - f_L)."""
    nL, TL, nR, TR = 1.5, 1.5, 0.1, 0.5
    M = 200000
    a = (np.arange(M) + 0.5) * 2 * np.pi / M
    for w in (-0.7, -0.1, 0.3, 0.9):
        right = np.cos(a) < w
        # radial integrals of the rest-frame MJ: int p f dp = n/2pi, int p^2 f dp = nT/pi
        r1 = np.where(right, nR, nL) / (2 * np.pi)
        r2 = np.where(right, nR * TR, nL * TL) / np.pi
        d = 2 * np.pi / M
        ref = [np.sum(r1) * d, np.sum(r1 * np.cos(a)) * d, np.sum(r2) * d,
               np.sum(r2 * np.cos(a)) * d, np.sum(r2 * np.cos(a) ** 2) * d, np.sum(r2 * np.sin(a) ** 2) * d]
        got = O.free_streaming_tube(np.array([w]), nL, TL, nR, TR)
        np.testing.assert_allclose([g[0] for g in got], ref, rtol=2e-4, atol=2e-5)


@pytest.mark.slow
def test_free_streaming_tube_against_closed_form():
    """Fig. 2 setting: 2000 x 1 tube, tau -> inf, t = 0.9 t_max = 900 steps,
    the initial state of Sec. 3.1.  Third order with K = 120 reproduces the
    analytic profile (relative L2 error of beta at the 1e-3 level, the size of
    the asymptotic errors the paper quotes); K = 12 is much worse."""
    g = json.load(open(os.path.join(HERE, "golden", "paper_states.json")))["tube_1d"]
    nL, TL, nR, TR = g["left"]["n"], g["left"]["T"], g["right"]["n"], g["right"]["T"]
    nx, t = 2000, 900
    xc = np.arange(nx) + 0.5 - nx / 2
    N0, Nx, T00, T0x, Txx, Tyy = O.free_streaming_tube(xc / t, nL, TL, nR, TR)
    eps_ref, beta_ref, n_ref = O.landau_1d(N0, Nx, T00, T0x, Txx)
    errs = {}
    for K in (120, 12):
        q = O.Quadrature(4, K, 3)
        fld = W.tube(nx, 1, nL, TL, nR, TR)
        sim = O.Sim(q, nx, 1, *fld, tau=np.inf, dt=1.0, bcx=1, bcy=0)
        sim.step(t)
        n, eps, ux, uy = (a[0] for a in sim.fields())
        beta = ux / np.sqrt(1 + ux * ux + uy * uy)
        errs[K] = (O.rel_l2(beta, beta_ref), O.rel_l2(n, n_ref), O.rel_l2(eps, eps_ref))
        if K == 120:
            # rotated shells are not mirror-symmetric in y, so a small
            # transverse flow is a property of the discretisation, not zero
            assert np.abs(uy).max() < 0.01 * np.abs(ux).max()
    assert errs[120][0] < 3e-3, errs
    assert errs[120][1] < 2e-3 and errs[120][2] < 2e-3, errs
    assert errs[12][0] > 3 * errs[120][0], errs


# --- Brute force on a tiny lattice --------------------------------------------------------------

@pytest.mark.slow
def test_tiny_lattice_against_arbitrary_precision_brute_force():
    """4 x 3 periodic grid, Np=3, K=5, N=2 (the smallest exact set), random
    moving states, finite tau: oracle vs a 40-digit independent evaluation."""
    import mp_reference as MP
    nx, ny, steps = 4, 3, 6
    u = W.uniform(123, np.arange(4 * nx * ny)).reshape(4, ny, nx)
    fields = (0.5 + u[0], 0.7 + 0.6 * u[1], 0.4 * (u[2] - 0.5), 0.4 * (u[3] - 0.5))
    tau, dt = 2.5, 1.0
    ref = MP.Lattice(3, 5, 2, nx, ny, [a.tolist() for a in fields], tau, dt)
    q = O.Quadrature(3, 5, 2)
    sim = O.Sim(q, nx, ny, *fields, tau=tau, dt=dt)
    f_or = sim.get_f()
    f_mp = np.array([[[float(ref.f[(v, y, x)]) for x in range(nx)] for y in range(ny)] for v in range(q.nvel)])
    np.testing.assert_allclose(f_or, f_mp, rtol=1e-13, atol=1e-15)
    for s in range(steps):
        ref.step()
    sim.step(steps)
    got = sim.fields()
    exp = [np.array([[float(v) for v in row] for row in fld]) for fld in ref.fields()]
    for g_, e_ in zip(got, exp):
        np.testing.assert_allclose(g_, e_, rtol=1e-12, atol=1e-13)
