"""Pins of the oracle's wall and fixed boundaries (Sec. 4 names boundary
conditions as the method's next step; the readings are stated in the
oracle's stream pass): conservation at walls, the wall against its mirror
image in a periodic domain of twice the length, fixed edges against clamped
ones while no signal has reached them, rest states, and an arbitrary-
precision brute force on a tiny lattice."""
import numpy as np
import pytest

import oracle as O
import workloads as W

WALL, FIXED = 2, 3


def test_walls_conserve_mass_and_energy_but_not_momentum():
    q = O.Quadrature(4, 16, 3)
    nx, ny = 30, 20
    fld = W.paper_quadrant(nx, ny)
    sim = O.Sim(q, nx, ny, *fld, tau=3.0, dt=1.0, bcx=WALL, bcy=WALL)
    c0 = sim.charges()
    sim.step(150)
    c1 = sim.charges()
    assert sim.nonphys() == 0
    np.testing.assert_allclose(c1[:2], c0[:2], rtol=1e-12)
    assert abs(c1[2] - c0[2]) > 1e-6 or abs(c1[3] - c0[3]) > 1e-6   # the walls take up momentum


@pytest.mark.parametrize("tau", [np.inf, 8.0])
def test_wall_equals_its_mirror_image_in_a_periodic_domain(tau):
    """A tube of L cells between two walls against a periodic tube of 2L cells
    holding the state and its mirror image: with a velocity set symmetric
    under theta -> -theta (no shell rotation) a state symmetric in y stays so,
    and then the wall's reversal theta -> theta + pi equals the mirror's
    reflection theta -> pi - theta, so the two runs agree on the first L
    cells, also after the waves have reflected."""
    L, steps = 40, 100
    q = O.Quadrature(4, 32, 3, rotate=False)
    n, T, ux, uy = W.tube(L, 1, 1.5, 1.5, 0.1, 0.5)
    wall = O.Sim(q, L, 1, n, T, tau=tau, dt=1.0, bcx=WALL, bcy=0)
    mir = [np.concatenate([a, a[:, ::-1]], axis=1) for a in (n, T)]
    per = O.Sim(q, 2 * L, 1, *mir, tau=tau, dt=1.0, bcx=0, bcy=0)
    wall.step(steps)
    per.step(steps)
    a, b = wall.fields(), per.fields()
    for k in range(3):
        np.testing.assert_allclose(a[k], b[k][:, :L], rtol=1e-12, atol=1e-13)


def test_fixed_edges_equal_clamped_edges_until_the_waves_arrive():
    """Until a signal from the discontinuity reaches an edge (one cell per
    step), the edge cells hold their initial state, so a reservoir at that
    state (FIXED) and a zero-gradient edge (clamp) feed the same values."""
    q = O.Quadrature(3, 32, 3)
    nx = 120
    fld = W.tube(nx, 1)
    runs = {}
    for bc in (1, FIXED):
        s = O.Sim(q, nx, 1, *fld, tau=6.0, dt=1.0, bcx=bc, bcy=0)
        s.step(40)
        runs[bc] = s.fields()
    for k in range(3):
        np.testing.assert_allclose(runs[FIXED][k], runs[1][k], rtol=1e-13, atol=1e-14)
    for bc in (1, FIXED):   # later the reservoirs and the clamped edges differ
        s = O.Sim(q, nx, 1, *fld, tau=6.0, dt=1.0, bcx=bc, bcy=0)
        s.step(150)
        runs[bc] = s.fields()
    assert np.abs(runs[FIXED][0] - runs[1][0]).max() > 1e-4


@pytest.mark.parametrize("bc", [WALL, FIXED])
def test_uniform_rest_state_stays_at_rest_with_walls_and_reservoirs(bc):
    q = O.Quadrature(4, 24, 3)
    sim = O.Sim(q, 12, 9, 0.7, 1.3, tau=2.0, dt=1.0, bcx=bc, bcy=bc)
    f0 = sim.get_f()
    sim.step(30)
    np.testing.assert_allclose(sim.get_f(), f0, rtol=1e-13, atol=1e-16)


def test_reservoir_feeds_a_lower_density_grid():
    """A grid below the density of its FIXED edges fills up."""
    q = O.Quadrature(3, 16, 2)
    nx, ny = 20, 10
    n = np.full((ny, nx), 0.5)
    n[:, 0] = n[:, -1] = 1.0
    n[0, :] = n[-1, :] = 1.0
    sim = O.Sim(q, nx, ny, n, np.ones((ny, nx)), tau=2.0, dt=1.0, bcx=FIXED, bcy=FIXED)
    m0 = sim.charges()[0]
    sim.step(40)
    assert sim.charges()[0] > m0 * 1.05


def test_odd_angle_count_has_no_wall():
    q = O.Quadrature(3, 7, 2)
    with pytest.raises(ValueError):
        O.Sim(q, 4, 4, 1.0, 1.0, tau=1.0, bcx=WALL)


@pytest.mark.slow
def test_tiny_lattice_with_wall_and_fixed_edges_against_brute_force():
    """4 x 3 grid, Np=3, K=6, N=2, a wall across x and reservoirs across y,
    random moving state: oracle vs the 40-digit independent evaluation."""
    import mp_reference as MP
    nx, ny, steps = 4, 3, 5
    u = W.uniform(321, np.arange(4 * nx * ny)).reshape(4, ny, nx)
    fields = (0.5 + u[0], 0.7 + 0.6 * u[1], 0.4 * (u[2] - 0.5), 0.4 * (u[3] - 0.5))
    tau, dt = 2.0, 1.0
    ref = MP.Lattice(3, 6, 2, nx, ny, [a.tolist() for a in fields], tau, dt, bc=("wall", "fixed"))
    sim = O.Sim(O.Quadrature(3, 6, 2), nx, ny, *fields, tau=tau, dt=dt, bcx=WALL, bcy=FIXED)
    for s in range(steps):
        ref.step()
    sim.step(steps)
    got = sim.fields()
    exp = [np.array([[float(v) for v in row] for row in fld]) for fld in ref.fields()]
    for g_, e_ in zip(got, exp):
        np.testing.assert_allclose(g_, e_, rtol=1e-12, atol=1e-13)
