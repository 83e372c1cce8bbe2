"""The accuracy study of Sec. 3.1 (Fig. 3) on the oracle alone, at a reduced
size: the error of the velocity profile (Eq. rel_err) against a run with
many more angles on a refined grid saturates at about 100 populations in
the near-hydrodynamic regime (Kn = 0.05) and keeps falling with the
population count in the near-ballistic one (Kn = 10), as Sec. 3.1 reports.

The run parameters restate the study's rules: Kn = tau / L on each grid,
comparison at 0.9 t_max with t_max = L / 2, time step 1 (tau > 2 here),
order 3 with Np = 4 shells, the paper's tube state clamped in x."""
import numpy as np

import oracle as O
import workloads as W


def oracle_beta(L, K, Kn):
    tau = Kn * L
    steps = int(round(0.9 * L / 2.0))
    sim = O.Sim(O.Quadrature(4, K, 3), L, 1, *W.tube(L, 1, 1.5, 1.5, 0.1, 0.5), tau=tau, dt=1.0, bcx=1, bcy=0)
    sim.step(steps)
    n, eps, ux, uy = sim.fields()
    g = np.sqrt(1.0 + ux * ux + uy * uy)
    return np.stack([ux / g, uy / g])


def oracle_tube_errors(L, refine, K_ref, Ks, Kn):
    """Eq. rel_err of each K against K_ref on the grid refined by `refine`,
    the reference averaged over the refine cells of each coarse cell."""
    ref = oracle_beta(L * refine, K_ref, Kn)
    ref = ref.reshape(2, 1, L, refine).mean(axis=3)
    return [float(np.linalg.norm(oracle_beta(L, K, Kn) - ref) / np.linalg.norm(ref)) for K in Ks]


def test_tube_error_saturates_only_in_the_hydrodynamic_regime():
    Ks = (8, 24, 96)                       # N_pop = 32, 96, 384
    lo = oracle_tube_errors(400, 2, 240, Ks, 0.05)
    hi = oracle_tube_errors(400, 2, 240, Ks, 10.0)
    assert lo[1] < 1.2 * lo[2]             # Kn 0.05: saturated by N_pop ~ 100
    assert lo[0] > 2 * lo[1]               # ... after falling from N_pop 32
    assert hi[0] > hi[1] > 2 * hi[2]       # Kn 10: still falling beyond 96
    assert hi[1] > 2 * lo[1]               # at N_pop 96 the ballistic regime is far from saturation
