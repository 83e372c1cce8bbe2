"""Accuracy studies of Sec. 3 on the built path: how the error of the
velocity field depends on the angle count K (and so N_pop = Np K) and on the
grid, across Knudsen numbers.

- tube_study (Sec. 3.1, Fig. 3): the tube of Sec. 3.1, (n, T) = (1.5, 1.5)
  left of the middle and (0.1, 0.5) right, at rest, L x 1 cells, clamped in
  x; order 3 (Np = 4 shells); error against a reference with K = 600
  (N_pop = 2400) on a grid refined by `refine`.
- convergence_study (Sec. 3.1, Fig. 4): the same tube at N_pop = 48, 240,
  480 over a range of grid sizes, against N_pop = 2400 on the finest grid.
- square_study (Sec. 3.2, Fig. 6): the 2D quadrant problem of Sec. 3.2 on
  L x L cells (clamped), against K = 600 on a grid refined by `refine`.
- fig5_study (Sec. 3.2, Fig. 5): that problem with K = 600 on 1000 x 1000
  against K = 12 on 500 x 500, at Kn = 0.002, 0.1 and 100.

The error is Eq. rel_err: || beta - beta_ref ||_2 / || beta_ref ||_2 with
beta = U / U^0 (both components in 2D), taken at t = 0.9 t_max, t_max = L / 2
(light-crossing time from the middle to the edge, in cells of the grid),
after averaging the reference over the cells of the coarser grid.  The
relaxation time follows Kn = tau / L on each grid.  The time step is
min(dt_max, tau / 2) with dt_max = 1, as in the benchmark workloads, except
in the hydrodynamic regime (Kn < 0.01), where dt_max = 0.5: at Kn = 0.002
and a time step of 1 the tube leaves the physical region (no timelike
Landau frame) within 50 to 200 steps on grids of 1000 cells and more, where
the axis-aligned velocities move exactly one cell per step with no
numerical diffusion to damp the shock; with 0.5 it runs through.  The step
counts keep the physical time equal across grids.

Everything runs through the library (rlbm.Solver); numpy only averages the
reference onto the coarse grid and takes norms.

    python -m paper_2011_06856_amd.studies [--quick] [--out results.json]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

NP = 4   # shells of the order-3 quadrature (N + 1)


def run(fields, nx, ny, K, Kn, precision="f64", bc=(1, 1), Np=NP, with_density=False):
    """Advance the state to t = 0.9 t_max and return beta = (bx, by) (and the
    density with `with_density`)."""
    from paper_2011_06856_amd import rlbm
    L = nx
    tau = W.tau_of(Kn, L)
    dt = min(1.0 if Kn >= 0.01 else 0.5, tau / 2.0)
    steps = int(round(0.9 * (L / 2.0) / dt))
    s = rlbm.Solver(Np, K, Np - 1)
    s.init_fields(nx, ny, *fields, tau=tau, dt=dt, bcx=bc[0], bcy=bc[1], precision=precision)
    s.step(steps)
    try:
        n, eps, ux, uy, _ = s.moments()
    except rlbm.NonPhysicalState:
        return None   # a site left the physical region (reported as NaN error)
    finally:
        del s
    g = np.sqrt(1.0 + ux * ux + uy * uy)
    beta = np.stack([ux / g, uy / g])
    return (beta, n[None]) if with_density else beta


def restrict(beta, r, two_d):
    """Average r (x r) blocks of a refined field onto the coarse grid."""
    if beta is None:
        return None
    c, ny, nx = beta.shape
    if two_d:
        return beta.reshape(c, ny // r, r, nx // r, r).mean(axis=(2, 4))
    return beta.reshape(c, ny, nx // r, r).mean(axis=3)


def rel_err(b, ref):
    if b is None or ref is None:
        return float("nan")
    return float(np.linalg.norm(b - ref) / np.linalg.norm(ref))


def saturation(npops, errs, tol=1.1):
    """Smallest N_pop whose error is within `tol` of the asymptotic error
    (the error at the largest N_pop of the sweep)."""
    e0 = errs[-1]
    for n, e in zip(npops, errs):
        if e == e and e <= tol * e0:
            return n
    return npops[-1]


def tube_study(Kns=(0.05, 0.5, 2.0, 10.0), Ks=(8, 12, 18, 24, 36, 48, 60, 75, 90, 120, 150, 200, 300), L=2000, refine=2,
               K_ref=600, precision="f64", log=print):
    out = {}
    for Kn in Kns:
        t0 = time.perf_counter()
        ref = restrict(run(W.tube(L * refine, 1, 1.5, 1.5, 0.1, 0.5), L * refine, 1, K_ref, Kn, precision,
                           bc=(1, 0)), refine, False)
        errs = [rel_err(run(W.tube(L, 1, 1.5, 1.5, 0.1, 0.5), L, 1, K, Kn, precision, bc=(1, 0)), ref) for K in Ks]
        npops = [NP * K for K in Ks]
        out[Kn] = dict(npop=npops, eps=errs, eps0=errs[-1], saturation_npop=saturation(npops, errs))
        log("tube Kn=%g: saturation N_pop %d, eps0 %.3g (%.1f s)" % (Kn, out[Kn]["saturation_npop"], errs[-1],
                                                                     time.perf_counter() - t0))
    return out


def convergence_study(Kns=(0.002, 0.1, 100.0), npops=(48, 240, 480), Ls=(500, 1000, 2000, 4000, 6000), L_ref=12000,
                      K_ref=600, precision="f64", log=print):
    out = {}
    for Kn in Kns:
        t0 = time.perf_counter()
        fine = run(W.tube(L_ref, 1, 1.5, 1.5, 0.1, 0.5), L_ref, 1, K_ref, Kn, precision, bc=(1, 0))
        rows = {}
        for npop in npops:
            K = npop // NP
            rows[npop] = [rel_err(run(W.tube(L, 1, 1.5, 1.5, 0.1, 0.5), L, 1, K, Kn, precision, bc=(1, 0)),
                                  restrict(fine, L_ref // L, False)) for L in Ls]
        out[Kn] = dict(L=list(Ls), eps={int(k): v for k, v in rows.items()})
        log("convergence Kn=%g (%.1f s): %s" % (Kn, time.perf_counter() - t0,
                                                "  ".join("Npop %d: %s" % (k, ["%.2g" % e for e in v])
                                                          for k, v in rows.items())))
    return out


def square_study(Kns=(0.05, 0.5, 2.0, 10.0), Ks=(8, 12, 18, 24, 36, 48, 60, 75, 90, 120), L=250, refine=4,
                 K_ref=600, precision="f32", log=print):
    out = {}
    for Kn in Kns:
        t0 = time.perf_counter()
        ref = restrict(run(W.paper_quadrant(L * refine, L * refine), L * refine, L * refine, K_ref, Kn, precision),
                       refine, True)
        errs = [rel_err(run(W.paper_quadrant(L, L), L, L, K, Kn, precision), ref) for K in Ks]
        npops = [NP * K for K in Ks]
        out[Kn] = dict(npop=npops, eps=errs, eps0=errs[-1], saturation_npop=saturation(npops, errs))
        log("square Kn=%g: saturation N_pop %d, eps0 %.3g (%.1f s)" % (Kn, out[Kn]["saturation_npop"], errs[-1],
                                                                       time.perf_counter() - t0))
    return out


def fig5_study(Kns=(0.002, 0.1, 100.0), L_fine=1000, K_fine=600, L_coarse=500, K_coarse=12, precision="f32",
               log=print):
    """Sec. 3.2, Fig. 5: the 2D quadrant problem at 0.9 t_max with K = 600 on
    1000 x 1000 and K = 12 on 500 x 500; the relative L2 differences of the
    density and of beta after averaging the fine solution onto the coarse
    grid.  The paper finds the two in agreement in the hydrodynamic regime
    and the coarse stencil's artefacts growing with Kn."""
    out = {}
    r = L_fine // L_coarse
    for Kn in Kns:
        t0 = time.perf_counter()
        fine = run(W.paper_quadrant(L_fine, L_fine), L_fine, L_fine, K_fine, Kn, precision, with_density=True)
        coarse = run(W.paper_quadrant(L_coarse, L_coarse), L_coarse, L_coarse, K_coarse, Kn, precision,
                     with_density=True)
        fb, fn = restrict(fine[0], r, True), restrict(fine[1], r, True)
        out[Kn] = dict(density=rel_err(coarse[1], fn), beta=rel_err(coarse[0], fb))
        log("fig5 Kn=%g: density %.3g beta %.3g (%.1f s)" % (Kn, out[Kn]["density"], out[Kn]["beta"],
                                                              time.perf_counter() - t0))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--quick", action="store_true", help="smaller grids and sweeps")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the studies run on the GPU"
    say = lambda m: print(m, flush=True)
    if a.quick:
        res = dict(tube=tube_study(Kns=(0.05, 10.0), Ks=(8, 24, 96), L=400, K_ref=240, log=say),
                   square=square_study(Kns=(0.05, 10.0), Ks=(8, 24, 96), L=64, refine=2, K_ref=240, log=say))
    else:
        res = dict(tube=tube_study(log=say), convergence=convergence_study(log=say), square=square_study(log=say),
                   fig5=fig5_study(log=say))
    if a.out:
        json.dump(res, open(a.out, "w"), indent=1, default=float)


if __name__ == "__main__":
    main()
