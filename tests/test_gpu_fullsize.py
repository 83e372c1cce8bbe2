"""GPU parity at the benchmark sizes, on sampled sites.

The oracle cannot step a 1024^2 x 256 or 2048^2 x 1536 grid in a test, but
one step of the method at a site reads only the site and its upwind
neighbours (Eq. interpolation), and the collision is local.  So after t
steps a site depends only on the (2t + 1)^2 block around it.  The oracle
steps a block of half-width h > t cut from the initial fields (wrapped, as
the grid is periodic), with clamped edges.  The wrong values that the
clamped edges cause move inwards one ring per step and do not reach the
centre within t steps.  Its centre is then the exact result at the sampled
site, and the GPU run of the whole grid (in the configuration the benchmark
times) must match it there.

Tolerances as in test_gpu_parity: relative error per field <= 1e-12 for FP64
populations, <= 1e-4 for FP32.  At a sampled site n and eps are compared with
the oracle's value there; the flow vector with the largest oracle |u| among
the sampled sites (tests/fieldcheck.py), which include sites on the shock
fronts.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from fieldcheck import say, site_errors

pytestmark = pytest.mark.gpu

STEPS = 3
HALF = STEPS + 1


def _rlbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_06856_amd import rlbm
    rlbm.lib()
    return rlbm


def block(a, x, y, h):
    """The (2h + 1)^2 block of a periodic field centred on (x, y)."""
    ny, nx = a.shape
    rows = np.arange(y - h, y + h + 1) % ny
    cols = np.arange(x - h, x + h + 1) % nx
    return np.ascontiguousarray(a[np.ix_(rows, cols)])


def oracle_at(cfg, x, y):
    q = O.Quadrature(cfg["Np"], cfg["K"], cfg["N"])
    fld = [block(np.broadcast_to(f, (cfg["ny"], cfg["nx"])), x, y, HALF) for f in cfg["fields"]]
    w = 2 * HALF + 1
    sim = O.Sim(q, w, w, *fld, tau=cfg["tau"], dt=cfg["dt"], bcx=1, bcy=1)
    sim.step(STEPS)
    return [f[HALF, HALF] for f in sim.fields()]


def samples(nx, ny, extra, seed):
    """Tile edges, grid edges (the periodic wrap), the given sites and random ones."""
    pts = [(0, 0), (nx - 1, ny - 1), (63, 5), (64, 5), (nx - 64, ny // 2), (nx - 65, ny // 2 + 1)] + extra
    rng = np.random.default_rng(seed)
    pts += [(int(rng.integers(nx)), int(rng.integers(ny))) for _ in range(6)]
    return pts


def check_sites(rl, cfg, prec, tol, pts, label):
    import torch
    s = rl.Solver(cfg["Np"], cfg["K"], cfg["N"]).init_fields(cfg["nx"], cfg["ny"], *cfg["fields"], tau=cfg["tau"],
                                                              dt=cfg["dt"], precision=prec)
    say("case %s %s kernel=%s waves=%d" % (label, prec, s.get_kernel(), s.get_waves()))
    s.step(STEPS)
    n, eps, ux, uy, _ = s.moments()
    del s
    torch.cuda.empty_cache()
    refs = [oracle_at(cfg, x, y) for (x, y) in pts]
    uscale = max(np.hypot(r[2], r[3]) for r in refs)
    worst = 0.0
    for (x, y), ref in zip(pts, refs):
        e_n, e_eps, e_u = site_errors((n[y, x], eps[y, x], ux[y, x], uy[y, x]), ref, uscale)
        worst = max(worst, e_n, e_eps, e_u)
        assert e_n <= tol and e_eps <= tol and e_u <= tol, (label, prec, x, y, e_n, e_eps, e_u)
    say("%s %s: %d sites, worst relative error %.3e (flow scale %.3e)" % (label, prec, len(pts), worst, uscale))


@pytest.mark.parametrize("prec,tol", [("f32", 1e-4), ("f64", 1e-12)])
def test_circular_shock_full_size_sampled_sites(prec, tol):
    """1024^2, Np=4 x K=64, order 3, Kn=0.01: the headline workload and
    launch shape (tile kernel); sites on the disc edge among the samples."""
    rl = _rlbm()
    cfg = W.circular_shock(1024, Kn=0.01, steps=STEPS)
    pts = samples(1024, 1024, [(512 + 128, 512), (512, 512 - 128), (512 + 90, 512 + 91), (512, 512)], seed=3)
    check_sites(rl, cfg, prec, tol, pts, "circular_1024")


def test_quadrant_full_size_sampled_sites():
    """2048^2, Np=6 x K=256 (1536 velocities), order 5, Kn=10, FP32: the
    precision-form workload and launch shape (push kernel); sites at the
    quadrant boundaries among the samples."""
    rl = _rlbm()
    cfg = W.quadrant_shock(2048, steps=STEPS)
    pts = samples(2048, 2048, [(1023, 1024), (1024, 1023), (1024, 1024), (0, 1024), (1024, 2047)], seed=4)
    check_sites(rl, cfg, "f32", 1e-4, pts, "quadrant_2048")


def test_batch_full_size_sampled_sites():
    """The 48-problem batch (sides 128..1024, Kn 1e-3..10, K 48..128, FP32)
    in one launch per kernel per step: sampled sites of the two largest
    problems, one of each kernel, and one of the smallest."""
    import torch
    rl = _rlbm()
    probs = W.batch_problems(48, seed=0, steps=STEPS)
    b = rl.Batch(probs, precision="f32")
    say("case batch48 mode=%s waves=%d" % (b.get_mode(), b.get_waves()))
    b.step(STEPS)
    by_size = sorted(range(len(probs)), key=lambda i: probs[i]["nx"] * probs[i]["K"])
    tile = [i for i in by_size if 4 * probs[i]["K"] < 320]
    push = [i for i in by_size if 4 * probs[i]["K"] >= 320]
    pick = sorted({by_size[-1], by_size[-2], by_size[0]} | ({tile[-1]} if tile else set()) |
                  ({push[-1]} if push else set()))
    worst = 0.0
    for i in pick:
        p = probs[i]
        n, eps, ux, uy, _ = b.problem(i).moments()
        pts = samples(p["nx"], p["ny"], [(p["nx"] // 2 + p["nx"] // 8, p["ny"] // 2)], seed=10 + i)
        refs = [oracle_at(p, x, y) for (x, y) in pts]
        uscale = max(np.hypot(r[2], r[3]) for r in refs)
        for (x, y), ref in zip(pts, refs):
            e = max(site_errors((n[y, x], eps[y, x], ux[y, x], uy[y, x]), ref, uscale))
            worst = max(worst, e)
            assert e <= 1e-4, (i, p["nx"], p["K"], x, y, e)
    say("batch48: problems %s, worst relative error %.3e" % (pick, worst))
    del b
    torch.cuda.empty_cache()
