"""GPU tests of the C ABI's contract (include/rlbm.h) beyond the numerics:
the device Landau solve, re-initialisation of a context, and capture of
rlbm_step into a HIP graph (it allocates nothing and makes no synchronising
call, for both step kernels)."""
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


def test_device_landau_matches_the_oracle():
    """The kernels' Landau solve (rlbm_device_landau) on moments of
    equilibria and of perturbed states against the oracle's bisection; a
    state with no timelike eigenvector is flagged."""
    rl = _rlbm()
    q = O.Quadrature(4, 32, 3)
    rng = np.random.default_rng(21)
    moms = []
    for trial in range(40):
        f = q.feq(rng.uniform(0.2, 2.0), rng.uniform(0.5, 1.5), *rng.uniform(-0.8, 0.8, 2))
        if trial % 2:
            f = f * (1 + 0.2 * rng.uniform(-1, 1, size=q.nvel))
        moms.append(q.moments(f))
    moms.append([1, 0, 0, 1, 2, 0, 0.5, 0, 0.5])   # |T^0x| > T^00
    out = rl.device_landau(np.array(moms))
    for m, o in zip(moms[:-1], out[:-1]):
        ref, ok = O.landau(m)
        assert ok and o[6] == 1
        np.testing.assert_allclose(o[:6], ref[:6], rtol=1e-12, atol=1e-13)
    assert out[-1][6] == 0


def test_reinit_after_rejected_arguments_keeps_the_context():
    """A re-initialisation rejected in its argument checks changes nothing:
    the context keeps its fields and steps on as if the call had not been
    made.  A successful one on another grid replaces them."""
    rl = _rlbm()
    nx, ny = 70, 12
    fld = W.disc(nx, ny, 4.0, seed=2)
    a = rl.Solver(4, 24, 3).init_fields(nx, ny, *fld, tau=3.0, precision="f64")
    b = rl.Solver(4, 24, 3).init_fields(nx, ny, *fld, tau=3.0, precision="f64")
    for kern in ("tile", "push"):
        a.set_kernel(kern)
        b.set_kernel(kern)
        a.step(3)
        bad = np.array(fld[0])
        bad[1, 1] = -1.0
        with pytest.raises(rl.RlbmError):
            a.init_fields(nx, ny, bad, fld[1], tau=3.0, precision="f64")
        a.step(4)
        b.step(7)
        assert np.array_equal(a.get_populations(), b.get_populations()), kern
    small = W.quadrant(20, 6, seed=1)
    a.init_fields(20, 6, *small, tau=2.0, precision="f32")
    a.step(5)
    ref = O.Sim(O.Quadrature(4, 24, 3), 20, 6, *small, tau=2.0, dt=1.0)
    ref.step(5)
    check_fields(a.moments()[:4], ref.fields(), 1e-4, "reinit_other_grid")


@pytest.mark.parametrize("kernel,prec", [("tile", "f32"), ("push", "f32"), ("push", "bf16dev")])
def test_step_captured_in_a_graph_replays_like_eager_steps(kernel, prec):
    """rlbm_step(2) captured on the context's stream (torch's global capture
    mode rejects any allocation or synchronisation inside), replayed several
    times with eager work and synchronisations in between: every replay
    leaves the populations of the same steps issued eagerly, bit for bit
    (for bfloat16 deviations too: their stochastic rounding draws its random
    stream from the stored state)."""
    import torch
    rl = _rlbm()
    nx, ny = 130, 20
    fld = W.quadrant(nx, ny, seed=4)
    st = torch.cuda.Stream()
    g_run = rl.Solver(4, 48, 3).init_fields(nx, ny, *fld, tau=5.0, precision=prec, stream=st)
    g_run.set_kernel(kernel)
    ref = rl.Solver(4, 48, 3).init_fields(nx, ny, *fld, tau=5.0, precision=prec)
    ref.set_kernel(kernel)
    g_run.step(1)      # the push kernel's partial sums are built by an eager step
    ref.step(1)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=st):
        g_run.step(2)
    for r in range(4):
        with torch.cuda.stream(st):
            graph.replay()
        ref.step(2)
        x = torch.randn(1 << 16, device="cuda")          # eager work between replays
        torch.cuda.synchronize()
        assert float(x.abs().sum()) > 0
        say("graph %s %s replay %d" % (kernel, prec, r))
        assert np.array_equal(g_run.get_populations(), ref.get_populations()), (kernel, prec, r)
