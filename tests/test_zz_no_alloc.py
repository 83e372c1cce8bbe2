"""rlbm_moments_device, the entry point that allocates nothing (its partial
charges live in the library's fixed device scratch), against rlbm_moments on
the same populations: the fields bit for bit (the same kernel), the charges
to 1e-13 of the largest charge (a device reduction in another order; the
momentum charges T^0x, T^0y nearly cancel and have no scale of their own).  Two calls in a
row, the second on a smaller grid, then the same call captured into a HIP
graph under torch's global capture mode, which rejects any allocation."""
import numpy as np
import pytest

import workloads as W
from fieldcheck import say

pytestmark = pytest.mark.gpu


def _rlbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_06856_amd import rlbm
    rlbm.lib()
    return rlbm


def assert_charges(got, ref):
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max(), (got, ref)


def _compare(rl, s, label):
    import torch
    n, eps, ux, uy, ch = s.moments()
    d_f = torch.full((4 * s.nx * s.ny,), 7.0, dtype=torch.float64, device="cuda")
    d_c = torch.full((4,), 7.0, dtype=torch.float64, device="cuda")
    s.moments_device(d_f, d_c)
    torch.cuda.synchronize()
    f = d_f.cpu().numpy().reshape(4, s.ny, s.nx)
    for k, ref in enumerate((n, eps, ux, uy)):
        assert np.array_equal(f[k], ref), (label, k)
    c = d_c.cpu().numpy()
    assert_charges(c, ch)
    say("%s: fields bitwise, charges %s" % (label, c))
    return d_f, d_c


def test_moments_device_matches_moments_on_two_calls():
    import torch
    rl = _rlbm()
    big = rl.Solver(4, 32, 3).init_fields(300, 70, *W.disc(300, 70, 20.0, seed=3), tau=4.0, precision="f32")
    big.step(6)
    _compare(rl, big, "first call 300x70")
    small = rl.Solver(3, 16, 2).init_fields(40, 9, *W.quadrant(40, 9, seed=8), tau=2.0, precision="f64")
    small.step(5)
    _compare(rl, small, "second call 40x9")
    # only the charges, then only the fields
    d_c = torch.zeros(4, dtype=torch.float64, device="cuda")
    small.moments_device(None, d_c)
    torch.cuda.synchronize()
    assert_charges(d_c.cpu().numpy(), small.moments()[4])


def test_moments_device_under_graph_capture():
    import torch
    rl = _rlbm()
    st = torch.cuda.Stream()
    s = rl.Solver(4, 24, 3).init_fields(150, 33, *W.quadrant(150, 33, seed=2), tau=3.0, precision="f32", stream=st)
    s.step(2)
    d_f = torch.zeros(4 * 150 * 33, dtype=torch.float64, device="cuda")
    d_c = torch.zeros(4, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        s.step(2)
        s.moments_device(d_f, d_c)
    for r in range(3):
        with torch.cuda.stream(st):
            g.replay()
        torch.cuda.synchronize()
        n, eps, ux, uy, ch = s.moments()
        f = d_f.cpu().numpy().reshape(4, 33, 150)
        assert np.array_equal(f[0], n) and np.array_equal(f[1], eps), r
        assert_charges(d_c.cpu().numpy(), ch)
        say("graph replay %d: moments_device matches moments" % r)


def test_moments_device_rejects_out_of_order_calls():
    rl = _rlbm()
    s = rl.Solver(3, 8, 2)
    with pytest.raises(rl.RlbmError):
        s.nx = s.ny = 1
        s.moments_device(None, None)
