"""GPU tests of the batched form: one persistent, graph-replayed launch per
step over many problems of uneven size, quadrature and Knudsen number.

Each problem of a batch must evolve exactly as when stepped alone with the
same work-group shape (same kernel body, same summation order): bitwise.
"""
import sys

import numpy as np
import pytest

import oracle as O
import workloads as W
from fieldcheck import check_fields

pytestmark = pytest.mark.gpu


def _rlbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2011_06856_amd import rlbm
    rlbm.lib()
    return rlbm


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def small_problems(seed=0, count=6):
    """Uneven problems: sides 40..150 (ragged tiles), K in {12, 16, 24, 28},
    Kn from 0.01 to 10, disc or quadrant states."""
    sides = [(150, 37), (64, 64), (97, 20), (40, 90), (128, 33), (70, 70), (33, 12), (120, 8)]
    Ks = [12, 16, 24, 28]
    out = []
    for i in range(count):
        u = W.uniform(seed, 8 * i + np.arange(4))
        nx, ny = sides[i % len(sides)]
        K = Ks[int(4 * u[0]) % 4]
        Kn = 10.0 ** (-2 + 3 * u[1])
        tau = W.tau_of(Kn, nx)
        fld = W.disc(nx, ny, min(nx, ny) / 6, seed=i) if u[2] < 0.5 else W.quadrant(nx, ny, seed=i)
        out.append(dict(Np=4, K=K, N=3, nx=nx, ny=ny, fields=fld, tau=tau, dt=W.dt_of(tau)))
    return out


@pytest.mark.parametrize("prec,mode", [("f32", "persistent"), ("f64", "persistent"), ("f32", "flat"), ("f64", "flat")])
def test_batch_problem_equals_single_run_bitwise(prec, mode):
    rl = _rlbm()
    probs = small_problems(1)
    b = rl.Batch(probs, precision=prec)
    b.set_mode(mode)
    assert b.get_mode() == mode
    waves = b.get_waves()
    say("batch %s %s waves=%d problems=%d" % (prec, mode, waves, len(b)))
    b.step(7)          # odd: graph pairs plus one eager step
    for i, p in enumerate(probs):
        s = rl.Solver(p["Np"], p["K"], p["N"]).init_fields(p["nx"], p["ny"], *p["fields"], tau=p["tau"],
                                                           dt=p["dt"], precision=prec)
        s.set_waves(waves)
        s.step(7)
        assert np.array_equal(b.problem(i).get_populations(), s.get_populations()), i
    b.step(4)
    for i in range(len(b)):
        b.problem(i).moments()   # finite, physical


def test_batch_fp64_matches_oracle():
    rl = _rlbm()
    probs = small_problems(2, count=3)
    b = rl.Batch(probs, precision="f64")
    b.step(12)
    for i, p in enumerate(probs):
        n, eps, ux, uy, _ = b.problem(i).moments()
        sim = O.Sim(O.Quadrature(p["Np"], p["K"], p["N"]), p["nx"], p["ny"], *p["fields"], tau=p["tau"], dt=p["dt"])
        sim.step(12)
        check_fields((n, eps, ux, uy), sim.fields(), 1e-12, "batch_fp64_%d" % i)


def test_graph_replays_match_eager_steps():
    """Replays of the captured graph, with eager work and synchronisations in
    between, give the populations of the same steps issued eagerly."""
    import torch
    rl = _rlbm()
    probs = small_problems(3, count=4)
    g = rl.Batch(probs)
    e = rl.Batch(probs)
    e.set_waves(g.get_waves())
    for rep in range(4):
        g.step(2)
        e.step_eager(2)
        torch.cuda.synchronize()
        x = torch.ones(1000, device="cuda").sum().item()   # unrelated eager work between replays
        assert x == 1000.0
        for i in range(len(g)):
            assert np.array_equal(g.problem(i).get_populations(), e.problem(i).get_populations()), (rep, i)


def test_autotune_keeps_state_and_picks_a_candidate(tmp_path):
    rl = _rlbm()
    probs = small_problems(4, count=4)
    b = rl.Batch(probs)
    b.step(3)
    before = [b.problem(i).get_populations().copy() for i in range(len(b))]
    cache = str(tmp_path / "tune.json")
    w, ms = b.autotune(candidates=(1, 2, 4), steps=4, cache=cache, key="test")
    assert w in (1, 2, 4) and ms > 0 and b.get_mode() in ("persistent", "flat")
    mode = b.get_mode()
    for i in range(len(b)):
        assert np.array_equal(b.problem(i).get_populations(), before[i])
    assert b.autotune(candidates=(1, 2, 4), cache=cache, key="test")[0] == w   # from the cache
    # stepping after tuning continues from the same state as an untuned batch
    ref = rl.Batch(probs)
    ref.step(3)
    ref.set_waves(w)
    ref.set_mode(mode)
    b.step(2)
    ref.step(2)
    for i in range(len(b)):
        assert np.array_equal(b.problem(i).get_populations(), ref.problem(i).get_populations())


def test_batch_with_push_kernel_problems_equals_single_runs_bitwise():
    """Problems with many velocities take the push kernel inside the batch
    (one extra flat launch per step); each still evolves exactly as when
    stepped alone, in both launch modes of the tile part."""
    rl = _rlbm()
    probs = small_problems(5, count=4)
    for i, K in ((1, 96), (3, 128)):        # 384 and 512 velocities: push kernel
        probs[i] = dict(probs[i], K=K)
    for prec in ("f32", "f64"):
        for mode in ("persistent", "flat"):
            b = rl.Batch(probs, precision=prec)
            b.set_mode(mode)
            waves = b.get_waves()
            say("batch+push %s %s waves=%d" % (prec, mode, waves))
            b.step(5)
            for i, p in enumerate(probs):
                s = rl.Solver(p["Np"], p["K"], p["N"]).init_fields(p["nx"], p["ny"], *p["fields"], tau=p["tau"],
                                                                   dt=p["dt"], precision=prec)
                assert s.get_kernel() == ("push" if p["K"] >= 96 else "tile")
                s.set_waves(waves)
                s.step(5)
                assert np.array_equal(b.problem(i).get_populations(), s.get_populations()), (prec, mode, i)


def _push_mix(seed):
    probs = small_problems(seed, count=4)
    for i, K in ((0, 96), (2, 112)):        # 384 and 448 velocities: push kernel
        probs[i] = dict(probs[i], K=K)
    return probs


def test_push_band_grouping_and_mode_changes_are_bitwise_neutral():
    """The band grouping of the push part only reorders work-groups, and the
    persistent launch leaves its work counters at zero: changing either
    between steps, and timing the first steps, leaves every problem on the
    trajectory it has when stepped alone."""
    rl = _rlbm()
    probs = _push_mix(6)
    b = rl.Batch(probs)
    assert b.get_push_bands() == 2
    b.set_push_bands(1)
    assert b.get_push_bands() == 1
    waves = b.get_waves()
    say("push bands: fresh batch, first call timed")
    assert b.step_timed(3) > 0           # the graph of the first call holds the push launch
    for bands, mode, n in ((8, "flat", 2), (3, "persistent", 3), (0, "persistent", 1), (4, "flat", 1)):
        say("push bands=%d mode=%s steps=%d" % (bands, mode, n))
        b.set_push_bands(bands)
        b.set_mode(mode)
        b.step(n)
    total = 3 + 2 + 3 + 1 + 1
    for i, p in enumerate(probs):
        s = rl.Solver(p["Np"], p["K"], p["N"]).init_fields(p["nx"], p["ny"], *p["fields"], tau=p["tau"],
                                                           dt=p["dt"], precision="f32")
        s.set_waves(waves)
        s.step(total)
        assert np.array_equal(b.problem(i).get_populations(), s.get_populations()), i


def test_autotune_with_push_problems_picks_bands_and_keeps_state():
    rl = _rlbm()
    probs = _push_mix(7)
    b = rl.Batch(probs)
    b.step(2)
    before = [b.problem(i).get_populations().copy() for i in range(len(b))]
    w, ms = b.autotune(candidates=(2, 4), steps=3)
    assert w in (2, 4) and ms > 0 and b.get_push_bands() in (1, 2, 4, 8)
    for i in range(len(b)):
        assert np.array_equal(b.problem(i).get_populations(), before[i]), i
    with pytest.raises(rl.RlbmError):
        b.set_push_bands(-1)
    with pytest.raises(rl.RlbmError):
        b.set_push_bands(65)
