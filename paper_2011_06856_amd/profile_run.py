"""Workload driver for rocprofv3 runs of the fused stream-and-collide kernel.

Runs `--steps` steps of the circular-shock workload (side^2 periodic grid,
Np=4 x K=64, order 3, Kn=0.01) or, with `--workload quadrant`, of the
quadrant Riemann problem (side^2, Np=6 x K=256, order 5, Kn=10) at the given
precision, or, with `--workload batch48`, of the 48-problem batch (FP32, one
graph replay per step; `--waves` sets its work-group shape, else the
library's default), or, with `--workload mlp`, `--steps` applications of the
learned form's readout network to a side^2 coarse run (64-128-128-128-4,
fused inference) and `--steps` training steps on 4096 rows (GEMMs, Adam),
then a device-to-device
copy of exactly `--copy-mib` MiB (read once, written once) whose FETCH_SIZE /
WRITE_SIZE readings calibrate the counters to bytes.

    rocprofv3 --kernel-trace --stats -d OUT -o run --output-format csv -- \
        python3 -m paper_2011_06856_amd.profile_run --steps 20
    rocprofv3 --pmc FETCH_SIZE ... (same command), then --pmc WRITE_SIZE
"""
import argparse
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def copy_calibration(mib):
    """One device copy of exactly `mib` MiB: read once, written once."""
    import torch
    n = mib * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--precision", default="f32")
    ap.add_argument("--side", type=int, default=1024)
    ap.add_argument("--Kn", type=float, default=0.01)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--workload", default="circular", choices=["circular", "quadrant", "batch48", "mlp"])
    ap.add_argument("--waves", type=int, default=0)
    a = ap.parse_args()
    import torch
    import workloads as W
    from paper_2011_06856_amd import rlbm
    if a.workload == "batch48":
        b = rlbm.Batch(W.batch_problems(48, seed=0, steps=a.steps), precision="f32")
        if a.waves:
            b.set_waves(a.waves)
        b.step(a.steps)
        torch.cuda.synchronize()
        what = "batch48 (mode %s, %d waves, %d site-velocity updates a step)" % (b.get_mode(), b.get_waves(), b.nsv)
        del b
        torch.cuda.empty_cache()
        copy_calibration(a.copy_mib)
        print("profile_run: %d steps of %s, then one %d MiB device copy" % (a.steps, what, a.copy_mib), flush=True)
        return
    if a.workload == "mlp":
        side = a.side
        cfg = W.circular_shock(side, Kn=1.0, steps=10)
        s = rlbm.Solver(4, 24, 3)
        s.init_fields(side, side, *cfg["fields"], tau=cfg["tau"], dt=cfg["dt"], precision="f32")
        s.step(10)
        net = rlbm.MLP(max_batch=side * side, out_dim=4)
        net.init_params(seed=1)
        # untrained weights: outputs scaled small, so that the corrected
        # fields stay physical
        net.set_norm(np.zeros(64), np.ones(64), np.zeros(4), np.full(4, 1e-4))
        for _ in range(a.steps):
            net.readout(s, 0.5)
        g = torch.Generator(device="cpu").manual_seed(0)
        X = torch.randn(4096, 64, generator=g).cuda()
        T = torch.randn(4096, 4, generator=g).cuda()
        for _ in range(a.steps):
            net.grad(X, T)
            net.adam_step()
        torch.cuda.synchronize()
        del net, s
        torch.cuda.empty_cache()
        copy_calibration(a.copy_mib)
        print("profile_run: %d readouts of a %d^2 coarse run and %d training steps of the readout network, then one "
              "%d MiB device copy" % (a.steps, side, a.steps, a.copy_mib), flush=True)
        return
    if a.workload == "circular":
        cfg = W.circular_shock(a.side, Kn=a.Kn, steps=a.steps)
    else:
        cfg = W.quadrant_shock(a.side, steps=a.steps)
    s = rlbm.Solver(cfg["Np"], cfg["K"], cfg["N"])
    s.init_fields(cfg["nx"], cfg["ny"], *cfg["fields"], tau=cfg["tau"], dt=cfg["dt"], precision=a.precision)
    if a.waves:
        s.set_waves(a.waves)
    s.step(a.steps)
    torch.cuda.synchronize()
    copy_calibration(a.copy_mib)
    print("profile_run: %d steps of %s (%s), then one %d MiB device copy" % (a.steps, cfg["name"], a.precision,
                                                                          a.copy_mib), flush=True)


if __name__ == "__main__":
    main()
