"""Benchmark of the fused stream-and-collide step on one MI355X.

Workload: the circular shock at 1024 x 1024 (periodic), Np = 4 radial shells x
K = 64 angles (256 velocities), equilibrium order 3, FP32 populations, disc of
radius 128 (n=1, T=1.5) in a background (n=0.5, T=1) with 1% seeded noise on
n; two runs, Kn = 0.01 and Kn = 1.  A step is one fused stream-and-collide
launch over the whole grid; the timed region holds `--steps` steps of each run
with the populations already resident in HBM.

Prints one JSON line with the throughput in site-velocity updates per second
(GSVUPS), the roofline of the fused kernel (algorithmic bytes / launch time
from HIP events on the library's stream, against the 8 TB/s HBM peak) and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
METRIC = "GSVUPS + % HBM roofline; coarse-angle+MLP vs fine-angle speedup at equal error"
BYTES_PER_SV = {"f32": 8, "f64": 16}


def counter_traffic(name):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    profiles/<name>.json, or None if absent or taken on other sources."""
    path = os.path.join(ROOT, "profiles", name + ".json")
    if not os.path.exists(path):
        return None
    from paper_2011_06856_amd.profile_summary import kernel_source_hash
    d = json.load(open(path))
    if d.get("kernel_sha256") != kernel_source_hash():
        return None
    return d.get("traffic_bytes")


def gpu_run(cfg, steps, warmup, precision, waves, keep_fields=False):
    import torch
    from paper_2011_06856_amd import rlbm
    s = rlbm.Solver(cfg["Np"], cfg["K"], cfg["N"])
    s.init_fields(cfg["nx"], cfg["ny"], *cfg["fields"], tau=cfg["tau"], dt=cfg["dt"], precision=precision)
    if waves:
        s.set_waves(waves)
    s.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_events = s.step_timed(steps)   # HIP events on the library's stream around the launches
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n, eps, ux, uy, ch = s.moments()
    ok = bool(np.isfinite(n).all() and np.isfinite(eps).all())
    out = dict(wall_s=wall, event_ms=ms_events, sv=float(cfg["nx"] * cfg["ny"] * s.nvel * steps),
               waves=s.get_waves(), kernel=s.get_kernel(), finite=ok, charges=ch.tolist())
    if keep_fields:
        out["fields"] = (n, eps, ux, uy)
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s):
    """The FP64 oracle on a bounded sample: the same quadrature and state on a
    256 x 256 grid (Kn = 0.01 with tau scaled to the side), steps sized to the
    budget after one timed probe step; once on all the host threads OpenMP
    gets, then on one (with a third of the budget)."""
    import oracle as O
    side = 256
    cfg = W.circular_shock(side, Kn=0.01, steps=1)
    q = O.Quadrature(cfg["Np"], cfg["K"], cfg["N"])

    def leg(budget):
        sim = O.Sim(q, side, side, *cfg["fields"], tau=cfg["tau"], dt=cfg["dt"])
        t0 = time.perf_counter()
        sim.step(1)
        probe = time.perf_counter() - t0
        nsteps = max(1, int(budget / max(probe, 1e-3)))
        t0 = time.perf_counter()
        sim.step(nsteps)
        dt = time.perf_counter() - t0
        return side * side * q.nvel * nsteps / dt / 1e9, nsteps

    cores = O.num_threads()
    v_all, n_all = leg(budget_s)
    O.set_threads(1)
    v_one, n_one = leg(budget_s / 3.0)
    O.set_threads(cores)
    sample = "%dx%d grid, Np=4 x K=64 (256 velocities), order 3, Kn=0.01, FP64" % (side, side)
    return dict(value=v_all, unit="GSVUPS", cores=cores, kind="oracle",
                sample="%s, %d steps" % (sample, n_all), cpu_model=cpu_model(), host_threads=os.cpu_count(),
                single_core={"value": v_one, "unit": "GSVUPS", "cores": 1, "sample": "%s, %d steps" % (sample, n_one)})


def copy_bandwidth(nbytes=2 << 30, iters=10):
    """Device-to-device copy rate on this GPU, measured in the same run: torch's
    copy of nbytes between two HBM buffers, bytes read plus bytes written per
    second (GB/s), the best of `iters` event-timed copies."""
    import torch
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    b.copy_(a)
    best = None
    for _ in range(iters):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * nbytes / (best * 1e-3) / 1e9


def batched_form(a):
    """Batched form: 48 independent shock problems of uneven side (128..1024),
    Knudsen number (1e-3..10, log-uniform) and angle count (48..128), Np=4,
    FP32, advanced together by one persistent graph-replayed launch per step
    with the autotuned work-group shape; compared with the same problems
    stepped one after another by the plain per-problem launch."""
    import torch
    from paper_2011_06856_amd import rlbm
    probs = W.batch_problems(48, seed=0, steps=a.steps)
    print("bench: batched form, %d problems" % len(probs), file=sys.stderr, flush=True)
    b = rlbm.Batch(probs, precision="f32")
    waves, tune_ms = b.autotune(candidates=(2, 3, 4, 6, 8), steps=4,
                                cache=os.path.join(ROOT, "_tune_cache.json") if a.tune_cache else None,
                                key="batch48_seed0_gfx950_f32_modes_bands")
    mode = b.get_mode()
    bands = b.get_push_bands()
    b.step(a.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = b.step_timed(a.steps)
    wall = time.perf_counter() - t0
    finite = all(np.isfinite(b.problem(i).moments(raise_nonphysical=False)[0]).all() for i in range(len(b)))
    sv = float(b.nsv) * a.steps
    del b
    torch.cuda.empty_cache()
    # plain path: each problem alone, same number of steps (timed on the library stream)
    plain_ms = 0.0
    for p in probs:
        s = rlbm.Solver(p["Np"], p["K"], p["N"])
        s.init_fields(p["nx"], p["ny"], *p["fields"], tau=p["tau"], dt=p["dt"], precision="f32")
        s.step(a.warmup)
        plain_ms += s.step_timed(a.steps)
        del s
    return {
        "metric": METRIC, "value": sv / wall / 1e9, "unit": "GSVUPS", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * wall / a.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch48_uneven_shocks_np4", "problems": len(probs),
                   "site_velocities_per_step": sv / a.steps, "autotuned_waves": waves, "autotuned_mode": mode,
                   "autotuned_push_bands": bands,
                   "fields_finite": bool(finite)},
        "batched_vs_plain": {"batched_gsvups_events": sv / (ms * 1e-3) / 1e9,
                             "plain_sequential_gsvups": sv / (plain_ms * 1e-3) / 1e9,
                             "speedup": plain_ms / ms},
    }


def field_errors(a, ref):
    """Per-field relative L2 and max errors of (n, eps, U^x, U^y) against a
    reference; the velocity as beta = U^i / U^0."""
    def beta(f):
        g = np.sqrt(1 + f[2] ** 2 + f[3] ** 2)
        return np.stack([f[2] / g, f[3] / g])
    out = {}
    for k, name in ((0, "n"), (1, "eps")):
        out[name] = {"rel_l2": float(np.linalg.norm(a[k] - ref[k]) / np.linalg.norm(ref[k])),
                     "rel_max": float(np.abs(a[k] - ref[k]).max() / np.abs(ref[k]).max())}
    ba, br = beta(a), beta(ref)
    out["beta"] = {"rel_l2": float(np.linalg.norm(ba - br) / np.linalg.norm(br)),
                   "abs_max": float(np.abs(ba - br).max())}
    return out


def precision_form(a):
    """Precision form: the quadrant Riemann problem at 2048^2 (periodic),
    Np=6 x K=256 (1536 velocities), order 5, Kn=10, with FP32 populations and
    with bfloat16 deviations from the local equilibrium (BF16DEV), both timed;
    the same steps in FP64 on the GPU give their per-field errors at full
    size.  (Their errors against the FP64 oracle, on a reduced grid of the
    same problem after 1000 steps, are measured by
    tests/test_gpu_deviation.py.)"""
    import torch
    side = a.side if a.side != 1024 else 2048
    cfg = W.quadrant_shock(side, steps=a.steps)
    runs = {}
    for prec in ("f32", "bf16dev", "f64"):
        print("bench: precision form %s %s steps=%d" % (cfg["name"], prec, a.steps), file=sys.stderr, flush=True)
        runs[prec] = gpu_run(cfg, a.steps, a.warmup, prec, a.waves if prec == "f32" else 0, keep_fields=True)
        torch.cuda.empty_cache()
    r32, rb, r64 = runs["f32"], runs["bf16dev"], runs["f64"]
    sv = r32["sv"]
    S = side * side
    # algorithmic bytes per launch: FP32 one 4-byte read and write per
    # site-velocity; BF16DEV 2 + 2 bytes plus the per-site equilibrium
    # coefficients (6 shells x 11, FP32) read and written once
    bytes32 = 8 * sv / a.steps
    bytesb = 4 * sv / a.steps + 2 * 4 * 6 * 11 * S

    def roof(r, nbytes, traffic_name):
        launch_ms = r["event_ms"] / a.steps
        ach = nbytes / (launch_ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": counter_traffic(traffic_name) if r["kernel"] == "push" else None,
                "kernel": "k_push_step" if r["kernel"] == "push" else "k_stream_collide",
                "algorithmic_bytes_per_sv": nbytes / (sv / a.steps), "avg_launch_ms": launch_ms}


    def charges_vs64(r):
        # global charges (sum N^0, T^00, T^0x, T^0y) minus FP64's, relative to the FP64 sums of N^0 and T^00
        return [float((x - y) / abs(r64["charges"][0 if i == 0 else 1]))
                for i, (x, y) in enumerate(zip(r["charges"], r64["charges"]))]

    return {
        "metric": METRIC, "value": sv / r32["wall_s"] / 1e9, "unit": "GSVUPS", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": 1e3 * r32["wall_s"] / a.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": cfg["name"] + "_order5", "grid": [side, side], "velocities": 1536, "order": 5,
                   "kernel": r32["kernel"], "fields_finite": r32["finite"] and rb["finite"] and r64["finite"]},
        "roofline": roof(r32, bytes32, "push_step_f32_quadrant_%d" % side),
        "fp32_error_vs_fp64": field_errors(r32["fields"], r64["fields"]),
        "charges_fp32_minus_fp64": charges_vs64(r32),
        "bf16dev": {"value": sv / rb["wall_s"] / 1e9, "unit": "GSVUPS", "ms_per_step": 1e3 * rb["wall_s"] / a.steps,
                    "dtype": "bf16 deviations, f32 arithmetic",
                    "roofline": roof(rb, bytesb, "push_step_bf16dev_quadrant_%d" % side),
                    "error_vs_fp64": field_errors(rb["fields"], r64["fields"]),
                    "charges_minus_fp64": charges_vs64(rb)},
        "fp64_reference": {"gsvups_events": sv / (r64["event_ms"] * 1e-3) / 1e9,
                           "avg_launch_ms": r64["event_ms"] / a.steps},
    }


def learned_form(a):
    """Learned form: 512^2 periodic shocks, Np=4; coarse K=24 plus the MLP
    correction (of the fields at readout, or of the shear stress after every
    step) against the plain solver swept over K in 24..384, all measured
    against plain K=384.  Reports the equal-error angle count K* per field
    and the speedup wall(plain K*) / wall(coarse + MLP)."""
    from paper_2011_06856_amd import learned as Lr
    say = lambda m: print("bench: " + m, file=sys.stderr, flush=True)
    r = Lr.study(side=a.side, steps=a.steps, train_seeds=range(a.train_seeds),
                 eval_seeds=range(10000, 10000 + a.eval_seeds), epochs=a.epochs, mode=a.learned_mode,
                 rows=a.rows, log=say)
    sp = [v for v in r["speedup"].values() if v]
    return {
        "metric": METRIC, "value": min(sp) if len(sp) == 3 else None, "unit": "x (wall plain K* / wall coarse+MLP)",
        "n_gpus": 1, "steps": a.steps, "warmup": 0, "ms_per_step": 1e3 * r["wall_corrected_s"] / a.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "learned_shocks_%d_np4_k24_vs_k384" % a.side, "train_seeds": a.train_seeds,
                   "eval_seeds": a.eval_seeds, "steps_per_run": a.steps, "epochs": a.epochs,
                   "correction": a.learned_mode, "rows": a.rows},
        "learned": r,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--side", type=int, default=1024)
    ap.add_argument("--waves", type=int, default=0)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--form", default="plain", choices=["plain", "batched", "learned", "precision"])
    ap.add_argument("--train-seeds", type=int, default=200, help="learned form: training seeds")
    ap.add_argument("--eval-seeds", type=int, default=20, help="learned form: held-out seeds")
    ap.add_argument("--epochs", type=int, default=15, help="learned form: training epochs")
    ap.add_argument("--rows", type=int, default=4096,
                    help="learned form: sampled sites per snapshot (10 snapshots a seed in the step mode; "
                         "the readout takes 10x this many sites of each run's end state)")
    ap.add_argument("--learned-mode", default="readout", choices=["readout", "step"],
                    help="learned form: correct the fields at readout, or the shear stress after every step")
    ap.add_argument("--tune-cache", action="store_true", help="reuse/store the autotuner choice in _tune_cache.json")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(the step would shard by row slabs with a one-row halo exchange per step); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.form == "batched":
        print(json.dumps(batched_form(a)), flush=True)
        return
    if a.form == "precision":
        print(json.dumps(precision_form(a)), flush=True)
        return
    if a.form == "learned":
        print(json.dumps(learned_form(a)), flush=True)
        return
    runs = {}
    for Kn in (0.01, 1.0):
        cfg = W.circular_shock(a.side, Kn=Kn, steps=a.steps)
        print("bench: run Kn=%g %s steps=%d" % (Kn, cfg["name"], a.steps), file=sys.stderr, flush=True)
        runs[Kn] = gpu_run(cfg, a.steps, a.warmup, a.precision, a.waves)
    sv = sum(r["sv"] for r in runs.values())
    wall = sum(r["wall_s"] for r in runs.values())
    ev_ms = sum(r["event_ms"] for r in runs.values())
    launches = 2 * a.steps
    launch_ms = ev_ms / launches
    bytes_per_launch = BYTES_PER_SV[a.precision] * sv / launches
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": sv / wall / 1e9,
        "unit": "GSVUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * wall / launches,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": a.precision,
        "data": "synthetic",
        "config": {"workload": "circular_shock_%d_np4_k64_order3" % a.side, "grid": [a.side, a.side],
                   "velocities": 256, "Kn": [0.01, 1.0], "runs": 2, "steps_per_run": a.steps,
                   "kernel": runs[0.01]["kernel"], "waves_per_group": runs[0.01]["waves"],
                   "fields_finite": all(r["finite"] for r in runs.values())},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": counter_traffic("stream_collide_%s_circular_%d" % (a.precision, a.side)),
                     "kernel": "k_stream_collide" if runs[0.01]["kernel"] == "tile" else "k_push_step",
                     "algorithmic_bytes_per_sv": BYTES_PER_SV[a.precision],
                     "avg_launch_ms": launch_ms},
    }
    print("bench: copy bandwidth", file=sys.stderr, flush=True)
    cb = copy_bandwidth()
    out["roofline"]["copy_measured"] = cb
    out["roofline"]["frac_of_copy"] = achieved / cb
    if not a.no_cpu_baseline:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(a.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
