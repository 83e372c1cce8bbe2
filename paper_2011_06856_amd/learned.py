"""Learned form: a coarse-angle run plus an MLP correction of its traceless
stress, trained on fine-angle runs of the same method.

Workflow (all lattice work and all network arithmetic run in the library's
HIP kernels; numpy only samples and normalises training rows on the host):

1. data (teacher-forced, `collect`): for each training seed, a random disc or
   quadrant shock at Kn = 10^(-1 + 2u) is run at K_fine and at K_coarse
   angles in lockstep from the same initial state; after every coarse step
   its shear stress is set to the fine run's.  At snapshot steps the coarse
   run's 3x3 field patches (before that correction) are the inputs and the
   correction pi_fine - pi_coarse at the patch centre the target, so the
   rows come from the states of a corrected run (no drift between the
   states seen in training and in use).  `dagger` rounds add rows from runs
   corrected by the network itself.
2. training: mini-batch Adam on the GPU (rlbm_mlp_grad, rlbm_mlp_adam_step).
3. use: after every coarse step, rlbm_mlp_correct adds the predicted change
   of the stress to the populations (conserving N^mu and T^0mu).
4. reference and fallback: the plain fine-angle solver; errors are Eq. rel_err
   per field; the equal-error angle count K* of the plain solver, by log-log
   interpolation over a sweep of K, gives the speedup wall(plain K*) /
   wall(coarse + MLP).  In use (`corrected_fields`) a correction that is not
   finite, not physical, or made on inputs outside the training range falls
   back to the fine solver.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from paper_2011_06856_amd import rlbm  # noqa: E402

FIELDS = ("n", "eps", "ux", "uy")


def make_solver(K, side, fields, tau, dt, Np=4, precision="f32"):
    s = rlbm.Solver(Np, K, Np - 1)
    s.init_fields(side, side, *fields, tau=tau, dt=dt, precision=precision)
    return s


def shock(side, seed):
    Kn, fld = W.random_shock(side, seed)
    tau = W.tau_of(Kn, side)
    return Kn, fld, tau, W.dt_of(tau)


def run_fields(s):
    n, eps, ux, uy, _ = s.moments()
    return dict(n=n, eps=eps, ux=ux, uy=uy)


def rel_errors(a, ref):
    """Eq. rel_err per field (beta for the velocity, as in the paper)."""
    out = {}
    for k in ("n", "eps"):
        out[k] = float(np.linalg.norm(a[k] - ref[k]) / np.linalg.norm(ref[k]))

    def beta(f):
        g = np.sqrt(1 + f["ux"] ** 2 + f["uy"] ** 2)
        return np.stack([f["ux"] / g, f["uy"] / g])
    ba, br = beta(a), beta(ref)
    out["beta"] = float(np.linalg.norm(ba - br) / np.linalg.norm(br))
    return out


def collect(side, seeds, K_coarse, K_fine, steps, snapshots, rows_per_snapshot, net=None, seed_rows=0, log=None):
    """Training rows, teacher-forced.  A fine and a coarse run start from the
    same state and step in lockstep; after every coarse step its shear stress
    is set to the fine run's (the exact correction, added through the m = 2
    basis), so the coarse states are those of a perfectly corrected run.  At
    snapshot steps the input is the coarse run's 3x3 field patch before the
    correction (with log10 Kn in column 63) and the target the correction
    itself, pi_fine - pi_coarse, at the patch centre.  With `net`, the network's own correction is applied
    instead of the exact one, so that the rows come from the states it meets
    in use (targets stay the exact gaps)."""
    import torch
    X, T = [], []
    snap = set(int(round(steps * (k + 1) / snapshots)) for k in range(snapshots))
    ident = rlbm.MLP(max_batch=side * side, n_hidden=1, hidden=8)   # feature kernel with unit scales
    ident.set_norm(np.zeros(7), np.ones(7), np.zeros(3), np.ones(3))
    for si, sd in enumerate(seeds):
        if log and si % 20 == 0:
            log("learned: collecting seed %d of %d" % (si, len(seeds)))
        Kn, fld, tau, dt = shock(side, sd)
        f = make_solver(K_fine, side, fld, tau, dt)
        c = make_solver(K_coarse, side, fld, tau, dt)
        if net is not None:
            net.set_extra(np.log10(Kn))
        for t in range(1, steps + 1):
            f.step(1)
            c.step(1)
            gap = (rlbm.site_stats(f)[:, 4:7] - rlbm.site_stats(c)[:, 4:7]).contiguous()
            if t in snap:
                raw = ident.features(c)[:, :63]
                idx = W.uniform(seed_rows * 7919 + sd * 131 + t, np.arange(rows_per_snapshot))
                sel = torch.as_tensor((idx * side * side).astype(np.int64), device="cuda")
                X.append(np.concatenate([raw[sel].cpu().numpy(), np.full((rows_per_snapshot, 1), np.log10(Kn))],
                                        axis=1))
                T.append(gap[sel].cpu().numpy())
            if net is None:
                rlbm.add_stress(c, gap)
            else:
                net.correct(c)
        del f, c
    return np.concatenate(X), np.concatenate(T)


def collect_readout(side, seeds, K_coarse, K_fine, steps, rows, log=None):
    """Training rows of the readout correction.  Per seed a fine and a coarse
    run go to the end; the input is the coarse run's 3x3 field patch at the
    end with log10 Kn in column 63, the target the fine-minus-coarse fields
    at the patch centre: relative for n and eps, absolute for U^x, U^y."""
    X, T = [], []
    ident = rlbm.MLP(max_batch=side * side, n_hidden=1, hidden=8)   # feature kernel with unit scales
    ident.set_norm(np.zeros(7), np.ones(7), np.zeros(3), np.ones(3))
    for si, sd in enumerate(seeds):
        if log and si % 20 == 0:
            log("learned: collecting seed %d of %d" % (si, len(seeds)))
        Kn, fld, tau, dt = shock(side, sd)
        f = make_solver(K_fine, side, fld, tau, dt)
        f.step(steps)
        F = run_fields(f)
        del f
        c = make_solver(K_coarse, side, fld, tau, dt)
        c.step(steps)
        C = run_fields(c)
        raw = ident.features(c)[:, :63].cpu().numpy()
        del c
        tgt = np.stack([(F["n"] - C["n"]) / C["n"], (F["eps"] - C["eps"]) / C["eps"], F["ux"] - C["ux"],
                        F["uy"] - C["uy"]], axis=-1).reshape(-1, 4)
        idx = (W.uniform(sd * 17 + 5, np.arange(rows)) * side * side).astype(np.int64)
        X.append(np.concatenate([raw[idx], np.full((rows, 1), np.log10(Kn))], axis=1))
        T.append(tgt[idx])
    return np.concatenate(X), np.concatenate(T)


class Normaliser:
    def __init__(self, X, T):
        centre = X[:, 28:35]   # neighbour 4 = the site itself
        self.in_mu = centre.mean(axis=0)
        self.in_sig = centre.std(axis=0) + 1e-6
        self.out_mu = T.mean(axis=0)
        self.out_sig = T.std(axis=0) + 1e-9
        # the training inputs' range per normalised field (the trust region
        # of the correction in use)
        Xn = ((X[:, :63].reshape(-1, 9, 7) - self.in_mu) / self.in_sig).reshape(-1, 7)
        self.in_lo = Xn.min(axis=0)
        self.in_hi = Xn.max(axis=0)

    def inputs(self, X):
        """Normalised patches; column 63 carried over from X when it has one
        (the readout's per-run input), else zero."""
        Xn = (X[:, :63].reshape(-1, 9, 7) - self.in_mu) / self.in_sig
        extra = X[:, 63:64] if X.shape[1] == 64 else np.zeros((X.shape[0], 1))
        return np.concatenate([Xn.reshape(-1, 63), extra], axis=1).astype(np.float32)

    def targets(self, T):
        return ((T - self.out_mu) / self.out_sig).astype(np.float32)

    def apply(self, net):
        net.set_norm(self.in_mu, self.in_sig, self.out_mu, self.out_sig)


def train(net, Xn, Tn, epochs=20, batch=4096, lr=1e-3, seed=0, log=None):
    """Mini-batch Adam over shuffled rows; returns the mean loss per epoch."""
    import torch
    Xd = torch.as_tensor(Xn, device="cuda")
    Td = torch.as_tensor(Tn, device="cuda")
    n = Xd.shape[0]
    losses = []
    for ep in range(epochs):
        order = np.argsort(W.uniform(seed * 1000 + ep, np.arange(n)))
        perm = torch.as_tensor(order, device="cuda")
        tot, nb = 0.0, 0
        for k in range(0, n - batch + 1, batch):
            idx = perm[k:k + batch]
            loss = net.grad(Xd[idx].contiguous(), Td[idx].contiguous())
            net.adam_step(lr)
            tot += loss
            nb += 1
        losses.append(tot / max(nb, 1))
        if log:
            log("epoch %d loss %.5f" % (ep, losses[-1]))
    return losses


def evaluate(net, side, seeds, K_coarse, K_fine, steps, scale=1.0, relax=False):
    """Per-seed errors of the plain coarse run and of the corrected coarse run
    against the plain fine run, and the mean wall time per step of each."""
    import torch
    res = []
    for sd in seeds:
        Kn, fld, tau, dt = shock(side, sd)
        f = make_solver(K_fine, side, fld, tau, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f.step(steps)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        ref = run_fields(f)
        del f
        c = make_solver(K_coarse, side, fld, tau, dt)
        c.step(steps)
        plain = rel_errors(run_fields(c), ref)
        del c
        c = make_solver(K_coarse, side, fld, tau, dt)
        net.set_extra(np.log10(Kn))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(steps):
            c.step(1)
            net.correct(c, scale, relax=relax)
        try:
            fields = run_fields(c)
            tc = time.perf_counter() - t0
            corr = rel_errors(fields, ref)
        except rlbm.NonPhysicalState:
            tc = time.perf_counter() - t0
            corr = {k: float("inf") for k in plain}
        del c
        res.append(dict(seed=sd, Kn=Kn, plain=plain, corrected=corr, t_fine=tf, t_corrected=tc))
    return res


def evaluate_readout(net, side, seeds, K_coarse, K_fine, steps):
    """Per-seed errors of the plain coarse run and of its readout-corrected
    fields against the plain fine run, and the wall time of the coarse run
    with its readout."""
    import torch
    res = []
    for sd in seeds:
        Kn, fld, tau, dt = shock(side, sd)
        f = make_solver(K_fine, side, fld, tau, dt)
        f.step(steps)
        ref = run_fields(f)
        del f
        c = make_solver(K_coarse, side, fld, tau, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step(steps)
        n, eps, ux, uy = net.readout(c, float(np.log10(Kn)))
        tc = time.perf_counter() - t0
        plain = rel_errors(run_fields(c), ref)
        corr = rel_errors(dict(n=n, eps=eps, ux=ux, uy=uy), ref)
        del c
        res.append(dict(seed=sd, Kn=Kn, plain=plain, corrected=corr, t_corrected=tc))
    return res


def corrected_fields(net, norm, side, fld, tau, dt, Kn, steps, K_coarse=24, K_fine=384, margin=0.25):
    """The learned form in use, with the plain fine-angle solver as its
    fallback: a coarse run of `steps` steps and its readout correction are
    returned unless the correction cannot be trusted, in which case the fine
    run is made and its fields returned.  The correction is not trusted when
    a corrected field is not finite or not physical (n <= 0, eps <= 0, |U|
    not finite), or when the coarse run's normalised inputs leave the
    training range by more than `margin` of its width (norm.in_lo / in_hi,
    per field).  Returns (fields, source, reason) with source "network" or
    "fine"."""
    c = make_solver(K_coarse, side, fld, tau, dt)
    c.step(steps)
    net.set_extra(float(np.log10(Kn)))
    X = net.features(c)[:, :63].cpu().numpy().reshape(-1, 7)
    width = norm.in_hi - norm.in_lo
    outside = bool((X < norm.in_lo - margin * width).any() or (X > norm.in_hi + margin * width).any())
    n, eps, ux, uy = net.readout(c, float(np.log10(Kn)))
    del c
    reason = None
    if not all(np.isfinite(a).all() for a in (n, eps, ux, uy)):
        reason = "non-finite corrected field"
    elif (n <= 0).any() or (eps <= 0).any():
        reason = "non-physical corrected field"
    elif outside:
        reason = "inputs outside the training range"
    if reason is None:
        return dict(n=n, eps=eps, ux=ux, uy=uy), "network", None
    f = make_solver(K_fine, side, fld, tau, dt)
    f.step(steps)
    return run_fields(f), "fine", reason


def sweep_plain(side, seeds, Ks, K_fine, steps):
    """Mean error of the plain solver per angle count against K_fine, and its
    time per run (steps and the read-out of its fields)."""
    import torch
    out = {}
    refs = {}
    for sd in seeds:
        Kn, fld, tau, dt = shock(side, sd)
        f = make_solver(K_fine, side, fld, tau, dt)
        f.step(steps)
        refs[sd] = run_fields(f)
        del f
    for K in Ks:
        errs, times = [], []
        for sd in seeds:
            Kn, fld, tau, dt = shock(side, sd)
            s = make_solver(K, side, fld, tau, dt)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(steps)
            fields = run_fields(s)   # the run's output, read out as the corrected runs' are
            times.append(time.perf_counter() - t0)
            errs.append(rel_errors(fields, refs[sd]))
            del s
        out[K] = dict(err={k: float(np.mean([e[k] for e in errs])) for k in errs[0]}, time=float(np.mean(times)))
    return out


def equal_error_K(sweep, target, field="beta"):
    """Angle count at which the plain solver's mean error equals `target`, by
    log-log interpolation between the swept counts (None if outside)."""
    Ks = sorted(sweep)
    for a, b in zip(Ks, Ks[1:]):
        ea, eb = sweep[a]["err"][field], sweep[b]["err"][field]
        if (ea - target) * (eb - target) <= 0 and ea != eb:
            la, lb = np.log(ea), np.log(eb)
            w = (np.log(target) - la) / (lb - la)
            return float(np.exp(np.log(a) + w * (np.log(b) - np.log(a))))
    return None


def time_at_K(sweep, K):
    Ks = sorted(sweep)
    for a, b in zip(Ks, Ks[1:]):
        if a <= K <= b:
            w = (np.log(K) - np.log(a)) / (np.log(b) - np.log(a))
            return float(np.exp(np.log(sweep[a]["time"]) + w * (np.log(sweep[b]["time"]) - np.log(sweep[a]["time"]))))
    return None


def study(side=512, K_coarse=24, K_fine=384, steps=230, train_seeds=range(200), eval_seeds=range(10000, 10020),
          Ks=(24, 32, 48, 64, 96, 128, 192, 256, 384), snapshots=10, rows=4096, epochs=10, batch=4096, lr=1e-3,
          dagger=0, mode="readout", log=None):
    """The learned form end to end: data, training, use on held-out seeds,
    the plain sweep over K and the equal-error comparison.  mode "readout":
    the network corrects the coarse run's fields at the end (rows of
    collect_readout, 4 outputs); mode "step": it corrects the shear stress
    after every step (teacher-forced rows of collect, 3 outputs).  Returns a
    dict of errors, K* and speedups per field."""
    import torch
    say = log or (lambda m: None)
    t0 = time.perf_counter()
    if mode == "readout":
        X, T = collect_readout(side, list(train_seeds), K_coarse, K_fine, steps, rows * snapshots, log=say)
    else:
        X, T = collect(side, list(train_seeds), K_coarse, K_fine, steps, snapshots, rows, log=say)
    say("learned: %d training rows in %.1f s" % (X.shape[0], time.perf_counter() - t0))
    nm = Normaliser(X, T)
    net = rlbm.MLP(max_batch=side * side, out_dim=T.shape[1])
    net.init_params(seed=1)
    nm.apply(net)
    t1 = time.perf_counter()
    losses = train(net, nm.inputs(X), nm.targets(T), epochs=epochs, batch=batch, lr=lr, log=say)
    for r in range(dagger if mode == "step" else 0):
        seeds = [100000 + 1000 * r + k for k in range(len(list(train_seeds)) // 4)]
        X2, T2 = collect(side, seeds, K_coarse, K_fine, steps, snapshots, rows, net=net, seed_rows=r + 1)
        X, T = np.concatenate([X, X2]), np.concatenate([T, T2])
        losses += train(net, nm.inputs(X), nm.targets(T), epochs=max(1, epochs // 2), batch=batch, lr=lr / 2)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    say("learned: trained, loss %.4g -> %.4g in %.1f s" % (losses[0], losses[-1], t_train))
    if mode == "readout":
        res = evaluate_readout(net, side, list(eval_seeds), K_coarse, K_fine, steps)
    else:
        res = evaluate(net, side, list(eval_seeds), K_coarse, K_fine, steps)
    corr = {k: float(np.mean([r["corrected"][k] for r in res])) for k in ("n", "eps", "beta")}
    plain = {k: float(np.mean([r["plain"][k] for r in res])) for k in ("n", "eps", "beta")}
    t_corr = float(np.mean([r["t_corrected"] for r in res]))
    say("learned: coarse %s corrected %s" % (plain, corr))
    sw = sweep_plain(side, list(eval_seeds), Ks, K_fine, steps)
    out = dict(mode=mode, plain_coarse_err=plain, corrected_err=corr, wall_corrected_s=t_corr,
               per_seed=[dict(seed=r["seed"], Kn=r["Kn"], plain=r["plain"], corrected=r["corrected"]) for r in res],
               sweep={int(K): v for K, v in sw.items()}, train_rows=int(X.shape[0]), train_loss=[losses[0], losses[-1]],
               train_s=t_train, K_star={}, speedup={})
    for f in ("n", "eps", "beta"):
        Ks_ = equal_error_K(sw, corr[f], f)
        out["K_star"][f] = Ks_
        tk = time_at_K(sw, Ks_) if Ks_ is not None else None
        out["speedup"][f] = tk / t_corr if tk else None
    return out
