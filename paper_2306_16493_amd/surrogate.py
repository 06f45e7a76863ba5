"""Surrogate-with-fallback orchestration of the scattering rates (argument
marshalling and scheduling only; the arithmetic is in the HIP kernels).

Steps, each a C-ABI call:
  1. eph_select_states             every window state (k, n, eps, v);
  2. eph_scattering_rates          plain rates on a seeded fraction of the
                                   k points that carry states (training set);
  3. eph_mlp_features/_train       an ensemble of MLPs fit to log(1/tau);
  4. eph_mlp_predict/_blend        ensemble mean and relative spread for
                                   every state;
  5. eph_scattering_rates          plain rates again at the k points of the
     + eph_merge_rates             states whose spread exceeds the threshold
                                   (and the training states), merged in;
  6. eph_conductivity              sigma from the blended rates.
fit() does steps 1-4 once; finish() does steps 4 (blend) to 6 for one
threshold, so several thresholds can share one fit; run() chains them.
The choice of k points (a seeded permutation of the k indices) and the
learning-rate schedule (successive eph_mlp_train calls, which keep Adam's
moments) are host-side bookkeeping of which work to do.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class SurrogateResult:
    inv_tau: "object"          # torch [nt][ns] blended rates
    sigma: np.ndarray          # [nt][3][3]
    n_states: int
    n_train_k: int
    n_train_states: int
    n_flagged: int
    n_fallback_k: int
    loss: np.ndarray
    times: dict = field(default_factory=dict)
    states: tuple = ()         # (k, n, e, v) device tensors
    raw_inv_tau: "object" = None  # network-only ensemble mean (before fallback)
    train_k: "object" = None   # k points whose rates came from the plain kernel for training
    fallback_k: "object" = None  # k points recomputed by the plain kernel


@dataclass
class Fitted:
    """Steps 1-4 done: the window states, the training rates, the ensemble's
    prediction; finish() takes it through steps 5-6 for one threshold."""
    ctx: "object"
    P: "object"
    temps: list
    grid: int
    mu: float
    states: tuple
    train: "object"            # plain result at the training k points
    ktrain: np.ndarray
    y: "object"                # ensemble predictions (members x states x temps)
    mlp: "object"
    loss: np.ndarray
    times: dict


# step decay of the learning rate: (fraction of the steps, factor on lr)
DECAY = ((0.5, 1.0), (0.25, 0.25), (0.125, 1.0 / 16), (0.125, 1.0 / 64))


def fit(ctx, grid, mu, temps, eta, win_lo, win_hi, band_lo=0, band_hi=-1, train_frac=0.02, members=5,
        steps=2000, batch=256, lr=2e-3, seed=1649307, precision="fp64", log=None, decay=False):
    import torch
    from .eph import Mlp

    def say(*a):
        if log:
            log(*a)

    temps = list(np.atleast_1d(temps))
    nt = len(temps)
    times = {}
    t0 = time.perf_counter()
    P = lambda ks=None: ctx.params(grid, mu, temps, eta, win_lo, win_hi, band_lo, band_hi, precision=precision,
                                   k_subset=ks)
    sk, sn, se, sv = ctx.select_states(P())
    torch.cuda.synchronize()
    ns = int(sk.shape[0])
    times["select_s"] = time.perf_counter() - t0
    # ---- training set: a seeded fraction of the k points with states ----
    kall = np.unique(sk.cpu().numpy())
    rng = np.random.default_rng(seed)
    ntk = max(1, int(round(train_frac * kall.size)))
    ktrain = np.sort(rng.choice(kall, size=ntk, replace=False))
    t1 = time.perf_counter()
    tr, _ = ctx.scattering_rates(P(ktrain))
    torch.cuda.synchronize()
    times["train_rates_s"] = time.perf_counter() - t1
    say(f"[surrogate] {ns} states, training on {tr.state_k.shape[0]} states at {ntk} k points")
    # ---- fit ----
    t2 = time.perf_counter()
    mlp = Mlp(ctx, members=members, n_out=nt, seed=seed)
    x_tr, y_tr = mlp.features(tr.state_k, tr.energy, tr.vel, grid, mu, inv_tau=tr.inv_tau)
    if decay:  # Adam's moments carry over between the segments
        for frac, fac in DECAY:
            loss = mlp.train(x_tr, y_tr, steps=max(1, int(round(frac * steps))), batch=batch, lr=lr * fac)
    else:
        loss = mlp.train(x_tr, y_tr, steps=steps, batch=batch, lr=lr)
    torch.cuda.synchronize()
    times["fit_s"] = time.perf_counter() - t2
    say(f"[surrogate] member losses {np.array2string(loss, precision=4)}")
    # ---- predict every state ----
    t3 = time.perf_counter()
    x_all, _ = mlp.features(sk, se, sv, grid, mu)
    y = mlp.predict(x_all)
    torch.cuda.synchronize()
    times["predict_s"] = time.perf_counter() - t3
    return Fitted(ctx, P, temps, grid, mu, (sk, sn, se, sv), tr, ktrain, y, mlp, loss, times)


def finish(f, threshold=0.01, log=None, fallback_chunk=400000):
    import torch
    from .eph import merge_rates

    def say(*a):
        if log:
            log(*a)

    ctx = f.ctx
    sk, sn, se, sv = f.states
    times = dict(f.times)
    t3 = time.perf_counter()
    inv_tau, flag, nflag = f.mlp.blend(f.y, threshold)
    raw = inv_tau.clone()
    torch.cuda.synchronize()
    times["blend_s"] = time.perf_counter() - t3
    # ---- fallback: plain rates at the k points of flagged states ----
    t4 = time.perf_counter()
    tr = f.train
    merge_rates(ctx, sk, sn, inv_tau, tr.state_k, tr.state_n, tr.inv_tau)
    kflag = np.unique(sk[flag.bool()].cpu().numpy()) if nflag else np.zeros(0, np.int64)
    kflag = np.setdiff1d(kflag, f.ktrain)
    # in chunks of at most fallback_chunk k points (bounded buffers, progress)
    for c0 in range(0, kflag.size, fallback_chunk):
        fb, _ = ctx.scattering_rates(f.P(kflag[c0:c0 + fallback_chunk]))
        merge_rates(ctx, sk, sn, inv_tau, fb.state_k, fb.state_n, fb.inv_tau)
        torch.cuda.synchronize()
        say(f"[surrogate] fallback {min(c0 + fallback_chunk, kflag.size)}/{kflag.size} k points, "
            f"{time.perf_counter() - t4:.1f} s")
    torch.cuda.synchronize()
    times["fallback_s"] = time.perf_counter() - t4
    say(f"[surrogate] threshold {threshold}: {nflag} states flagged, plain fallback at {kflag.size} k points")
    sig = ctx.conductivity(se, sv, inv_tau.reshape(-1), f.mu, f.temps, f.grid ** 3)
    times["total_s"] = sum(times[k] for k in ("select_s", "train_rates_s", "fit_s", "predict_s", "blend_s",
                                              "fallback_s"))
    return SurrogateResult(inv_tau, sig, int(sk.shape[0]), int(f.ktrain.size), int(tr.state_k.shape[0]), nflag,
                           int(kflag.size), f.loss, times, f.states, raw, f.ktrain, kflag)


def run(ctx, grid, mu, temps, eta, win_lo, win_hi, band_lo=0, band_hi=-1, train_frac=0.02, members=5,
        steps=2000, batch=256, lr=2e-3, threshold=0.01, seed=1649307, precision="fp64", log=None,
        fallback_chunk=400000, decay=False):
    """Steps 1-6 for one threshold."""
    f = fit(ctx, grid, mu, temps, eta, win_lo, win_hi, band_lo, band_hi, train_frac, members, steps, batch, lr,
            seed, precision, log, decay)
    try:
        return finish(f, threshold, log, fallback_chunk)
    finally:
        f.mlp.close()
