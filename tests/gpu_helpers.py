"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same seeded inputs, and compare gauge-invariant
results."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synth import make_system, workload  # noqa: E402


def log(*a):
    print(*a, flush=True)


def params_for(ctx, w, system, grid=None, k_subset=None, precision="fp64", temps=None, window=None):
    N = grid or w.grid
    mu = system.mu_centroid
    lo, hi = window if window is not None else (mu + w.window[0], mu + w.window[1])
    return ctx.params(N, mu, temps or w.temps, w.eta, lo, hi, band_lo=w.band_lo, band_hi=w.band_hi,
                      precision=precision, k_subset=k_subset), (N, mu, lo, hi)


def gpu_run(ctx, params):
    import torch
    res, bufs = ctx.scattering_rates(params)
    torch.cuda.synchronize()
    out = dict(state_k=res.state_k.cpu().numpy(), state_n=res.state_n.cpu().numpy(),
               energy=res.energy.cpu().numpy(), vel=res.vel.cpu().numpy(),
               inv_tau=res.inv_tau.cpu().numpy(), counts=res.counts, res=res)
    return out


def degenerate_mask(eps_table, state_k, state_n, tol=1e-6):
    """States whose band has another band within tol at the same k."""
    e = eps_table[state_k]
    d = np.abs(e - e[np.arange(len(state_k)), state_n][:, None])
    d[np.arange(len(state_k)), state_n] = np.inf
    return d.min(axis=1) < tol


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))
