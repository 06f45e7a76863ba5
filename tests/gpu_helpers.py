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


def degenerate_groups(eps_table, state_k, state_n, tol=1e-6):
    """Label of the degenerate group of each state: states at the same k
    whose band energies are chained within tol share a label."""
    lab = np.arange(len(state_k))
    order = np.lexsort((eps_table[state_k, state_n], state_k))
    for a, b in zip(order[:-1], order[1:]):
        if state_k[a] == state_k[b] and abs(eps_table[state_k[b], state_n[b]] - eps_table[state_k[a], state_n[a]]) < tol:
            lab[b] = lab[a]
    return lab


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def compare_rates(g, o_inv, eps_table, sk, sn, tol=1e-10):
    """Per-state 1/tau where the state is non-degenerate; sums over each
    degenerate group (bands within 1e-6 eV at one k) otherwise, the
    gauge-invariant quantity there."""
    lab = degenerate_groups(eps_table, sk, sn)
    uniq, inv, cnt = np.unique(lab, return_inverse=True, return_counts=True)
    deg = cnt[inv] > 1
    it_g, it_o = g["inv_tau"], o_inv
    scale = np.max(np.abs(it_o))
    for t in range(it_o.shape[0]):
        a, b = it_g[t][~deg], it_o[t][~deg]
        err = np.abs(a - b) / np.maximum(np.abs(b), 1e-12 * scale)
        msg = f"  T{t}: max rel err 1/tau = {err.max() if err.size else 0:.3e} over {err.size} states"
        if deg.any():
            ga = np.bincount(inv, weights=it_g[t])[cnt > 1]
            gb = np.bincount(inv, weights=it_o[t])[cnt > 1]
            gerr = np.abs(ga - gb) / np.maximum(np.abs(gb), 1e-12 * scale)
            msg += f"; {deg.sum()} near-degenerate states in {gerr.size} groups, max rel err of group sums {gerr.max():.3e}"
            assert gerr.max() < tol
        log(msg)
        assert err.size == 0 or err.max() < tol
