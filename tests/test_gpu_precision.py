"""Reduced-precision forms against the FP64 oracle.

The BF16x3 form differs from the FP32 form only in the Re transform, which
runs on bf16 MFMA with each FP32 operand split as hi + lo and the three
products hi*hi + hi*lo + lo*hi accumulated in FP32 (the dropped lo*lo term is
~2^-16 relative, below FP32 rounding of the sums), so it shares the FP32
bounds.

The FP32 form runs the Re and Rp transforms and the band/mode rotations in
FP32 (FP32 tables) with energies, the sieve and the 1/tau and sigma
accumulations in FP64.  Its error comes from ~1e-7 unit roundoff amplified by
sums over a few hundred lattice vectors, so the stated bounds are: per-state
1/tau within 1e-4 relative, sigma within 1e-4 relative (the acceptance bound
for sigma in reduced precision is 1e-3).  Integer counts are exact because the
sieve uses the FP64 energies in every form.
"""
import numpy as np
import pytest

from gpu_helpers import log, params_for, gpu_run, rel_err
from synth import make_system, workload
from oracle import Oracle

pytestmark = pytest.mark.gpu

TOL_RATE = 1e-4
TOL_SIGMA = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name,grid,prec", [("al_fcc_100", 12, "fp32"), ("toy_sc_8", 8, "fp32"),
                                            ("al_fcc_100", 12, "bf16x3"), ("toy_sc_8", 8, "bf16x3")])
def test_reduced_form_vs_oracle(torch_cuda, name, grid, prec):
    from paper_2306_16493_amd import Context
    w = workload(name, grid)
    s = make_system(w.system)
    ctx = Context(s)
    p32, (N, mu, lo, hi) = params_for(ctx, w, s, grid, precision=prec)
    g = gpu_run(ctx, p32)
    r = Oracle(s).run(N, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi)
    assert np.array_equal(g["state_k"], r["state_k"]) and np.array_equal(g["state_n"], r["state_n"])
    err = np.abs(g["inv_tau"] - r["inv_tau"]) / np.maximum(np.abs(r["inv_tau"]), 1e-12 * r["inv_tau"].max())
    log(f"[{prec}] {name} N={N}: max rel err 1/tau {err.max():.3e}")
    assert err.max() < TOL_RATE
    c = g["counts"]
    assert c["n_kq"] == r["n_kq"] and c["n_terms"] == int(r["n_terms"].sum())
    res = g["res"]
    sig = ctx.conductivity(res.energy, res.vel, res.inv_tau.reshape(-1), mu, w.temps, N ** 3)
    serr = rel_err(sig, r["sigma"])
    log(f"[{prec}] {name} N={N}: sigma rel err {serr:.3e}")
    assert serr < TOL_SIGMA


def test_fp32_form_si_two_atoms(torch_cuda):
    from paper_2306_16493_amd import Context
    w = workload("si_fcc_150", 6)
    s = make_system("si_fcc")
    o = Oracle(s)
    eps, _, _ = o.electrons(6)
    cbm = eps[:, 4].min()
    ctx = Context(s)
    p32, (N, mu, lo, hi) = params_for(ctx, w, s, 6, precision="fp32", window=(cbm - 1e-7, cbm + 0.4))
    g = gpu_run(ctx, p32)
    r = o.run(N, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi)
    err = np.abs(g["inv_tau"] - r["inv_tau"]) / np.maximum(np.abs(r["inv_tau"]), 1e-12 * r["inv_tau"].max())
    log(f"[fp32] si_fcc N=6: max rel err 1/tau {err.max():.3e}")
    assert err.max() < TOL_RATE
