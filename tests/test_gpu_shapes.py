"""Parity of the HIP path with the oracle on the remaining (orbitals, modes)
shapes the rate kernel instantiates: 1 and 8 orbitals with 3 modes, 2 and 4
orbitals with 6 modes (small models, every block 4^3), on an odd 5^3 grid
with every state in the window; FP64 to 1e-10 and the FP32 form to its
1e-4 bound."""
import numpy as np
import pytest

from gpu_helpers import log, gpu_run, compare_rates, rel_err
from synth import make_system
from oracle import Oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name,prec", [("mini_w1", "fp64"), ("mini_w8", "fp64"), ("mini_w2a2", "fp64"),
                                       ("mini_w4a2", "fp64"), ("mini_w8", "fp32"), ("mini_w2a2", "fp32")])
def test_shape_vs_oracle(torch_cuda, name, prec):
    from paper_2306_16493_amd import Context
    s = make_system(name)
    N, eta, temps = 5, 0.05, [300.0, 600.0]
    mu = s.mu_centroid
    ctx = Context(s)
    p = ctx.params(N, mu, temps, eta, -1e3, 1e3, precision=prec)
    g = gpu_run(ctx, p)
    r = Oracle(s).run(N, mu, temps, eta, -1e3, 1e3)
    assert np.array_equal(g["state_k"], r["state_k"]) and np.array_equal(g["state_n"], r["state_n"])
    tol = 1e-10 if prec == "fp64" else 1e-4
    log(f"[shape] {name} {prec}: nw={s.nw} modes={s.nmodes} states={len(r['state_k'])}")
    compare_rates(g, r["inv_tau"], r["tables"][0], r["state_k"], r["state_n"], tol=tol)
    c = g["counts"]
    assert c["n_kq"] == r["n_kq"] and c["n_terms"] == int(r["n_terms"].sum())
    res = g["res"]
    sig = ctx.conductivity(res.energy, res.vel, res.inv_tau.reshape(-1), mu, temps, N ** 3)
    assert rel_err(sig, r["sigma"]) < tol
    ctx.close()
