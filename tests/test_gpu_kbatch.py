"""The k-batch order of the vertex (Sec. III.D), the ablation partner of the
q-batch rate kernel: the same rates, another association of the same sum,
against the FP64 oracle (1e-10 relative per state, counts exact) and against
the q-batch path."""
import numpy as np
import pytest

from gpu_helpers import log, params_for, gpu_run, compare_rates, rel_err
from synth import make_system, workload
from oracle import Oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("name,grid,qb", [("toy_sc_8", 5, 7), ("al_fcc_100", 8, 64), ("si_fcc_150", 4, 5)])
def test_kbatch_order_vs_oracle(torch_cuda, name, grid, qb):
    from paper_2306_16493_amd import Context
    w = workload(name, grid)
    s = make_system(w.system)
    ctx = Context(s)
    if name.startswith("si"):
        o = Oracle(s)
        eps, _, _ = o.electrons(grid)
        cbm = eps[:, 4].min()
        p, (N, mu, lo, hi) = params_for(ctx, w, s, grid, window=(cbm - 1e-7, cbm + 0.5))
    else:
        p, (N, mu, lo, hi) = params_for(ctx, w, s, grid)
    kb, _ = ctx.rates_kbatch(p, q_batch=qb)
    g = dict(inv_tau=kb.inv_tau.cpu().numpy())
    r = Oracle(s).run(N, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi)
    log(f"[kbatch] {name} N={N}, q batch {qb}: {len(r['state_k'])} states")
    assert np.array_equal(kb.state_k.cpu().numpy(), r["state_k"])
    compare_rates(g, r["inv_tau"], r["tables"][0], r["state_k"], r["state_n"])
    assert kb.counts["n_nkq"] == int(r["n_q_valid"].sum())
    assert kb.counts["n_terms"] == int(r["n_terms"].sum())
    qbr = gpu_run(ctx, p)
    assert rel_err(g["inv_tau"], qbr["inv_tau"]) < 1e-12
    ctx.close()
