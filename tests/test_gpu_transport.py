"""Transport coefficients and carrier density through the C ABI against the
FP64 oracle (tolerance 1e-10 relative to the largest element of each
tensor, as for sigma)."""
import numpy as np
import pytest

from gpu_helpers import log, params_for, gpu_run, rel_err
from synth import make_system, workload
from oracle import Oracle

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_transport_al_three_temperatures(torch_cuda):
    from paper_2306_16493_amd import Context
    w = workload("al_fcc_100", 12)
    s = make_system(w.system)
    ctx = Context(s)
    p, (N, mu, lo, hi) = params_for(ctx, w, s, 12)
    g = gpu_run(ctx, p)
    res = g["res"]
    sig, see, kap = ctx.transport(res.energy, res.vel, res.inv_tau.reshape(-1), mu, w.temps, N ** 3)
    o = Oracle(s)
    # the reduction alone, on the GPU's own per-state data
    s0, e0, k0 = o.transport(g["energy"], g["vel"], g["inv_tau"], mu, w.temps, N ** 3)
    for a, b, name in ((sig, s0, "sigma"), (see, e0, "seebeck"), (kap, k0, "kappa")):
        err = rel_err(a, b)
        log(f"[transport] {name}: rel err vs oracle reduction {err:.2e}")
        assert err < 1e-12
    # the whole path: oracle rates and oracle reduction
    r = o.run(N, mu, w.temps, w.eta, lo, hi, w.band_lo, w.band_hi)
    s1, e1, k1 = o.transport(r["energy"], r["vel"], r["inv_tau"], mu, w.temps, N ** 3)
    for a, b, name in ((sig, s1, "sigma"), (see, e1, "seebeck"), (kap, k1, "kappa")):
        err = rel_err(a, b)
        log(f"[transport] {name}: rel err vs oracle path {err:.2e}")
        assert err < TOL
    assert np.allclose(sig, ctx.conductivity(res.energy, res.vel, res.inv_tau.reshape(-1), mu, w.temps, N ** 3),
                       rtol=0, atol=0)
    ctx.close()


def test_carrier_density_and_mobility_si(torch_cuda):
    from paper_2306_16493_amd import Context, mobility
    s = make_system("si_fcc")
    o = Oracle(s)
    N = 6
    eps, _, _ = o.electrons(N)
    cbm = eps[:, 4].min()
    mu = cbm - 0.25
    temps = [300.0, 500.0]
    ctx = Context(s)
    n_gpu = ctx.carrier_density(N, 4, 7, mu, temps)
    n_orc = o.carrier_density(eps, 4, 7, mu, temps)
    err = np.max(np.abs(n_gpu - n_orc) / n_orc)
    log(f"[density] si_fcc N=6: n = {n_gpu}, rel err {err:.2e}")
    assert err < TOL
    # mobility of the conduction-band window states
    w = workload("si_fcc_150", N)
    p, _ = params_for(ctx, w, s, N, window=(cbm - 1e-7, cbm + 0.4), temps=temps)
    g = gpu_run(ctx, p)
    res = g["res"]
    sig = ctx.conductivity(res.energy, res.vel, res.inv_tau.reshape(-1), mu, temps, N ** 3)
    mob = mobility(sig, n_gpu)
    assert np.allclose(mob, sig / (n_orc[:, None, None] * 1.602176634e-19) * 1e4, rtol=1e-10, atol=0)
    ctx.close()
