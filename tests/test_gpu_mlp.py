"""The surrogate's hand-written MLP kernels against the FP64 reference, and
the surrogate-with-fallback path against the full plain computation.

Bounds: the FP32 gradient of the loss over 96 samples (three tiles) agrees
with the FP64 reference to 1e-4 of its largest component (rounding of
128-term FP32 dot products on the matrix cores); forward predictions to 1e-4
relative; the blend, computed in FP64, to 1e-12 relative with exact flags.
"""
import numpy as np
import pytest

from gpu_helpers import log, params_for, gpu_run, rel_err
from synth import make_system, workload
from oracle import mlp as ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2306_16493_amd import Context
    c = Context(make_system("toy_sc"))
    yield c
    c.close()


@pytest.mark.parametrize("nout,members", [(1, 2), (3, 3), (4, 1), (2, 5)])
def test_gradient_vs_fp64_reference(ctx, nout, members):
    import torch
    from paper_2306_16493_amd.eph import Mlp
    m = Mlp(ctx, members=members, n_out=nout, seed=3)
    rng = np.random.default_rng(nout)
    p = (rng.standard_normal((members, m.n_params)) * 0.08).astype(np.float32)
    m.set_params(p)
    assert np.array_equal(m.get_params(), p)
    n = 96
    x = rng.standard_normal((n, ref.NIN)).astype(np.float32)
    y = rng.standard_normal((n, nout)).astype(np.float32)
    dev = torch.device("cuda")
    loss, g = m.gradient(torch.tensor(x, device=dev), torch.tensor(y, device=dev))
    for e in range(members):
        lr_, gr = ref.loss_and_grad(p[e].astype(np.float64), x, y, nout)
        assert abs(loss[e] - lr_) <= 1e-4 * abs(lr_)
        err = np.max(np.abs(g[e] - gr)) / np.max(np.abs(gr))
        log(f"[mlp] member {e}: grad max err {err:.2e}")
        assert err < 1e-4


def test_forward_and_training(ctx):
    import torch
    from paper_2306_16493_amd.eph import Mlp
    m = Mlp(ctx, members=2, n_out=2, seed=5)
    rng = np.random.default_rng(7)
    n = 4096
    x = rng.uniform(-1, 1, (n, ref.NIN)).astype(np.float32)
    y = np.stack([np.sin(2 * x[:, 0]) + 0.5 * x[:, 3] ** 2, np.cos(x[:, 1] - x[:, 4])], axis=1).astype(np.float32)
    dev = torch.device("cuda")
    xt, yt = torch.tensor(x, device=dev), torch.tensor(y, device=dev)
    l0 = m.train(xt, yt, steps=1, batch=256, lr=1e-3)
    l1 = m.train(xt, yt, steps=1500, batch=256, lr=2e-3)
    log(f"[mlp] loss {l0} -> {l1}")
    assert np.all(l1 < 0.05 * l0)
    # forward pass of the GPU against the reference with the same normalisation
    pr = m.get_params()
    xm, xs = x.astype(np.float64).mean(0), x.astype(np.float64).std(0)
    ym, ys = y.astype(np.float64).mean(0), y.astype(np.float64).std(0)
    pred = m.predict(xt[:256]).cpu().numpy()
    for e in range(2):
        yr, _, _ = ref.forward(pr[e].astype(np.float64), (x[:256] - xm) / xs, 2)
        yr = yr * ys + ym
        assert np.max(np.abs(pred[e] - yr)) < 1e-4 * np.max(np.abs(yr)) + 1e-5
        # a ragged count (two full tiles and a partial one) gives the same rows
        pr77 = m.predict(xt[:77]).cpu().numpy()
        assert pr77.shape == (2, 77, 2)
        assert np.max(np.abs(pr77[e] - yr[:77])) < 1e-4 * np.max(np.abs(yr)) + 1e-5
    assert m.predict(xt[:0]).shape == (2, 0, 2)


def test_blend_against_numpy(ctx):
    """eph_mlp_blend: per state and output the ensemble mean of exp(y) and
    the relative spread (population standard deviation over the mean), the
    state flagged where the largest spread over outputs exceeds the
    threshold; a ragged count of states and an empty one."""
    import torch
    from paper_2306_16493_amd.eph import Mlp
    members, nout = 5, 3
    m = Mlp(ctx, members=members, n_out=nout, seed=2)
    rng = np.random.default_rng(17)
    for n in (77, 0):
        # members agree up to a per-state noise of 0..5 % in log space
        y = rng.normal(-3.0, 1.0, (1, n, nout)) + rng.normal(0.0, 1.0, (members, n, nout)) * \
            rng.uniform(0.0, 0.05, (1, n, 1))
        y = y.astype(np.float32)
        r = np.exp(y.astype(np.float64))
        mean = r.mean(axis=0)
        spread = (np.sqrt(np.maximum((r * r).mean(axis=0) - mean * mean, 0.0)) / mean).max(axis=1)
        srt = np.sort(spread)
        thr = float(0.5 * (srt[n // 2] + srt[n // 2 + 1])) if n else 0.05  # between two states
        if n:
            assert np.min(np.abs(spread - thr)) > 1e-9  # no state on the edge
        it, flag, nf = m.blend(torch.tensor(y, device="cuda"), thr)
        it, flag = it.cpu().numpy(), flag.cpu().numpy()
        assert it.shape == (nout, n) and flag.shape == (n,)
        if n:
            assert np.allclose(it, mean.T, rtol=1e-12, atol=0.0)
            assert np.array_equal(flag.astype(bool), spread > thr)
        assert nf == int(np.sum(spread > thr))
    m.close()


def test_invalid_sizes_leave_the_ensemble_usable(ctx):
    """Sizes outside the documented ranges are rejected with EPH_E_INVALID
    (members 1..64, outputs 1..MAX_TEMPS, batch a positive multiple of
    32, steps >= 0, lr > 0, gradient samples a positive multiple of 32); the
    ensemble is untouched and trains afterwards."""
    import torch
    from paper_2306_16493_amd import eph
    from paper_2306_16493_amd.eph import Mlp, EphError
    for members, nout in ((0, 1), (65, 1), (2, 0), (2, eph.MAX_TEMPS + 1)):
        with pytest.raises(EphError) as ei:
            Mlp(ctx, members=members, n_out=nout, seed=1)
        assert ei.value.code == eph.EPH_E_INVALID
    m = Mlp(ctx, members=2, n_out=eph.MAX_TEMPS, seed=9)
    p0 = m.get_params()
    rng = np.random.default_rng(3)
    n = 640
    xh = rng.uniform(-1, 1, (n, ref.NIN)).astype(np.float32)
    yh = np.stack([np.sin(2 * xh[:, t]) + 0.3 * xh[:, t + 4] for t in range(eph.MAX_TEMPS)], axis=1)
    x = torch.tensor(xh, device="cuda")
    y = torch.tensor(yh.astype(np.float32), device="cuda")
    for kw in (dict(steps=1, batch=48), dict(steps=1, batch=0), dict(steps=-1, batch=64),
               dict(steps=1, batch=64, lr=0.0)):
        with pytest.raises(EphError) as ei:
            m.train(x, y, **kw)
        assert ei.value.code == eph.EPH_E_INVALID
    with pytest.raises(EphError) as ei:
        m.gradient(x[:40], y[:40])
    assert ei.value.code == eph.EPH_E_INVALID
    assert np.array_equal(m.get_params(), p0)
    l0 = m.train(x, y, steps=1, batch=64, lr=1e-3)
    l1 = m.train(x, y, steps=300, batch=64, lr=2e-3)
    assert np.all(np.isfinite(l1)) and np.all(l1 < l0)
    m.close()


def test_surrogate_with_fallback_vs_plain():
    """Al-like 24^3: the ensemble fit on plain rates of a seeded k subset,
    with plain fallback where the members disagree by more than 1%, gives
    sigma within 1e-3 of the full plain run; the network alone (no fallback)
    beats the method without it, a constant rate (the geometric mean of the
    same training rates) for every state."""
    import torch
    from paper_2306_16493_amd import Context, surrogate
    w = workload("al_fcc_100", 24)
    s = make_system(w.system)
    c = Context(s)
    mu = s.mu_centroid
    lo, hi = mu + w.window[0], mu + w.window[1]
    temps = [300.0]
    full = gpu_run(c, c.params(24, mu, temps, w.eta, lo, hi))
    res = full["res"]
    sig_full = c.conductivity(res.energy, res.vel, res.inv_tau.reshape(-1), mu, temps, 24 ** 3)
    # fallback in chunks of 1000 k points: several rates calls merged in turn
    r = surrogate.run(c, 24, mu, temps, w.eta, lo, hi, train_frac=0.25, steps=6000, batch=512, decay=True,
                      threshold=0.01, log=log, fallback_chunk=1000)
    assert r.n_fallback_k > 2000
    err = rel_err(r.sigma, sig_full)
    log(f"[surrogate] sigma rel err {err:.3e}; flagged {r.n_flagged}/{r.n_states}; times {r.times}")
    assert np.array_equal(r.states[0].cpu().numpy(), full["state_k"])
    assert err < 1e-3
    # gain over the method without the network: one constant rate, the
    # geometric mean of the plain rates of the training states
    sk, sn, se, sv = r.states
    raw = r.raw_inv_tau.reshape(-1)
    sig_net = c.conductivity(se, sv, raw, mu, temps, 24 ** 3)
    train = np.isin(full["state_k"], r.train_k)
    it_train = full["inv_tau"][0][train]
    assert it_train.size == r.n_train_states
    const = torch.full_like(raw, float(np.exp(np.mean(np.log(it_train)))))
    sig_const = c.conductivity(se, sv, const, mu, temps, 24 ** 3)
    e_net, e_const = rel_err(sig_net, sig_full), rel_err(sig_const, sig_full)
    log(f"[surrogate] network-only sigma err {e_net:.3e} vs constant-rate {e_const:.3e}")
    assert e_net < e_const
