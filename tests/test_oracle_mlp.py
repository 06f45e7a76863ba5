"""Pin of the FP64 reference MLP (oracle/mlp.py) by central finite
differences, so that it can in turn check the GPU backward kernels."""
import numpy as np

from oracle import mlp as ref


def test_reference_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    for nout in (1, 3):
        p = rng.standard_normal(ref.n_params(nout)) * 0.1
        x = rng.standard_normal((16, ref.NIN))
        y = rng.standard_normal((16, nout))
        loss, g = ref.loss_and_grad(p, x, y, nout)
        idx = rng.choice(p.size, size=60, replace=False)
        # include every block (first/last weight and bias of each layer)
        idx = np.concatenate([idx, [0, ref.H * ref.NIN, ref.H * ref.NIN + ref.H, p.size - 1, p.size - nout - 1]])
        h = 1e-6
        for i in idx:
            pp, pm = p.copy(), p.copy()
            pp[i] += h
            pm[i] -= h
            fd = (ref.loss_and_grad(pp, x, y, nout)[0] - ref.loss_and_grad(pm, x, y, nout)[0]) / (2 * h)
            assert abs(fd - g[i]) <= 1e-7 + 1e-6 * abs(g[i]), (i, fd, g[i])


def test_reference_forward_layer_shapes_and_silu():
    rng = np.random.default_rng(1)
    p = rng.standard_normal(ref.n_params(2)) * 0.1
    x = rng.standard_normal((5, ref.NIN))
    yhat, zs, hs = ref.forward(p, x, 2)
    assert yhat.shape == (5, 2) and len(zs) == 3 and len(hs) == 4
    z = np.linspace(-5, 5, 11)
    assert np.allclose(ref.silu(z), z / (1 + np.exp(-z)))
    assert ref.n_params(1) == 34561  # 10 inputs: 128*10 + 128 + 2*(128*128 + 128) + 128 + 1
