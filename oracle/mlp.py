"""FP64 numpy reference of the surrogate MLP (test infrastructure).

Same network and parameter layout as the HIP kernels: 10 -> 128 -> 128 -> 128
-> n_out, SiLU after each hidden layer, loss = mean over samples and outputs
of (prediction - target)^2.  Used to check the GPU forward pass and the
hand-written backward pass; it is itself pinned against finite differences.
"""
from __future__ import annotations

import numpy as np

NIN, H = 10, 128


def n_params(nout):
    return H * NIN + H + 2 * (H * H + H) + nout * H + nout


def unpack(p, nout):
    p = np.asarray(p, np.float64)
    o = 0

    def take(n, shape):
        nonlocal o
        a = p[o:o + n].reshape(shape)
        o += n
        return a
    W1 = take(H * NIN, (H, NIN)); b1 = take(H, (H,))
    W2 = take(H * H, (H, H)); b2 = take(H, (H,))
    W3 = take(H * H, (H, H)); b3 = take(H, (H,))
    W4 = take(nout * H, (nout, H)); b4 = take(nout, (nout,))
    return [(W1, b1), (W2, b2), (W3, b3), (W4, b4)]


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, x, nout):
    layers = unpack(p, nout)
    h = np.asarray(x, np.float64)
    zs, hs = [], [h]
    for i, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if i < 3:
            zs.append(z)
            h = silu(z)
            hs.append(h)
        else:
            h = z
    return h, zs, hs


def loss_and_grad(p, x, y, nout):
    """Loss and its gradient w.r.t. the flat parameter vector."""
    yhat, zs, hs = forward(p, x, nout)
    y = np.asarray(y, np.float64)
    m = yhat.size
    d = yhat - y
    loss = float(np.sum(d * d) / m)
    layers = unpack(p, nout)
    grads = []
    dz = 2.0 * d / m                        # dL/d(output pre-activation)
    for i in range(3, -1, -1):
        W, b = layers[i]
        hin = hs[i]
        grads.append((dz.T @ hin, dz.sum(axis=0)))
        if i > 0:
            dz = (dz @ W) * dsilu(zs[i - 1])
    grads = grads[::-1]
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat
