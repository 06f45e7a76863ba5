"""Pins of the oracle's transition rates and iterative BTE (Sec. II.C, the
iteration equation; Sec. III.E, storage of the summed transition rates)
against closed forms, symmetry and plain linear algebra (no GPU)."""
import math

import numpy as np
import pytest

from synth import make_system
from oracle import Oracle, bruteforce as bf
from test_oracle_pins import nn_band, CPH, HBAR, KB


def _run(system, N, mu, temps, eta, lo=-1e3, hi=1e3, sw=6.0):
    o = Oracle(system)
    eps, evec, vel = o.electrons(N)
    om, u, _ = o.phonons(N)
    sk, sn = o.select_states(eps, 0, -1, lo, hi)
    r = o.rates(N, eps, evec, om, u, sk, sn, mu, temps, eta, sw)
    gam = o.gamma(N, eps, evec, om, u, sk, sn, mu, temps, eta, sw)
    return o, eps, vel, sk, sn, r, gam


def test_gamma_rows_sum_to_inv_tau():
    """Gamma holds the terms of 1/tau before the sum over final states, so
    every row sums to that state's 1/tau, at every temperature."""
    s = make_system("toy_sc")
    o, eps, vel, sk, sn, r, gam = _run(s, 5, s.mu_centroid, [200.0, 500.0], 0.05)
    rs, val = gam["row_start"], gam["val"]
    rows = np.add.reduceat(val, rs[:-1], axis=0) if val.size else np.zeros((0, 2))
    empty = rs[1:] == rs[:-1]
    rows[empty] = 0.0
    assert np.allclose(rows.T, r["inv_tau"], rtol=1e-12, atol=0)
    # one entry per (state, final state) with a kept term: n_q_valid <= entries <= n_terms
    cnt = np.diff(rs)
    assert np.all(cnt >= r["n_q_valid"]) and np.all(cnt <= r["n_terms"])
    for s0 in range(len(sk)):
        f = gam["fin"][rs[s0]:rs[s0 + 1]]
        assert np.unique(f).size == f.size


def test_gamma_einstein_local_vertex_closed_form():
    """Single band, Einstein phonon w0, g only at (0,0): every entry is
    (2 pi/hbar)(1/N^3) C|c|^2/(2 M w0) [(N0 + f') delta(e + w0 - e') +
    (1 + N0 - f') delta(e - w0 - e')] over the analytic cosine band."""
    eps0, t, a, M, w0, eta = 0.0, -0.25, 3.0, 26.98, 0.03, 0.04
    c = np.array([0.3 + 0.1j, -0.2, 0.05j])
    s = nn_band(eps0, t, a=a, mass=M, omega0=w0, g0=c.reshape(3, 1, 1))
    N, T, mu = 5, [150.0, 400.0], 0.1
    o, eps, vel, sk, sn, r, gam = _run(s, N, mu, T, eta, sw=40.0)
    kp = bf.grid_points(N) / N
    e = eps0 + 2 * t * np.cos(2 * math.pi * kp).sum(axis=1)
    g2 = CPH * np.sum(np.abs(c) ** 2) / (2 * M * w0)
    delta = lambda x: np.exp(-(x / eta) ** 2) / (math.sqrt(math.pi) * eta)
    rs = gam["row_start"]
    for ti, TT in enumerate(T):
        kt = KB * TT
        n0 = 1 / math.expm1(w0 / kt)
        f = 1 / (np.exp((e - mu) / kt) + 1)
        for si in range(len(sk)):
            ek = e[sk[si]]
            ref = (2 * math.pi / HBAR) / N ** 3 * g2 * ((n0 + f) * delta(ek + w0 - e) +
                                                        (1 + n0 - f) * delta(ek - w0 - e))
            fin = gam["fin"][rs[si]:rs[si + 1]]
            assert np.allclose(gam["val"][rs[si]:rs[si + 1], ti], ref[fin], rtol=1e-12, atol=0)
            # final states beyond the sieve (|x| > 40 eta) carry a negligible closed form
            dropped = np.setdiff1d(np.arange(N ** 3), fin)
            assert np.all(ref[dropped] < 1e-300 + 1e-14 * ref.max())


def test_iteration_zero_is_serta_sigma():
    s = make_system("toy_sc")
    o, eps, vel, sk, sn, r, gam = _run(s, 4, s.mu_centroid, [300.0], 0.05)
    energy, v = eps[sk, sn], vel[sk, sn]
    sig, F = o.bte(4, sk, sn, energy, v, r["inv_tau"], gam, s.mu_centroid, [300.0], 4 ** 3, 0)
    ref = o.sigma(energy, v, r["inv_tau"], s.mu_centroid, [300.0], 4 ** 3)
    assert np.allclose(sig[0], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    assert np.allclose(F[0], v / r["inv_tau"][0][:, None], rtol=1e-15)


def test_isotropic_scattering_leaves_serta_unchanged():
    """With an Einstein phonon and a local vertex, Gamma depends on the two
    energies only, and the cosine band is inversion symmetric with
    v(-k) = -v(k): the in-scattering sum cancels pairwise, so every
    iteration returns F0 and sigma stays at its SERTA value."""
    eps0, t, M, w0, eta = 0.0, -0.25, 26.98, 0.03, 0.04
    c = np.array([0.3 + 0.1j, -0.2, 0.05j])
    s = nn_band(eps0, t, mass=M, omega0=w0, g0=c.reshape(3, 1, 1))
    N, T, mu = 6, [300.0], 0.1
    o, eps, vel, sk, sn, r, gam = _run(s, N, mu, T, eta)
    energy, v = eps[sk, sn], vel[sk, sn]
    sig, F = o.bte(N, sk, sn, energy, v, r["inv_tau"], gam, mu, T, N ** 3, 5)
    scale = np.abs(sig[0]).max()
    assert scale > 0
    for i in range(1, 6):
        assert np.max(np.abs(sig[i] - sig[0])) < 1e-12 * scale
    assert np.max(np.abs(F[0] - v / r["inv_tau"][0][:, None])) < 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("name,N,window", [("toy_sc", 4, None), ("al_fcc", 6, 0.6)])
def test_iterates_are_neumann_partial_sums(name, N, window):
    """F^n = sum_{i<=n} A^i F0 with A = diag(tau) Gamma restricted to final
    states in the list (dense matrix products in numpy); where the series
    converges, the fixed point solves (1 - A) F = F0 (numpy.linalg.solve)."""
    s = make_system(name)
    mu = s.mu_centroid
    lo, hi = (-1e3, 1e3) if window is None else (mu - window, mu + window)
    T = [300.0]
    o, eps, vel, sk, sn, r, gam = _run(s, N, mu, T, 0.05, lo, hi)
    ns, nw = len(sk), s.nw
    energy, v = eps[sk, sn], vel[sk, sn]
    it = r["inv_tau"][0]
    assert np.all(it > 0)
    sidx = -np.ones(N ** 3 * nw, np.int64)
    sidx[sk.astype(np.int64) * nw + sn] = np.arange(ns)
    G = np.zeros((ns, ns))
    rs = gam["row_start"]
    for si in range(ns):
        for e in range(rs[si], rs[si + 1]):
            j = sidx[gam["fin"][e]]
            if j >= 0:
                G[si, j] += gam["val"][e, 0]
    A = G / it[:, None]
    F0 = v / it[:, None]
    n = 4
    sig, F = o.bte(N, sk, sn, energy, v, r["inv_tau"], gam, mu, T, N ** 3, n)
    ref, term = F0.copy(), F0.copy()
    for _ in range(n):
        term = A @ term
        ref += term
    assert np.max(np.abs(F[0] - ref)) < 1e-12 * np.abs(ref).max()
    # rows of A sum to at most 1 (to exactly 1 when every final state is in
    # the list), so the spectral radius is at most 1
    rho = np.max(np.abs(np.linalg.eigvals(A)))
    assert rho <= 1.0 + 1e-12
    if rho < 0.5:
        sig, F = o.bte(N, sk, sn, energy, v, r["inv_tau"], gam, mu, T, N ** 3, 60)
        fix = np.linalg.solve(np.eye(ns) - A, F0)
        assert np.max(np.abs(F[0] - fix)) < 1e-10 * np.abs(fix).max()
