"""Pins of the FP64 oracle against closed forms, invariants, library routines
and brute force (no GPU).  Each test names the part of the paper it pins.

Independent constants come from scipy.constants (CODATA), never from the
oracle.
"""
import math

import numpy as np
import pytest
import scipy.constants as sc
from scipy import integrate, special

from synth import System, make_system, ws_block, lattice_block
import oracle
from oracle import Oracle, bruteforce as bf

HBAR = sc.hbar / sc.e
KB = sc.k / sc.e
CPH = sc.hbar ** 2 / (sc.physical_constants["atomic mass constant"][0] * 1e-20) / sc.e
VU = sc.e * 1e-10 / sc.hbar


def custom(lattice, mass, ham_terms, nw, ifc_terms, g_terms, re_n=1, rp_n=1, tau=None):
    """Build a System from dicts {R(tuple): matrix}."""
    rh = np.array(sorted(ham_terms), np.int32)
    ham = np.array([ham_terms[tuple(r)] for r in rh.tolist()], np.complex128).reshape(-1, nw, nw)
    rd = np.array(sorted(ifc_terms), np.int32)
    ifc = np.array([ifc_terms[tuple(r)] for r in rd.tolist()], np.float64)
    re, rp = lattice_block(re_n), lattice_block(rp_n)
    na = len(mass)
    gw = np.zeros((re.shape[0], rp.shape[0], 3 * na, nw, nw), np.complex128)
    for (a, b), v in g_terms.items():
        ia = [i for i, r in enumerate(re.tolist()) if tuple(r) == a][0]
        ib = [i for i, r in enumerate(rp.tolist()) if tuple(r) == b][0]
        gw[ia, ib] = v
    if tau is None:
        tau = np.zeros((na, 3))
    return System("custom", np.asarray(lattice, float), tau, np.asarray(mass, float), nw, rh,
                  np.ones(rh.shape[0]), ham, rd, np.ones(rd.shape[0]), ifc, re, rp, gw, 0.0)


def nn_band(eps0, t, a=3.0, nw=1, mass=26.98, omega0=None, g0=None):
    """Single-orbital (or diagonal multi-orbital) NN simple-cubic band, with an
    Einstein phonon (Phi(0) = M w0^2/C) and a local vertex when given."""
    eps0 = np.atleast_1d(eps0) * np.ones(nw)
    t = np.atleast_1d(t) * np.ones(nw)
    terms = {(0, 0, 0): np.diag(eps0)}
    for ax in range(3):
        for sgn in (1, -1):
            r = [0, 0, 0]
            r[ax] = sgn
            terms[tuple(r)] = np.diag(t)
    if omega0 is None:
        ifc = {(0, 0, 0): np.eye(3)}
    else:
        ifc = {(0, 0, 0): np.eye(3) * mass * omega0 ** 2 / CPH}
    g = {} if g0 is None else {((0, 0, 0), (0, 0, 0)): g0}
    return custom(np.diag([a, a, a]), [mass], terms, nw, ifc, g)


# ---------------------------------------------------------------- P1 / A1
def test_constants_match_codata():
    c = Oracle.constants()
    assert c["hbar_evs"] == pytest.approx(HBAR, rel=1e-15)
    assert c["kb_evk"] == pytest.approx(KB, rel=1e-15)
    assert c["cph_ev"] == pytest.approx(CPH, rel=1e-12)
    assert c["vel_unit"] == pytest.approx(VU, rel=1e-15)


def test_nn_cosine_band_closed_form():
    """Wannier interpolation of H (Sec. II.B): NN s-band on sc is
    eps0 + 2t sum cos(2 pi k_i)."""
    N = 8
    o = Oracle(nn_band(0.3, -0.7))
    eps, evec, vel = o.electrons(N)
    pts = bf.grid_points(N) / N
    ref = 0.3 + 2 * -0.7 * np.cos(2 * math.pi * pts).sum(axis=1)
    assert np.max(np.abs(eps[:, 0] - ref)) < 1e-13


def test_diagonal_multiorbital_sorted_cosines():
    N = 6
    o = Oracle(nn_band([0.0, 0.5, -0.4], [-0.3, 0.2, 0.45], nw=3))
    eps, _, _ = o.electrons(N)
    pts = bf.grid_points(N) / N
    c = np.cos(2 * math.pi * pts).sum(axis=1)
    ref = np.sort(np.stack([0.0 - 0.6 * c, 0.5 + 0.4 * c, -0.4 + 0.9 * c], axis=1), axis=1)
    assert np.max(np.abs(eps - ref)) < 1e-13


@pytest.mark.parametrize("name", ["al_fcc", "si_fcc"])
def test_eigensolver_vs_lapack(name):
    """Jacobi eigenpairs vs numpy.linalg.eigh (LAPACK) on the random systems:
    eigenvalues and band projectors |v><v|."""
    s = make_system(name)
    o = Oracle(s)
    N = 7
    kidx = np.array([0, 1, 17, 100, 200, 342], np.int64)
    eps, evec, vel = o.electrons(N, kidx)
    pts = bf.grid_points(N)
    for t, k in enumerate(kidx):
        H, dH = bf.hk(s, pts[k] / N)
        w, v = np.linalg.eigh(H)
        scale = np.max(np.abs(w))
        assert np.max(np.abs(eps[t] - w)) < 1e-13 * scale
        for n in range(s.nw):
            po = np.outer(evec[t, n], evec[t, n].conj())
            pl = np.outer(v[:, n], v[:, n].conj())
            gap = np.min(np.abs(np.delete(w, n) - w[n]))
            assert np.max(np.abs(po - pl)) < 1e-13 * scale / gap
        ref_v = np.real(np.einsum("in,aij,jn->na", v.conj(), dH, v)) * VU
        assert np.max(np.abs(vel[t] - ref_v)) <= 1e-12 * VU * np.abs(dH).max() * s.nw


def test_eigvec_orthonormal_and_residual():
    s = make_system("si_fcc")
    o = Oracle(s)
    N = 5
    eps, evec, _ = o.electrons(N)
    pts = bf.grid_points(N)
    for k in range(0, N ** 3, 11):
        H, _ = bf.hk(s, pts[k] / N)
        V = evec[k].T  # columns = eigenvectors
        assert np.max(np.abs(V.conj().T @ V - np.eye(s.nw))) < 1e-13
        assert np.max(np.abs(H @ V - V * eps[k][None, :])) < 1e-12


# ---------------------------------------------------------------- P2
def test_nn_velocity_closed_form():
    """Velocity of the NN band: v_i = -(2 t a/hbar) sin(2 pi k_i)."""
    N, t, a = 8, -0.7, 3.0
    o = Oracle(nn_band(0.3, t, a=a))
    _, _, vel = o.electrons(N)
    pts = bf.grid_points(N) / N
    ref = -2 * t * a * np.sin(2 * math.pi * pts) * VU
    assert np.max(np.abs(vel[:, 0, :] - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("name", ["al_fcc", "si_fcc"])
def test_velocity_finite_difference(name):
    """Hellmann-Feynman velocity vs central differences of the band energies
    on a 2^20 grid (reduced step 2^-20)."""
    s = make_system(name)
    o = Oracle(s)
    N = 1 << 20
    rng = np.random.default_rng(7)
    A = np.asarray(s.lattice)
    for _ in range(3):
        k = rng.integers(0, N, size=3)
        idx = lambda kk: int(kk[0] % N + N * ((kk[1] % N) + N * (kk[2] % N)))
        kl = [idx(k)]
        for ax in range(3):
            for d in (1, -1):
                kk = k.copy()
                kk[ax] += d
                kl.append(idx(kk))
        eps, _, vel = o.electrons(N, np.array(kl, np.int64))
        deps = np.stack([(eps[1 + 2 * ax] - eps[2 + 2 * ax]) * N / 2 for ax in range(3)], axis=1)
        grad = (A.T @ deps.T).T / (2 * math.pi)  # eV*A, per band
        gaps = np.min(np.abs(eps[0][:, None] - eps[0][None, :]) + np.eye(s.nw) * 1e9, axis=1)
        for n in range(s.nw):
            if gaps[n] < 1e-3:
                continue
            assert np.allclose(vel[0, n], grad[n] * VU, rtol=1e-6, atol=1e-6 * np.abs(grad).max() * VU)


# ---------------------------------------------------------------- P3
@pytest.mark.parametrize("name", ["toy_sc", "al_fcc", "si_fcc", "mini_w2a2", "mini_w4a2"])
def test_acoustic_sum_rule_and_psd(name):
    """D(q) from the spring construction: three zero modes at Gamma (acoustic
    sum rule), positive semidefinite on the whole grid, max w <= 40 meV."""
    s = make_system(name)
    o = Oracle(s)
    N = 6
    om, u, lam = o.phonons(N)
    lmax = np.max(np.abs(lam))
    assert np.sum(np.abs(lam[0]) <= 1e-12 * lmax) == 3
    assert np.all(lam >= -1e-12 * lmax)
    assert om.max() <= 0.040 + 1e-12
    # excluded modes carry zero displacement
    assert np.all(u[0][om[0] < 1e-4] == 0)


def test_isotropic_springs_closed_form():
    """NN isotropic springs K on sc: lambda = (2K/M) sum(1 - cos 2 pi q_i), 3-fold."""
    M, K = 26.98, 1.7
    ifc = {(0, 0, 0): 6 * K * np.eye(3)}
    for ax in range(3):
        for sgn in (1, -1):
            r = [0, 0, 0]
            r[ax] = sgn
            ifc[tuple(r)] = -K * np.eye(3)
    s = custom(np.eye(3) * 3.0, [M], {(0, 0, 0): np.zeros((1, 1))}, 1, ifc, {})
    N = 6
    om, u, lam = Oracle(s).phonons(N)
    q = bf.grid_points(N) / N
    ref = 2 * K / M * (1 - np.cos(2 * math.pi * q)).sum(axis=1)
    assert np.max(np.abs(lam - ref[:, None])) < 1e-13 * ref.max()
    hw = np.sqrt(CPH * ref)
    assert np.max(np.abs(om - hw[:, None])) < 1e-12
    # u = e sqrt(C/(2 M w)): columns have norm sqrt(C/(2 M w))
    for t in range(1, N ** 3):
        nrm = np.linalg.norm(u[t], axis=1)
        assert np.allclose(nrm, np.sqrt(CPH / (2 * M * hw[t])), rtol=1e-12)



def diatomic_chain(M1, M2, K, a=3.0):
    """Simple-cubic cell with atoms at 0 and a/2 along x, isotropic springs
    K (eV/A^2) between x-neighbours only: the x, y and z displacements each
    form the textbook diatomic chain."""
    I, z = np.eye(3), np.zeros((3, 3))
    ifc = {(0, 0, 0): np.block([[2 * K * I, -K * I], [-K * I, 2 * K * I]]),
           (1, 0, 0): np.block([[z, z], [-K * I, z]]),     # atom 2 at 0 <-> atom 1 at +a
           (-1, 0, 0): np.block([[z, -K * I], [z, z]])}
    return custom(np.diag([a, a, a]), [M1, M2], {(0, 0, 0): np.zeros((1, 1))}, 1, ifc, {},
                  tau=np.array([[0.0, 0.0, 0.0], [a / 2, 0.0, 0.0]]))


def test_diatomic_chain_unequal_masses_closed_form():
    """Dynamical matrix with the mass scaling 1/sqrt(M M') (Sec. II.B): for
    the diatomic chain, lambda = K(1/M1 + 1/M2) +- K sqrt((1/M1 + 1/M2)^2 -
    4 sin^2(theta/2)/(M1 M2)), theta = 2 pi q1, each 3-fold; hbar w =
    sqrt(C lambda).  Unequal masses make a slip such as sqrt(M M') -> M fail."""
    M1, M2, K = 26.98, 69.72, 1.3
    o = Oracle(diatomic_chain(M1, M2, K))
    N = 6
    om, u, lam = o.phonons(N)
    th = 2 * math.pi * bf.grid_points(N)[:, 0] / N
    s = 1 / M1 + 1 / M2
    root = np.sqrt(np.maximum(s * s - 4 * np.sin(th / 2) ** 2 / (M1 * M2), 0.0))
    ref = np.sort(np.repeat(np.stack([K * (s - root), K * (s + root)], 1), 3, axis=1), axis=1)
    assert np.max(np.abs(lam - ref)) < 1e-13 * ref.max()
    assert np.max(np.abs(om - np.sqrt(CPH * np.maximum(ref, 0.0)))) < 1e-13 * om.max()


def test_displacements_mass_weighted_norm_and_eigenvectors():
    """Mode displacements u = e (hbar / 2 M_mu w)^(1/2) (Sec. II.B) with
    unequal masses: sum_mu M_mu |u_mu nu|^2 = C / (2 hbar w_nu) for every
    kept mode, and e = u sqrt(2 M_mu hbar w / C) is an eigenvector of the
    mass-scaled dynamical matrix of the chain, written out here:
    D11 = 2K/M1, D22 = 2K/M2, D12 = -K (1 + e^{-i theta}) / sqrt(M1 M2)."""
    M1, M2, K = 26.98, 69.72, 1.3
    o = Oracle(diatomic_chain(M1, M2, K))
    N = 6
    om, u, lam = o.phonons(N, omega_cut=1e-4)
    mass = np.repeat([M1, M2], 3)
    kept = om >= 1e-4
    # the springs act along x only, so the acoustic branch vanishes on the whole q1 = 0 plane
    assert kept.sum() == 6 * N ** 3 - 3 * N ** 2
    norm = np.einsum("qnm,m->qn", np.abs(u) ** 2, mass)
    ref = CPH / (2 * np.where(kept, om, 1.0))
    assert np.max(np.abs(norm - ref)[kept] / ref[kept]) < 1e-13
    assert np.all(np.abs(u[~kept]) == 0)
    th = 2 * math.pi * bf.grid_points(N)[:, 0] / N
    for q in range(N ** 3):
        d12 = -K * (1 + np.exp(-1j * th[q])) / math.sqrt(M1 * M2)
        D = np.zeros((6, 6), complex)
        D[:3, :3] = np.eye(3) * 2 * K / M1
        D[3:, 3:] = np.eye(3) * 2 * K / M2
        D[:3, 3:] = np.eye(3) * d12
        D[3:, :3] = np.eye(3) * np.conj(d12)
        for nu in np.nonzero(kept[q])[0]:
            e = u[q, nu] * np.sqrt(2 * mass * om[q, nu] / CPH)
            assert abs(np.linalg.norm(e) - 1) < 1e-12
            assert np.max(np.abs(D @ e - lam[q, nu] * e)) < 1e-12 * np.abs(D).max()

# ---------------------------------------------------------------- P4
def test_single_vertex_term_phase_free():
    """g nonzero at one (Re0, Rp0) only: |g(k,q)| does not depend on the
    phases, so it equals |U(k+q) g0 U+(k) u(q)| built from LAPACK vectors."""
    base = make_system("al_fcc")
    g0 = np.zeros((3, 4, 4), complex)
    rng = np.random.default_rng(3)
    g0[:] = rng.standard_normal((3, 4, 4)) + 1j * rng.standard_normal((3, 4, 4))
    s = custom(base.lattice, base.mass, {tuple(r): h for r, h in zip(base.rh.tolist(), base.ham)}, 4,
               {tuple(r): f for r, f in zip(base.rd.tolist(), base.ifc)}, {((1, -1, 0), (0, 1, 1)): g0},
               re_n=3, rp_n=3)
    s.rh_w, s.rd_w = base.rh_w, base.rd_w
    o = Oracle(s)
    N = 5
    eps, evec, _ = o.electrons(N)
    om, u, _ = o.phonons(N)
    beps, bV, _ = bf.electrons(s, N)
    bom, bu = bf.phonons(s, N)
    pts = bf.grid_points(N)
    for k, q in [(3, 7), (11, 0), (50, 99), (124, 64)]:
        p = int(np.dot((pts[k] + pts[q]) % N, [1, N, N * N]))
        g = o.vertex(N, k, q, evec[k], evec[p], u[q])
        ref = np.einsum("im,uij,jn,uv->mnv", bV[p].conj(), g0, bV[k], bu[q])
        assert np.allclose(np.abs(g), np.abs(ref), rtol=1e-11, atol=1e-13 * np.abs(ref).max())


def test_vertex_vs_literal_five_fold_sum():
    """General vertex vs the literal five-fold sum (gauge-invariant |g|)."""
    s = make_system("toy_sc")
    o = Oracle(s)
    N = 3
    eps, evec, _ = o.electrons(N)
    om, u, _ = o.phonons(N)
    beps, bV, _ = bf.electrons(s, N)
    bom, bu = bf.phonons(s, N)
    pts = bf.grid_points(N)
    for k in range(N ** 3):
        for q in (1, 5, 13, 26):
            p = int(np.dot((pts[k] + pts[q]) % N, [1, N, N * N]))
            g = o.vertex(N, k, q, evec[k], evec[p], u[q])
            ref = bf.vertex(s, N, pts[k], pts[q], bV[k], bV[p], bu[q])
            assert np.allclose(np.abs(g), np.abs(ref), rtol=1e-10, atol=1e-12 * np.abs(ref).max())


# ---------------------------------------------------------------- P5
def test_basis_change_invariance():
    """Gauge: a constant unitary change of the Wannier basis (H' = W H W+,
    g' = W g W+) and an orthogonal rotation of the displacement axes leave
    energies, frequencies and every 1/tau unchanged."""
    s = make_system("toy_sc")
    rng = np.random.default_rng(11)
    W, _ = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    O, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    s2 = make_system("toy_sc")
    s2.ham = np.einsum("ab,rbc,dc->rad", W, s.ham, W.conj())
    s2.ifc = np.einsum("ab,rbc,dc->rad", O, s.ifc, O)
    s2.gw = np.einsum("ab,xybij,ci,dj->xyacd", O, s.gw, W, W.conj())
    N, mu, T, eta = 4, s.mu_centroid, [300.0], 0.05
    r1 = Oracle(s).run(N, mu, T, eta, -1e3, 1e3)
    r2 = Oracle(s2).run(N, mu, T, eta, -1e3, 1e3)
    assert np.max(np.abs(r1["energy"] - r2["energy"])) < 1e-12
    assert np.allclose(r1["inv_tau"], r2["inv_tau"], rtol=1e-10, atol=1e-10 * r1["inv_tau"].max())


def test_degenerate_group_sum_invariant():
    """H = h (x) I2 makes every band two-fold; individual |g|^2 depend on the
    basis chosen inside each pair, the pair sums do not: oracle (Jacobi) vs
    brute force (LAPACK) agree on group sums."""
    rng = np.random.default_rng(5)
    h = {}
    for r in lattice_block(3).tolist():
        h[tuple(r)] = rng.standard_normal() * math.exp(-np.linalg.norm(r))
    for r in list(h):
        neg = tuple(-x for x in r)
        v = 0.5 * (h[r] + h[neg])
        h[r] = h[neg] = v
    ham = {r: v * np.eye(2) for r, v in h.items()}
    g0 = rng.standard_normal((3, 2, 2)) + 1j * rng.standard_normal((3, 2, 2))
    ifc = {(0, 0, 0): np.diag([1.0, 1.3, 1.7])}
    s = custom(np.eye(3) * 3.0, [26.98], ham, 2, ifc, {((0, 0, 0), (0, 0, 0)): g0})
    N, eta, T = 3, 0.05, [300.0]
    o = Oracle(s)
    r = o.run(N, 0.0, T, eta, -1e3, 1e3, sw=40.0)
    bt, _ = bf.rates(s, N, 0.0, T, eta, states=list(zip(r["state_k"].tolist(), r["state_n"].tolist())))
    it = r["inv_tau"][0].reshape(-1, 2).sum(axis=1)
    bt = bt[0].reshape(-1, 2).sum(axis=1)
    assert np.allclose(it, bt, rtol=1e-10)


# ---------------------------------------------------------------- P6
def test_time_reversal():
    """Real H, Phi and g: eps(k) = eps(-k), v(-k) = -v(k), 1/tau(k) = 1/tau(-k)."""
    s = make_system("toy_sc", real_g=True)
    N = 4
    o = Oracle(s)
    r = o.run(N, s.mu_centroid, [300.0], 0.05, -1e3, 1e3)
    pts = bf.grid_points(N)
    neg = np.array([int(np.dot((-p) % N, [1, N, N * N])) for p in pts])
    eps, _, vel, _, _ = r["tables"]
    assert np.max(np.abs(eps - eps[neg])) < 1e-12
    assert np.max(np.abs(vel + vel[neg])) < 1e-10 * np.abs(vel).max()
    it = r["inv_tau"][0].reshape(N ** 3, s.nw)
    assert np.allclose(it, it[neg], rtol=1e-10, atol=1e-12 * it.max())


# ---------------------------------------------------------------- P7 / P8
def test_einstein_local_vertex_closed_form():
    """Single band, Einstein phonon w0, g only at (0,0) = c: sum_nu |g|^2 =
    C|c|^2/(2 M w0) for every (k,q), so 1/tau is a smeared one-dimensional
    density-of-states sum over the analytic cosine band."""
    eps0, t, a, M, w0, eta = 0.0, -0.25, 3.0, 26.98, 0.03, 0.04
    c = np.array([0.3 + 0.1j, -0.2, 0.05j])
    s = nn_band(eps0, t, a=a, mass=M, omega0=w0, g0=c.reshape(3, 1, 1))
    N, T, mu = 6, [150.0, 400.0], 0.1
    r = Oracle(s).run(N, mu, T, eta, -1e3, 1e3, sw=40.0)
    kp = bf.grid_points(N) / N
    e = eps0 + 2 * t * np.cos(2 * math.pi * kp).sum(axis=1)
    g2 = CPH * np.sum(np.abs(c) ** 2) / (2 * M * w0)
    delta = lambda x: np.exp(-(x / eta) ** 2) / (math.sqrt(math.pi) * eta)
    for ti, TT in enumerate(T):
        kt = KB * TT
        n0 = 1 / math.expm1(w0 / kt)
        f = 1 / (np.exp((e - mu) / kt) + 1)
        ref = np.array([(2 * math.pi / HBAR) / N ** 3 * g2 *
                        np.sum((n0 + f) * delta(ek + w0 - e) + (1 + n0 - f) * delta(ek - w0 - e)) for ek in e])
        assert np.allclose(r["inv_tau"][ti], ref, rtol=1e-12)


def test_delta_normalised():
    L = oracle.lib()
    for eta in (0.01, 0.05):
        x = np.linspace(-20 * eta, 20 * eta, 40001)
        d = np.array([L.orc_delta(float(v), eta) for v in x])
        assert abs(d.sum() * (x[1] - x[0]) - 1.0) < 1e-12
        assert L.orc_delta(0.0, eta) == pytest.approx(1 / (math.sqrt(math.pi) * eta), rel=1e-15)


# ---------------------------------------------------------------- P9
def test_constant_tau_sigma_cosine_band():
    """Constant tau: sigma = 2 e^2 tau/(N_k V) sum v v f(1-f)/k_B T, with the
    analytic velocities of the NN band; cubic: sigma_xx = yy = zz, xy = 0."""
    t, a, N, mu, T, tau = -0.7, 3.0, 10, 0.2, [300.0, 600.0], 2e-14
    o = Oracle(nn_band(0.0, t, a=a))
    eps, _, vel = o.electrons(N)
    kp = bf.grid_points(N) / N
    v = -2 * t * a * np.sin(2 * math.pi * kp) * VU
    e = eps[:, 0]
    inv = np.full((2, N ** 3), 1 / tau)
    sig = o.sigma(e, vel[:, 0], inv, mu, T, N ** 3)
    for ti, TT in enumerate(T):
        kt = KB * TT
        f = 1 / (np.exp((e - mu) / kt) + 1)
        ref = 2 * sc.e ** 2 * tau / (N ** 3 * a ** 3 * 1e-30) * np.einsum(
            "ka,kb,k->ab", v, v, f * (1 - f) / (kt * sc.e))
        assert np.allclose(sig[ti], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        d = np.diag(sig[ti])
        assert np.allclose(d, d[0], rtol=1e-12)
        assert np.max(np.abs(sig[ti] - np.diag(d))) < 1e-12 * d[0]


def test_sigma_skips_zero_rate_states():
    o = Oracle(nn_band(0.0, -0.5))
    e = np.array([0.0, 0.01])
    v = np.array([[1e5, 0, 0], [2e5, 0, 0]])
    inv = np.array([[1e13, 0.0]])
    s1 = o.sigma(e, v, inv, 0.0, [300.0], 8)
    s2 = o.sigma(e[:1], v[:1], inv[:, :1], 0.0, [300.0], 8)
    assert np.array_equal(s1, s2)


def test_carrier_density_full_band():
    """Bands far below mu are fully occupied: n_c = 2 nbands / V."""
    o = Oracle(nn_band([-5.0, -6.0], [0.1, 0.1], nw=2))
    eps, _, _ = o.electrons(4)
    nc = o.carrier_density(eps, 0, 1, 0.0, [300.0])
    assert nc[0] == pytest.approx(2 * 2 / (27.0 * 1e-30), rel=1e-12)


# ---------------------------------------------------------------- P10 + brute force
@pytest.mark.parametrize("N", [2, 3])
def test_rates_vs_brute_force(N):
    """Oracle 1/tau (sieved at 6 eta, q-batch bracket order, Jacobi vectors)
    vs the literal untruncated brute force (LAPACK vectors) on tiny grids."""
    s = make_system("toy_sc")
    mu, T, eta = s.mu_centroid, [200.0, 300.0], 0.5
    r = Oracle(s).run(N, mu, T, eta, -1e3, 1e3)
    states = list(zip(r["state_k"].tolist(), r["state_n"].tolist()))
    bt, _ = bf.rates(s, N, mu, T, eta, states=states)
    assert np.allclose(r["inv_tau"], bt, rtol=1e-10, atol=1e-12 * bt.max())


def test_rates_two_atom_vs_brute_force():
    s = make_system("si_fcc")
    # shrink the vertex to a 2^3 x 2^3 block to keep the brute force small
    s.re, s.rp = lattice_block(2), lattice_block(2)
    rng = np.random.default_rng(9)
    s.gw = (rng.standard_normal((8, 8, 6, 8, 8)) + 1j * rng.standard_normal((8, 8, 6, 8, 8))) * 0.05
    N, T, eta = 2, [300.0], 0.3
    o = Oracle(s)
    r = o.run(N, 0.0, T, eta, -1e3, 1e3)
    states = list(zip(r["state_k"].tolist(), r["state_n"].tolist()))
    bt, _ = bf.rates(s, N, 0.0, T, eta, states=states)
    assert np.allclose(r["inv_tau"], bt, rtol=1e-10, atol=1e-12 * bt.max())


def test_sieve_truncation_negligible():
    """Keeping |x| <= 6 eta vs keeping every term changes 1/tau below 1e-12."""
    s = make_system("toy_sc")
    o = Oracle(s)
    N = 6
    tables = (*o.electrons(N), *o.phonons(N)[:2])
    a = o.run(N, s.mu_centroid, [300.0], 0.05, -1e3, 1e3, tables=tables)
    b = o.run(N, s.mu_centroid, [300.0], 0.05, -1e3, 1e3, tables=tables, sw=60.0)
    assert np.allclose(a["inv_tau"], b["inv_tau"], rtol=1e-12, atol=1e-14 * b["inv_tau"].max())


def test_counts_vs_numpy_sieve():
    """n_q_valid, n_terms and n_kq against a direct numpy count."""
    s = make_system("toy_sc")
    o = Oracle(s)
    N, eta, sw = 5, 0.05, 6.0
    r = o.run(N, s.mu_centroid, [300.0], eta, s.mu_centroid - 0.5, s.mu_centroid + 0.5)
    eps, _, _, om, _ = r["tables"]
    pts = bf.grid_points(N)
    nkq = 0
    for k in np.unique(r["state_k"]):
        pidx = ((pts[k] + pts) % N) @ np.array([1, N, N * N])
        anyk = np.zeros(N ** 3, bool)
        for si in np.nonzero(r["state_k"] == k)[0]:
            e = eps[k, r["state_n"][si]]
            x = e + np.array([1, -1])[None, None, None, :] * om[:, None, :, None] - eps[pidx][:, :, None, None]
            ok = (np.abs(x) <= sw * eta) & (om[:, None, :, None] >= 1e-4)
            assert ok.sum() == r["n_terms"][si]
            assert ok.any(axis=(1, 2, 3)).sum() == r["n_q_valid"][si]
            anyk |= ok.any(axis=(1, 2, 3))
        nkq += anyk.sum()
    assert nkq == r["n_kq"]


# ---------------------------------------------------------------- transport coefficients
def test_transport_sigma_moment_equals_sigma():
    """The zeroth moment is sigma itself (same sum, same order)."""
    o = Oracle(nn_band(0.0, -0.4))
    eps, _, vel = o.electrons(6)
    rng = np.random.default_rng(5)
    inv = rng.uniform(1e13, 3e13, (2, 6 ** 3))
    sig, see, kap = o.transport(eps[:, 0], vel[:, 0], inv, 0.1, [300.0, 500.0], 6 ** 3)
    ref = o.sigma(eps[:, 0], vel[:, 0], inv, 0.1, [300.0, 500.0], 6 ** 3)
    assert np.allclose(sig, ref, rtol=1e-13, atol=0)


def test_seebeck_vanishes_for_particle_hole_symmetric_band():
    """NN simple-cubic band with mu at its centre and constant tau: states at
    eps0 + x and eps0 - x come in pairs (k -> k + (1/2,1/2,1/2)) with equal
    v v f(1-f), so the first moment and the Seebeck coefficient vanish; off
    centre it does not: below the centre the Fermi surface is electron-like
    (sigma(E) grows with E, so S < 0 by Mott's formula for charge -e
    carriers), above it hole-like (S > 0), with equal magnitudes."""
    o = Oracle(nn_band(0.0, -0.1))
    N = 16
    eps, _, vel = o.electrons(N)
    inv = np.full((1, N ** 3), 1e13)
    _, see0, _ = o.transport(eps[:, 0], vel[:, 0], inv, 0.0, [600.0], N ** 3)
    _, see_lo, _ = o.transport(eps[:, 0], vel[:, 0], inv, -0.3, [600.0], N ** 3)
    _, see_hi, _ = o.transport(eps[:, 0], vel[:, 0], inv, 0.3, [600.0], N ** 3)
    scale = abs(see_lo[0, 0, 0])
    assert scale > 1e-6
    assert np.max(np.abs(see0)) < 1e-10 * scale
    assert see_lo[0, 0, 0] < 0 < see_hi[0, 0, 0]
    assert see_hi[0, 0, 0] == pytest.approx(-see_lo[0, 0, 0], rel=1e-10)


def test_wiedemann_franz_degenerate_limit():
    """Constant tau, Fermi level inside a wide band, k_B T << band width:
    the Sommerfeld expansion gives kappa / (sigma T) = (pi^2/3)(k_B/e)^2,
    with corrections of relative order (k_B T / W)^2 (here ~1e-3)."""
    o = Oracle(nn_band(0.0, -1.0))
    N = 48
    eps, _, vel = o.electrons(N)
    inv = np.full((1, N ** 3), 1e13)
    T = 1500.0
    sig, _, kap = o.transport(eps[:, 0], vel[:, 0], inv, -1.5, [T], N ** 3)
    lorenz = kap[0, 0, 0] / (sig[0, 0, 0] * T)
    assert lorenz == pytest.approx(math.pi ** 2 / 3 * (sc.k / sc.e) ** 2, rel=0.03)


def _square_lattice_dos(e, t):
    """DOS of 2t(cos a + cos b) for a, b uniform, normalised to 1:
    K(1 - (e/4t)^2) / (2 pi^2 |t|) inside the band (complete elliptic
    integral of the first kind, parameter m = k^2)."""
    m = 1.0 - (e / (4 * t)) ** 2
    return special.ellipk(m) / (2 * math.pi ** 2 * abs(t)) if m > 0 else 0.0


def _transport_function_cosine_band(E, t):
    """Xi(E) = <sin^2 theta_x delta(E - 2t sum_i cos theta_i)>, up to a
    constant: the x integral of sin^2 times the 2-D DOS of the y, z part,
    by adaptive quadrature with break points where the 2-D DOS is singular
    (e = 0) or steps (e = +-4|t|)."""
    pts = []
    for e0 in (0.0, 4 * abs(t), -4 * abs(t)):
        c = (E - e0) / (2 * t)
        if abs(c) < 1:
            a = math.acos(c)
            pts += [a, 2 * math.pi - a]
    f = lambda th: math.sin(th) ** 2 * _square_lattice_dos(E - 2 * t * math.cos(th), t)
    v, _ = integrate.quad(f, 0, 2 * math.pi, points=sorted(pts), limit=400, epsabs=0, epsrel=1e-11)
    return v


def test_seebeck_magnitude_mott_formula():
    """Seebeck coefficient (Sec. II.C) in the degenerate limit: with constant
    tau, S = -(pi^2/3) k_B^2 T d ln Xi(E)/dE at E = mu (Mott), with Xi the
    transport function of the NN cosine band computed above from the 2-D
    DOS in closed form, independently of the oracle.  Corrections are of
    relative order (k_B T / t)^2 and from the finite grid; measured 0.3%."""
    t, mu, T, N = -1.0, -4.0, 1000.0, 64
    assert abs(integrate.quad(lambda e: _square_lattice_dos(e, t), -4, 4, points=[0], limit=400)[0] - 1) < 1e-9
    o = Oracle(nn_band(0.0, t))
    eps, _, vel = o.electrons(N)
    inv = np.full((1, N ** 3), 1e13)
    _, see, _ = o.transport(eps[:, 0], vel[:, 0], inv, mu, [T], N ** 3)
    h = 1e-3
    dlog = (math.log(_transport_function_cosine_band(mu + h, t)) -
            math.log(_transport_function_cosine_band(mu - h, t))) / (2 * h)
    mott = -(math.pi ** 2 / 3) * KB ** 2 * T * dlog
    assert see[0, 0, 0] == pytest.approx(mott, rel=0.02)
    assert see[0, 1, 1] == pytest.approx(see[0, 0, 0], rel=1e-10)
