"""Literal brute-force evaluation of the SERTA rates for tiny grids (numpy).

Test infrastructure: an independent second check of the C oracle.  It
evaluates the interpolation formula of g (Sec. II.B) as the literal five-fold
sum over (i, j, mu, Re, Rp) with the full phase exp(i(k.Re + q.Rp)) in
floating point, takes eigenvectors from numpy.linalg.eigh, and applies the
SERTA rate (Sec. II.C) with the untruncated Gaussian (no sieve).  Nothing here
is shared with the C oracle or with the HIP library.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.constants as sc

HBAR_EVS = sc.hbar / sc.e
KB_EVK = sc.k / sc.e
CPH_EV = sc.hbar ** 2 / (sc.physical_constants["atomic mass constant"][0] * 1e-20) / sc.e
VEL_UNIT = sc.e * 1e-10 / sc.hbar


def grid_points(N):
    i = np.arange(N ** 3)
    return np.stack([i % N, (i // N) % N, i // (N * N)], axis=1)


def hk(system, kred):
    """H(k) and dH/dk_alpha (Cartesian, eV*A) at reduced k."""
    ph = np.exp(2j * math.pi * (system.rh @ kred)) * system.rh_w
    cart = system.rh @ system.lattice
    H = np.einsum("r,rij->ij", ph, system.ham)
    dH = np.einsum("r,ra,rij->aij", 1j * ph, cart, system.ham)
    return H, dH


def dq(system, qred):
    sq = np.sqrt(np.repeat(system.mass, 3))
    ph = np.exp(2j * math.pi * (system.rd @ qred)) * system.rd_w
    return np.einsum("r,rab->ab", ph, system.ifc) / (sq[:, None] * sq[None, :])


def electrons(system, N):
    pts = grid_points(N)
    nk = pts.shape[0]
    nw = system.nw
    eps = np.zeros((nk, nw))
    V = np.zeros((nk, nw, nw), complex)
    vel = np.zeros((nk, nw, 3))
    for t in range(nk):
        H, dH = hk(system, pts[t] / N)
        w, v = np.linalg.eigh(H)
        eps[t], V[t] = w, v
        vel[t] = np.real(np.einsum("in,aij,jn->na", v.conj(), dH, v)) * VEL_UNIT
    return eps, V, vel


def phonons(system, N, omega_cut=1e-4):
    pts = grid_points(N)
    nq = pts.shape[0]
    nm = 3 * system.mass.shape[0]
    mass = np.repeat(system.mass, 3)
    om = np.zeros((nq, nm))
    u = np.zeros((nq, nm, nm), complex)  # u[q][mu][nu]
    for t in range(nq):
        lam, e = np.linalg.eigh(dq(system, pts[t] / N))
        hw = np.sqrt(CPH_EV * np.maximum(lam, 0.0))
        om[t] = hw
        for nu in range(nm):
            if hw[nu] >= omega_cut:
                u[t, :, nu] = e[:, nu] * np.sqrt(CPH_EV / (2.0 * mass * hw[nu]))
    return om, u


def vertex(system, N, kpt, qpt, Vk, Vp, uq):
    """g[m, n, nu] by the literal five-fold sum."""
    pe = np.exp(2j * math.pi * (system.re @ (kpt / N)))
    pp = np.exp(2j * math.pi * (system.rp @ (qpt / N)))
    gq = np.einsum("r,s,rsuij->uij", pe, pp, system.gw)
    return np.einsum("im,uij,jn,uv->mnv", Vp.conj(), gq, Vk, uq)


def rates(system, N, mu, temps, eta, states=None, omega_cut=1e-4):
    """1/tau[T][state] for states [(k_index, n)], all q, no sieve."""
    eps, V, vel = electrons(system, N)
    om, u = phonons(system, N, omega_cut)
    pts = grid_points(N)
    nw = system.nw
    if states is None:
        states = [(k, n) for k in range(N ** 3) for n in range(nw)]
    temps = np.asarray(temps, float)
    out = np.zeros((temps.shape[0], len(states)))
    pref = 2.0 * math.pi / HBAR_EVS / N ** 3
    for s, (k, n) in enumerate(states):
        for q in range(N ** 3):
            p = int(np.dot((pts[k] + pts[q]) % N, [1, N, N * N]))
            g = vertex(system, N, pts[k], pts[q], V[k], V[p], u[q])[:, n, :]
            g2 = np.abs(g) ** 2
            for nu in range(om.shape[1]):
                w = om[q, nu]
                if w < omega_cut:
                    continue
                for m in range(nw):
                    xp = eps[k, n] + w - eps[p, m]
                    xm = eps[k, n] - w - eps[p, m]
                    dp = math.exp(-(xp / eta) ** 2) / (math.sqrt(math.pi) * eta)
                    dm = math.exp(-(xm / eta) ** 2) / (math.sqrt(math.pi) * eta)
                    for t, T in enumerate(temps):
                        kt = KB_EVK * T
                        Nq = 1.0 / math.expm1(w / kt)
                        f = 1.0 / (math.exp((eps[p, m] - mu) / kt) + 1.0)
                        out[t, s] += pref * g2[m, nu] * ((Nq + f) * dp + (1.0 + Nq - f) * dm)
    return out, (eps, V, vel, om, u)
