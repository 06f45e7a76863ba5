"""FP64 CPU oracle for the EPWI SERTA transport path (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never does, and the
oracle shares no code with it.

The arithmetic lives in ``eph_oracle.c`` (plain C, FP64, OpenMP over k
points); this module only marshals numpy arrays through ctypes and does the
state selection of the paper's preprocessing step (states in an energy
window, Sec. III.A) in plain numpy.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "eph_oracle.c")


def build(force: bool = True) -> str:
    """Compile the oracle (gcc, -O2, IEEE arithmetic, OpenMP)."""
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               "-o", _LIB, _SRC, "-lm"])
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        for f in ("orc_hbar_evs", "orc_kb_evk", "orc_cph_ev", "orc_vel_unit"):
            getattr(_lib, f).restype = C.c_double
        _lib.orc_delta.restype = C.c_double
        _lib.orc_delta.argtypes = [C.c_double, C.c_double]
    return _lib


class _Model(C.Structure):
    _fields_ = [("lattice", C.c_double * 9), ("na", C.c_int32), ("mass", C.c_void_p),
                ("nw", C.c_int32), ("nrh", C.c_int32), ("rh", C.c_void_p), ("rh_w", C.c_void_p),
                ("ham", C.c_void_p), ("nrd", C.c_int32), ("rd", C.c_void_p), ("rd_w", C.c_void_p),
                ("ifc", C.c_void_p), ("nre", C.c_int32), ("re", C.c_void_p), ("nrp", C.c_int32),
                ("rp", C.c_void_p), ("gw", C.c_void_p)]


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _i64(x):
    return C.c_int64(int(x))


class Oracle:
    """Wraps one model system (a ``synth.System`` or any object with the same
    attributes)."""

    def __init__(self, system):
        self.sys = system
        self._keep = dict(
            mass=np.ascontiguousarray(system.mass, np.float64),
            rh=np.ascontiguousarray(system.rh, np.int32),
            rh_w=np.ascontiguousarray(system.rh_w, np.float64),
            ham=np.ascontiguousarray(system.ham, np.complex128),
            rd=np.ascontiguousarray(system.rd, np.int32),
            rd_w=np.ascontiguousarray(system.rd_w, np.float64),
            ifc=np.ascontiguousarray(system.ifc, np.float64),
            re=np.ascontiguousarray(system.re, np.int32),
            rp=np.ascontiguousarray(system.rp, np.int32),
            gw=np.ascontiguousarray(system.gw, np.complex128),
        )
        k = self._keep
        m = _Model()
        for i, v in enumerate(np.asarray(system.lattice, np.float64).ravel()):
            m.lattice[i] = v
        m.na = int(k["mass"].shape[0])
        m.mass = _p(k["mass"])
        m.nw = int(system.nw)
        m.nrh, m.rh, m.rh_w, m.ham = k["rh"].shape[0], _p(k["rh"]), _p(k["rh_w"]), _p(k["ham"])
        m.nrd, m.rd, m.rd_w, m.ifc = k["rd"].shape[0], _p(k["rd"]), _p(k["rd_w"]), _p(k["ifc"])
        m.nre, m.re, m.nrp, m.rp, m.gw = (k["re"].shape[0], _p(k["re"]), k["rp"].shape[0],
                                          _p(k["rp"]), _p(k["gw"]))
        self.model = m
        self.nw = int(system.nw)
        self.nm = 3 * m.na
        self.volume = float(abs(np.linalg.det(np.asarray(system.lattice))))

    # -- constants ------------------------------------------------------
    @staticmethod
    def constants():
        L = lib()
        return dict(hbar_evs=L.orc_hbar_evs(), kb_evk=L.orc_kb_evk(), cph_ev=L.orc_cph_ev(),
                    vel_unit=L.orc_vel_unit())

    # -- grid tables ----------------------------------------------------
    def electrons(self, N, kidx=None):
        if kidx is None:
            kidx = np.arange(N ** 3, dtype=np.int64)
        kidx = np.ascontiguousarray(kidx, np.int64)
        nk = kidx.shape[0]
        eps = np.zeros((nk, self.nw))
        evec = np.zeros((nk, self.nw, self.nw), np.complex128)
        vel = np.zeros((nk, self.nw, 3))
        lib().orc_electrons(C.byref(self.model), _i64(N), _i64(nk), _p(kidx), _p(eps), _p(evec), _p(vel))
        return eps, evec, vel

    def phonons(self, N, qidx=None, omega_cut=1e-4):
        if qidx is None:
            qidx = np.arange(N ** 3, dtype=np.int64)
        qidx = np.ascontiguousarray(qidx, np.int64)
        nq = qidx.shape[0]
        om = np.zeros((nq, self.nm))
        u = np.zeros((nq, self.nm, self.nm), np.complex128)
        lam = np.zeros((nq, self.nm))
        lib().orc_phonons(C.byref(self.model), _i64(N), _i64(nq), _p(qidx), C.c_double(omega_cut),
                          _p(om), _p(u), _p(lam))
        return om, u, lam

    def vertex(self, N, kidx, qidx, evec_k, evec_p, u_q):
        """g[m][n][nu] at one (k,q) from the given eigenvector/displacement
        rows (evec_k = V(k), evec_p = V(k+q), u_q = u(q))."""
        out = np.zeros((self.nw, self.nw, self.nm), np.complex128)
        ek = np.ascontiguousarray(evec_k, np.complex128)
        ep = np.ascontiguousarray(evec_p, np.complex128)
        uq = np.ascontiguousarray(u_q, np.complex128)
        lib().orc_vertex(C.byref(self.model), _i64(N), _i64(kidx), _i64(qidx), _p(ek), _p(ep), _p(uq),
                         _p(out))
        return out

    # -- states, rates, sigma --------------------------------------------
    @staticmethod
    def select_states(eps, band_lo, band_hi, win_lo, win_hi, k_subset=None):
        """States (k, n) with band_lo <= n <= band_hi and win_lo <= eps <= win_hi,
        sorted by k then n.  eps is the full-grid table [N^3][nw]."""
        nw = eps.shape[1]
        if band_hi < 0:
            band_hi = nw - 1
        ks = np.arange(eps.shape[0]) if k_subset is None else np.unique(np.asarray(k_subset, np.int64))
        sub = eps[ks]
        bands = np.arange(nw)
        ok = (sub >= win_lo) & (sub <= win_hi) & (bands >= band_lo)[None, :] & (bands <= band_hi)[None, :]
        kk, nn = np.nonzero(ok)
        return ks[kk].astype(np.int32), nn.astype(np.int32)

    def rates(self, N, eps, evec, omega, u, state_k, state_n, mu, temps, eta, sw=6.0, omega_cut=1e-4):
        state_k = np.ascontiguousarray(state_k, np.int32)
        state_n = np.ascontiguousarray(state_n, np.int32)
        ns = state_k.shape[0]
        temps = np.ascontiguousarray(temps, np.float64)
        nt = temps.shape[0]
        it = np.zeros((nt, ns))
        nqv = np.zeros(ns, np.int64)
        nte = np.zeros(ns, np.int64)
        nkq = np.zeros(1, np.int64)
        eps = np.ascontiguousarray(eps, np.float64)
        evec = np.ascontiguousarray(evec, np.complex128)
        omega = np.ascontiguousarray(omega, np.float64)
        u = np.ascontiguousarray(u, np.complex128)
        lib().orc_rates(C.byref(self.model), _i64(N), _p(eps), _p(evec), _p(omega), _p(u), _i64(ns),
                        _p(state_k), _p(state_n), C.c_double(mu), C.c_int32(nt), _p(temps),
                        C.c_double(eta), C.c_double(sw), C.c_double(omega_cut), _p(it), _p(nqv),
                        _p(nte), _p(nkq))
        return dict(inv_tau=it, n_q_valid=nqv, n_terms=nte, n_kq=int(nkq[0]))

    def gamma(self, N, eps, evec, omega, u, state_k, state_n, mu, temps, eta, sw=6.0, omega_cut=1e-4):
        """Transition rates of the iterative BTE: row_start [ns+1], fin [nnz]
        (final state p*nw + m), val [nnz][nt] (1/s), rows in state order."""
        state_k = np.ascontiguousarray(state_k, np.int32)
        state_n = np.ascontiguousarray(state_n, np.int32)
        ns = state_k.shape[0]
        temps = np.ascontiguousarray(temps, np.float64)
        nt = temps.shape[0]
        assert nt <= 8
        eps = np.ascontiguousarray(eps, np.float64)
        evec = np.ascontiguousarray(evec, np.complex128)
        omega = np.ascontiguousarray(omega, np.float64)
        u = np.ascontiguousarray(u, np.complex128)
        rs = np.zeros(ns + 1, np.int64)
        L = lib()
        L.orc_gamma.restype = C.c_int64
        args = lambda fin, val: (C.byref(self.model), _i64(N), _p(eps), _p(evec), _p(omega), _p(u), _i64(ns),
                                 _p(state_k), _p(state_n), C.c_double(mu), C.c_int32(nt), _p(temps),
                                 C.c_double(eta), C.c_double(sw), C.c_double(omega_cut), _p(rs), fin, val)
        nnz = L.orc_gamma(*args(None, None))
        fin = np.zeros(max(nnz, 1), np.int64)
        val = np.zeros((max(nnz, 1), nt))
        L.orc_gamma(*args(_p(fin), _p(val)))
        return dict(row_start=rs, fin=fin[:nnz], val=val[:nnz])

    def bte(self, N, state_k, state_n, energy, vel, inv_tau, gamma, mu, temps, nk_total, n_iter):
        """Iterative BTE from the SERTA start F0 = v tau: sigma after every
        iteration [n_iter+1][nt][3][3] and the final F [nt][ns][3]."""
        state_k = np.ascontiguousarray(state_k, np.int32)
        state_n = np.ascontiguousarray(state_n, np.int32)
        energy = np.ascontiguousarray(energy, np.float64)
        vel = np.ascontiguousarray(vel, np.float64)
        inv_tau = np.ascontiguousarray(inv_tau, np.float64)
        temps = np.ascontiguousarray(temps, np.float64)
        ns, nt = state_k.shape[0], temps.shape[0]
        rs = np.ascontiguousarray(gamma["row_start"], np.int64)
        fin = np.ascontiguousarray(gamma["fin"], np.int64)
        val = np.ascontiguousarray(gamma["val"], np.float64)
        assert val.shape[1:] == (nt,)
        sig = np.zeros((n_iter + 1, nt, 3, 3))
        F = np.zeros((nt, ns, 3))
        lib().orc_bte(_i64(N), C.c_int(self.nw), _i64(ns), _p(state_k), _p(state_n), _p(energy), _p(vel),
                      _p(inv_tau), _p(rs), _p(fin), _p(val), C.c_double(mu), C.c_int32(nt), _p(temps),
                      _i64(nk_total), C.c_double(self.volume), C.c_int32(n_iter), _p(sig), _p(F))
        return sig, F

    def sigma(self, energy, vel, inv_tau, mu, temps, nk_total):
        energy = np.ascontiguousarray(energy, np.float64)
        vel = np.ascontiguousarray(vel, np.float64)
        inv_tau = np.ascontiguousarray(inv_tau, np.float64)
        temps = np.ascontiguousarray(temps, np.float64)
        ns, nt = energy.shape[0], temps.shape[0]
        out = np.zeros((nt, 3, 3))
        lib().orc_sigma(_i64(ns), _p(energy), _p(vel), _p(inv_tau), C.c_double(mu), C.c_int32(nt),
                        _p(temps), _i64(nk_total), C.c_double(self.volume), _p(out))
        return out

    def transport(self, energy, vel, inv_tau, mu, temps, nk_total):
        """(sigma S/m, Seebeck V/K, electronic thermal conductivity W/(m K)),
        each [nt][3][3], from the moments of the SERTA sum."""
        energy = np.ascontiguousarray(energy, np.float64)
        vel = np.ascontiguousarray(vel, np.float64)
        inv_tau = np.ascontiguousarray(inv_tau, np.float64)
        temps = np.ascontiguousarray(temps, np.float64)
        ns, nt = energy.shape[0], temps.shape[0]
        sig, see, kap = np.zeros((nt, 3, 3)), np.zeros((nt, 3, 3)), np.zeros((nt, 3, 3))
        lib().orc_transport(_i64(ns), _p(energy), _p(vel), _p(inv_tau), C.c_double(mu), C.c_int32(nt), _p(temps),
                            _i64(nk_total), C.c_double(self.volume), _p(sig), _p(see), _p(kap))
        return sig, see, kap

    def carrier_density(self, eps, band_lo, band_hi, mu, temps):
        eps = np.ascontiguousarray(eps, np.float64)
        temps = np.ascontiguousarray(temps, np.float64)
        out = np.zeros(temps.shape[0])
        lib().orc_carrier_density(_i64(eps.shape[0]), C.c_int(eps.shape[1]), _p(eps), C.c_int(band_lo),
                                  C.c_int(band_hi), C.c_double(mu), C.c_int32(temps.shape[0]), _p(temps),
                                  C.c_double(self.volume), _p(out))
        return out

    # -- whole path --------------------------------------------------------
    def run(self, N, mu, temps, eta, win_lo, win_hi, band_lo=0, band_hi=-1, k_subset=None, sw=6.0,
            omega_cut=1e-4, tables=None):
        """Electrons and phonons on the full grid, states, 1/tau, sigma."""
        if tables is None:
            eps, evec, vel = self.electrons(N)
            om, u, _ = self.phonons(N, omega_cut=omega_cut)
        else:
            eps, evec, vel, om, u = tables
        sk, sn = self.select_states(eps, band_lo, band_hi, win_lo, win_hi, k_subset)
        r = self.rates(N, eps, evec, om, u, sk, sn, mu, temps, eta, sw, omega_cut)
        energy = eps[sk, sn]
        v = vel[sk, sn]
        sig = self.sigma(energy, v, r["inv_tau"], mu, temps, N ** 3)
        r.update(state_k=sk, state_n=sn, energy=energy, vel=v, sigma=sig,
                 tables=(eps, evec, vel, om, u))
        return r
