"""Python binding of the gfx950 EPWI library (argument marshalling only).

Every step of the computation runs in the HIP kernels of ``libeph.so``; this
module converts numpy model arrays to the C structs of ``include/eph.h`` and
passes torch device buffers (for memory and streams) through the C ABI.  If
the library is missing it raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("EPH_LIB", os.path.join(_HERE, "libeph.so"))

EPH_OK, EPH_E_INVALID, EPH_E_NOMEM, EPH_E_DEVICE, EPH_E_STATE, EPH_E_TRUNCATED, EPH_E_UNSUPPORTED = range(7)
EPH_FP64, EPH_FP32, EPH_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": EPH_FP64, "fp32": EPH_FP32, "bf16x3": EPH_BF16X3}
MAX_TEMPS = 4
MLP_FEATURES = 10  # inputs of the surrogate network (include/eph.h)

# every symbol declared in include/eph.h
EXPORTS = ("eph_load_wannier", "eph_free", "eph_last_error", "eph_scattering_rates", "eph_select_states",
           "eph_conductivity", "eph_conductivity_noalloc", "eph_transport", "eph_carrier_density", "eph_mobility",
           "eph_set_profiling", "eph_stage_times", "eph_mlp_create", "eph_mlp_free", "eph_mlp_params",
           "eph_mlp_features", "eph_mlp_train", "eph_mlp_gradient", "eph_mlp_predict", "eph_mlp_blend",
           "eph_merge_rates", "eph_gamma_estimate", "eph_rates_gamma", "eph_gamma_info", "eph_gamma_copy",
           "eph_gamma_free", "eph_bte_iterate", "eph_rates_kbatch")


class EphError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"eph status {code}: {msg}")
        self.code = code


class Model(C.Structure):
    _fields_ = [("lattice", C.c_double * 9), ("n_atoms", C.c_int32), ("mass_amu", C.c_void_p),
                ("n_wann", C.c_int32), ("n_rh", C.c_int32), ("rh", C.c_void_p), ("rh_w", C.c_void_p),
                ("ham", C.c_void_p), ("n_rd", C.c_int32), ("rd", C.c_void_p), ("rd_w", C.c_void_p),
                ("ifc", C.c_void_p), ("n_re", C.c_int32), ("re", C.c_void_p), ("n_rp", C.c_int32),
                ("rp", C.c_void_p), ("gw", C.c_void_p)]


class RatesParams(C.Structure):
    _fields_ = [("grid", C.c_int32 * 3), ("mu_eV", C.c_double), ("n_temps", C.c_int32),
                ("temps_K", C.c_void_p), ("eta_eV", C.c_double), ("sieve_width", C.c_double),
                ("win_lo_eV", C.c_double), ("win_hi_eV", C.c_double), ("band_lo", C.c_int32),
                ("band_hi", C.c_int32), ("omega_cut_eV", C.c_double), ("precision", C.c_int32),
                ("k_subset", C.c_void_p), ("n_k_subset", C.c_int64), ("mem_budget_bytes", C.c_int64),
                ("stream", C.c_void_p)]


class Counts(C.Structure):
    _fields_ = [("n_states", C.c_int64), ("n_kq", C.c_int64), ("n_nkq", C.c_int64), ("n_terms", C.c_int64),
                ("n_zero_rate", C.c_int64), ("n_excluded_modes", C.c_int64), ("n_vertex", C.c_int64)]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


_lib = None


def lib():
    """Load libeph.so (built in-tree by build.py); raise if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2306_16493_amd/build.py "
                              "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        L.eph_load_wannier.argtypes = [C.POINTER(Model), C.c_int32, C.POINTER(C.c_void_p)]
        L.eph_load_wannier.restype = C.c_int32
        L.eph_free.argtypes = [C.c_void_p]
        L.eph_free.restype = None
        L.eph_last_error.argtypes = [C.c_void_p]
        L.eph_last_error.restype = C.c_char_p
        L.eph_scattering_rates.argtypes = [C.c_void_p, C.POINTER(RatesParams), C.c_int64, C.c_void_p, C.c_void_p,
                                           C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(Counts)]
        L.eph_scattering_rates.restype = C.c_int32
        L.eph_select_states.argtypes = [C.c_void_p, C.POINTER(RatesParams), C.c_int64, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_void_p, C.POINTER(Counts)]
        L.eph_select_states.restype = C.c_int32
        L.eph_conductivity.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                       C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.eph_conductivity.restype = C.c_int32
        L.eph_conductivity_noalloc.argtypes = L.eph_conductivity.argtypes
        L.eph_conductivity_noalloc.restype = C.c_int32
        L.eph_set_profiling.argtypes = [C.c_void_p, C.c_int32]
        L.eph_set_profiling.restype = C.c_int32
        L.eph_stage_times.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.eph_stage_times.restype = C.c_int32
        vp, i32, i64, f32, f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
        L.eph_mlp_create.argtypes = [vp, i32, i32, C.c_uint64, C.POINTER(vp)]
        L.eph_mlp_free.argtypes = [vp]
        L.eph_mlp_free.restype = None
        L.eph_mlp_params.argtypes = [vp, vp, C.POINTER(i64), i32]
        L.eph_mlp_features.argtypes = [vp, i64, vp, vp, vp, i32, f64, vp, i32, vp, vp, vp]
        L.eph_mlp_train.argtypes = [vp, i64, vp, vp, i32, i32, f32, vp, vp]
        L.eph_mlp_gradient.argtypes = [vp, i64, vp, vp, vp, vp]
        L.eph_mlp_predict.argtypes = [vp, i64, vp, vp, vp]
        L.eph_mlp_blend.argtypes = [vp, i64, vp, f64, vp, vp, C.POINTER(i64), vp]
        L.eph_merge_rates.argtypes = [vp, i64, vp, vp, i64, vp, vp, vp, i32, vp, vp]
        L.eph_transport.argtypes = [vp, i64, vp, vp, vp, f64, i32, vp, i64, vp, vp, vp, vp]
        L.eph_carrier_density.argtypes = [vp, i32, i32, i32, f64, i32, vp, vp, vp]
        L.eph_mobility.argtypes = [i32, vp, vp, vp]
        L.eph_gamma_estimate.argtypes = [vp, C.POINTER(RatesParams), i64, vp, vp, vp, vp, C.POINTER(i64),
                                         C.POINTER(i64)]
        L.eph_rates_gamma.argtypes = [vp, C.POINTER(RatesParams), i64, vp, vp, vp, vp, vp, C.POINTER(Counts),
                                      C.POINTER(vp)]
        L.eph_gamma_info.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i32), C.POINTER(i32),
                                     C.POINTER(i64)]
        L.eph_gamma_copy.argtypes = [vp, vp, vp, vp]
        L.eph_gamma_free.argtypes = [vp]
        L.eph_gamma_free.restype = None
        L.eph_bte_iterate.argtypes = [vp, vp, vp, vp, vp, i64, i32, f64, vp, vp, C.POINTER(i32), vp]
        L.eph_rates_kbatch.argtypes = [vp, C.POINTER(RatesParams), i64, vp, vp, vp, vp, vp, C.POINTER(Counts), i32]
        for f in ("eph_gamma_estimate", "eph_rates_gamma", "eph_gamma_info", "eph_gamma_copy", "eph_bte_iterate",
                  "eph_rates_kbatch"):
            getattr(L, f).restype = C.c_int32
        for f in ("eph_mlp_create", "eph_mlp_params", "eph_mlp_features", "eph_mlp_train", "eph_mlp_gradient",
                  "eph_mlp_predict", "eph_mlp_blend", "eph_merge_rates", "eph_transport", "eph_carrier_density",
                  "eph_mobility"):
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


def _dptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


@dataclass
class RatesResult:
    state_k: "object"      # torch int32 [ns] on the device
    state_n: "object"
    energy: "object"       # float64 [ns]
    vel: "object"          # float64 [ns][3]
    inv_tau: "object"      # float64 [nt][ns]
    counts: dict


class Context:
    """An eph_ctx: the Wannier model resident on one GPU."""

    def __init__(self, system, device: int = 0):
        L = lib()
        self._keep = dict(
            mass=np.ascontiguousarray(system.mass, np.float64),
            rh=np.ascontiguousarray(system.rh, np.int32), rh_w=np.ascontiguousarray(system.rh_w, np.float64),
            ham=np.ascontiguousarray(system.ham, np.complex128),
            rd=np.ascontiguousarray(system.rd, np.int32), rd_w=np.ascontiguousarray(system.rd_w, np.float64),
            ifc=np.ascontiguousarray(system.ifc, np.float64),
            re=np.ascontiguousarray(system.re, np.int32), rp=np.ascontiguousarray(system.rp, np.int32),
            gw=np.ascontiguousarray(system.gw, np.complex128))
        k = self._keep
        m = Model()
        for i, v in enumerate(np.asarray(system.lattice, np.float64).ravel()):
            m.lattice[i] = float(v)
        m.n_atoms = k["mass"].shape[0]
        m.mass_amu = _ptr(k["mass"])
        m.n_wann = int(system.nw)
        m.n_rh, m.rh, m.rh_w, m.ham = k["rh"].shape[0], _ptr(k["rh"]), _ptr(k["rh_w"]), _ptr(k["ham"])
        m.n_rd, m.rd, m.rd_w, m.ifc = k["rd"].shape[0], _ptr(k["rd"]), _ptr(k["rd_w"]), _ptr(k["ifc"])
        m.n_re, m.re, m.n_rp, m.rp, m.gw = k["re"].shape[0], _ptr(k["re"]), k["rp"].shape[0], _ptr(k["rp"]), \
            _ptr(k["gw"])
        self._model = m
        h = C.c_void_p()
        st = L.eph_load_wannier(C.byref(m), int(device), C.byref(h))
        if st != EPH_OK:
            raise EphError(st, L.eph_last_error(None).decode())
        self._h = h
        self.device = device
        self.nw = int(system.nw)
        self.nm = 3 * k["mass"].shape[0]
        del self._keep["gw"]  # copied to the device; the host copy is not needed any more

    def close(self):
        if getattr(self, "_h", None):
            lib().eph_free(self._h)
            self._h = None

    __del__ = close

    def last_error(self):
        return lib().eph_last_error(self._h).decode()

    def _check(self, st, allow=()):
        if st != EPH_OK and st not in allow:
            raise EphError(st, self.last_error())
        return st

    @staticmethod
    def params(grid, mu, temps, eta, win_lo, win_hi, band_lo=0, band_hi=-1, sieve_width=6.0,
               omega_cut=1e-4, precision="fp64", k_subset=None, stream=None, mem_budget_bytes=0):
        p = RatesParams()
        p.grid[0] = p.grid[1] = p.grid[2] = int(grid)
        p.mu_eV = float(mu)
        temps = np.ascontiguousarray(np.atleast_1d(temps), np.float64)
        p.n_temps = temps.shape[0]
        p.temps_K = _ptr(temps)
        p.eta_eV, p.sieve_width = float(eta), float(sieve_width)
        p.win_lo_eV, p.win_hi_eV = float(win_lo), float(win_hi)
        p.band_lo, p.band_hi = int(band_lo), int(band_hi)
        p.omega_cut_eV = float(omega_cut)
        p.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        keep = [temps]
        if k_subset is not None:
            ks = np.ascontiguousarray(k_subset, np.int64)
            n = ks.shape[0]
            if n == 0:
                ks = np.zeros(1, np.int64)  # a valid pointer with zero entries
            keep.append(ks)
            p.k_subset, p.n_k_subset = _ptr(ks), n
        else:
            p.k_subset, p.n_k_subset = None, 0
        p.mem_budget_bytes = int(mem_budget_bytes)
        p.stream = C.c_void_p(stream) if stream else None
        p._keep = keep
        return p

    def count_states(self, params) -> int:
        cnt = Counts()
        st = lib().eph_scattering_rates(self._h, C.byref(params), 0, None, None, None, None, None, C.byref(cnt))
        self._check(st, allow=(EPH_E_TRUNCATED,))
        return int(cnt.n_states)

    def scattering_rates(self, params, capacity: Optional[int] = None, buffers=None) -> RatesResult:
        """Run eph_scattering_rates into torch device buffers (allocated here
        unless given as a dict from a previous result)."""
        import torch
        dev = torch.device("cuda", self.device)
        if capacity is None:
            capacity = self.count_states(params)
        nt = int(params.n_temps)
        cap = max(int(capacity), 1)
        if buffers is None:
            buffers = dict(k=torch.empty(cap, dtype=torch.int32, device=dev),
                           n=torch.empty(cap, dtype=torch.int32, device=dev),
                           e=torch.empty(cap, dtype=torch.float64, device=dev),
                           v=torch.empty(cap, 3, dtype=torch.float64, device=dev),
                           it=torch.empty(nt * cap, dtype=torch.float64, device=dev))
        cnt = Counts()
        st = lib().eph_scattering_rates(self._h, C.byref(params), int(capacity), _dptr(buffers["k"]),
                                        _dptr(buffers["n"]), _dptr(buffers["e"]), _dptr(buffers["v"]),
                                        _dptr(buffers["it"]), C.byref(cnt))
        self._check(st)
        ns = int(cnt.n_states)
        return RatesResult(buffers["k"][:ns], buffers["n"][:ns], buffers["e"][:ns], buffers["v"][:ns],
                           buffers["it"][:nt * ns].view(nt, ns), cnt.as_dict()), buffers

    def set_profiling(self, on=True):
        self._check(lib().eph_set_profiling(self._h, 1 if on else 0))

    def stage_times(self):
        ms = np.zeros(5)
        ln = np.zeros(2, np.int64)
        self._check(lib().eph_stage_times(self._h, _ptr(ms), _ptr(ln)))
        return dict(tables_ms=ms[0], prep_ms=ms[1], xform_ms=ms[2], rates_ms=ms[3], call_ms=ms[4],
                    xform_launches=int(ln[0]), rates_launches=int(ln[1]))

    def select_states(self, params):
        """(state_k, state_n, energy, vel) device tensors of the window states."""
        import torch
        dev = torch.device("cuda", self.device)
        ns = self.count_states(params)
        cap = max(ns, 1)
        k = torch.empty(cap, dtype=torch.int32, device=dev)
        n = torch.empty(cap, dtype=torch.int32, device=dev)
        e = torch.empty(cap, dtype=torch.float64, device=dev)
        v = torch.empty(cap, 3, dtype=torch.float64, device=dev)
        cnt = Counts()
        self._check(lib().eph_select_states(self._h, C.byref(params), ns, _dptr(k), _dptr(n), _dptr(e), _dptr(v),
                                            C.byref(cnt)))
        return k[:ns], n[:ns], e[:ns], v[:ns]

    def conductivity(self, energy, vel, inv_tau, mu, temps, n_kpoints, stream=None, noalloc=False):
        """sigma [nt][3][3] in S/m; noalloc=True calls eph_conductivity_noalloc
        (static device workspace, no allocation in the call)."""
        temps = np.ascontiguousarray(np.atleast_1d(temps), np.float64)
        out = np.zeros((temps.shape[0], 3, 3))
        ns = int(energy.shape[0])
        fn = lib().eph_conductivity_noalloc if noalloc else lib().eph_conductivity
        st = fn(self._h, ns, _dptr(energy.contiguous()), _dptr(vel.contiguous()),
                                    _dptr(inv_tau.contiguous()), float(mu), temps.shape[0], _ptr(temps),
                                    int(n_kpoints), C.c_void_p(stream) if stream else None, _ptr(out))
        self._check(st)
        return out


def _conductivity_args(energy, vel, inv_tau):
    return energy.contiguous(), vel.contiguous(), inv_tau.contiguous()


class _Transport:
    """Transport coefficients of a Context (mixed into Context below)."""

    def transport(self, energy, vel, inv_tau, mu, temps, n_kpoints, stream=None):
        """(sigma S/m, Seebeck V/K, electronic kappa W/(m K)), each [nt][3][3]."""
        temps = np.ascontiguousarray(np.atleast_1d(temps), np.float64)
        nt = temps.shape[0]
        sig, see, kap = np.zeros((nt, 3, 3)), np.zeros((nt, 3, 3)), np.zeros((nt, 3, 3))
        e, v, it = _conductivity_args(energy, vel, inv_tau)
        st = lib().eph_transport(self._h, int(energy.shape[0]), _dptr(e), _dptr(v), _dptr(it), float(mu), nt,
                                 _ptr(temps), int(n_kpoints), C.c_void_p(stream) if stream else None, _ptr(sig),
                                 _ptr(see), _ptr(kap))
        self._check(st)
        return sig, see, kap

    def carrier_density(self, grid, band_lo, band_hi, mu, temps, stream=None):
        """n(T) in m^-3 over bands band_lo..band_hi of the full grid."""
        temps = np.ascontiguousarray(np.atleast_1d(temps), np.float64)
        out = np.zeros(temps.shape[0])
        st = lib().eph_carrier_density(self._h, int(grid), int(band_lo), int(band_hi), float(mu), temps.shape[0],
                                       _ptr(temps), C.c_void_p(stream) if stream else None, _ptr(out))
        self._check(st)
        return out


def mobility(sigma, n_per_m3):
    """sigma [nt][3][3] (S/m) and n [nt] (m^-3) -> mobility [nt][3][3] in cm^2/(V s)."""
    sigma = np.ascontiguousarray(sigma, np.float64)
    n = np.ascontiguousarray(np.atleast_1d(n_per_m3), np.float64)
    out = np.zeros_like(sigma)
    st = lib().eph_mobility(n.shape[0], _ptr(sigma), _ptr(n), _ptr(out))
    if st != 0:
        raise EphError(st, "eph_mobility: densities must be positive")
    return out


class Gamma:
    """Transition rates of the iterative BTE (an eph_gamma handle)."""

    def __init__(self, ctx, handle):
        self.ctx, self._h = ctx, handle

    def info(self):
        ns, nnz, nt, host, b = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32(), C.c_int64()
        self.ctx._check(lib().eph_gamma_info(self._h, C.byref(ns), C.byref(nnz), C.byref(nt), C.byref(host),
                                             C.byref(b)))
        return dict(n_states=ns.value, nnz=nnz.value, n_temps=nt.value, on_host=bool(host.value), bytes=b.value)

    def rows(self):
        """(row_start [ns+1], col [nnz], val [nt][nnz]) as numpy arrays."""
        i = self.info()
        rs = np.zeros(i["n_states"] + 1, np.int64)
        col = np.zeros(max(i["nnz"], 1), np.int32)
        val = np.zeros((i["n_temps"], max(i["nnz"], 1)))
        self.ctx._check(lib().eph_gamma_copy(self._h, _ptr(rs), _ptr(col), _ptr(val)))
        return rs, col[:i["nnz"]], val[:, :i["nnz"]]

    def close(self):
        if getattr(self, "_h", None):
            lib().eph_gamma_free(self._h)
            self._h = None

    __del__ = close


class _Bte:
    """Iterative BTE entry points of a Context (mixed into Context below)."""

    def gamma_estimate(self, params):
        """(n_states, nnz, bytes) of the transition rates, from the sieve only."""
        import torch
        dev = torch.device("cuda", self.device)
        ns = self.count_states(params)
        cap = max(ns, 1)
        k = torch.empty(cap, dtype=torch.int32, device=dev)
        n = torch.empty(cap, dtype=torch.int32, device=dev)
        e = torch.empty(cap, dtype=torch.float64, device=dev)
        v = torch.empty(cap, 3, dtype=torch.float64, device=dev)
        nnz, b = C.c_int64(), C.c_int64()
        self._check(lib().eph_gamma_estimate(self._h, C.byref(params), ns, _dptr(k), _dptr(n), _dptr(e), _dptr(v),
                                             C.byref(nnz), C.byref(b)))
        return ns, nnz.value, b.value

    def rates_gamma(self, params):
        """eph_scattering_rates plus the transition rates: (RatesResult, Gamma)."""
        import torch
        dev = torch.device("cuda", self.device)
        ns = self.count_states(params)
        nt = int(params.n_temps)
        cap = max(ns, 1)
        bufs = dict(k=torch.empty(cap, dtype=torch.int32, device=dev),
                    n=torch.empty(cap, dtype=torch.int32, device=dev),
                    e=torch.empty(cap, dtype=torch.float64, device=dev),
                    v=torch.empty(cap, 3, dtype=torch.float64, device=dev),
                    it=torch.empty(nt * cap, dtype=torch.float64, device=dev))
        cnt = Counts()
        h = C.c_void_p()
        self._check(lib().eph_rates_gamma(self._h, C.byref(params), ns, _dptr(bufs["k"]), _dptr(bufs["n"]),
                                          _dptr(bufs["e"]), _dptr(bufs["v"]), _dptr(bufs["it"]), C.byref(cnt),
                                          C.byref(h)))
        res = RatesResult(bufs["k"][:ns], bufs["n"][:ns], bufs["e"][:ns], bufs["v"][:ns],
                          bufs["it"][:nt * ns].view(nt, ns), cnt.as_dict())
        return res, Gamma(self, h)

    def rates_kbatch(self, params, q_batch=256, buffers=None):
        """eph_rates_kbatch: the rates in the k-batch order (RatesResult, buffers)."""
        import torch
        dev = torch.device("cuda", self.device)
        ns = self.count_states(params)
        nt = int(params.n_temps)
        cap = max(ns, 1)
        if buffers is None:
            buffers = dict(k=torch.empty(cap, dtype=torch.int32, device=dev),
                           n=torch.empty(cap, dtype=torch.int32, device=dev),
                           e=torch.empty(cap, dtype=torch.float64, device=dev),
                           v=torch.empty(cap, 3, dtype=torch.float64, device=dev),
                           it=torch.empty(nt * cap, dtype=torch.float64, device=dev))
        cnt = Counts()
        self._check(lib().eph_rates_kbatch(self._h, C.byref(params), ns, _dptr(buffers["k"]), _dptr(buffers["n"]),
                                           _dptr(buffers["e"]), _dptr(buffers["v"]), _dptr(buffers["it"]),
                                           C.byref(cnt), int(q_batch)))
        return RatesResult(buffers["k"][:ns], buffers["n"][:ns], buffers["e"][:ns], buffers["v"][:ns],
                           buffers["it"][:nt * ns].view(nt, ns), cnt.as_dict()), buffers

    def bte_iterate(self, gamma, res, n_kpoints, max_iter=20, tol=1e-6, want_f=False, stream=None):
        """(sigma per iteration [n_done+1][nt][3][3], n_done, F or None)."""
        import torch
        nt = int(res.inv_tau.shape[0])
        ns = int(res.energy.shape[0])
        sig = np.zeros((max_iter + 1, nt, 3, 3))
        nd = C.c_int32()
        F = torch.empty((nt, max(ns, 1), 3), dtype=torch.float64, device=res.energy.device) if want_f else None
        self._check(lib().eph_bte_iterate(self._h, gamma._h, _dptr(res.energy.contiguous()),
                                          _dptr(res.vel.contiguous()), _dptr(res.inv_tau.contiguous()),
                                          int(n_kpoints), int(max_iter), float(tol),
                                          C.c_void_p(stream) if stream else None, _ptr(sig), C.byref(nd),
                                          _dptr(F) if F is not None else None))
        return sig[:nd.value + 1], nd.value, (F[:, :ns] if F is not None else None)


for _name in ("transport", "carrier_density"):
    setattr(Context, _name, getattr(_Transport, _name))
for _name in ("gamma_estimate", "rates_gamma", "bte_iterate", "rates_kbatch"):
    setattr(Context, _name, getattr(_Bte, _name))


class Mlp:
    """An eph_mlp ensemble bound to a Context (device buffers are torch tensors)."""

    def __init__(self, ctx: Context, members: int = 5, n_out: int = 1, seed: int = 0):
        h = C.c_void_p()
        st = lib().eph_mlp_create(ctx._h, int(members), int(n_out), C.c_uint64(seed), C.byref(h))
        ctx._check(st)
        self._h, self.ctx, self.members, self.n_out = h, ctx, int(members), int(n_out)
        n = C.c_int64()
        ctx._check(lib().eph_mlp_params(h, None, C.byref(n), 0))
        self.n_params = int(n.value)

    def close(self):
        if getattr(self, "_h", None):
            lib().eph_mlp_free(self._h)
            self._h = None

    __del__ = close

    def get_params(self):
        out = np.zeros((self.members, self.n_params), np.float32)
        self.ctx._check(lib().eph_mlp_params(self._h, _ptr(out), None, 0))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, np.float32)
        self.ctx._check(lib().eph_mlp_params(self._h, _ptr(p), None, 1))

    def features(self, state_k, energy, vel, grid, mu, inv_tau=None, stream=None):
        import torch
        n = int(state_k.shape[0])
        dev = state_k.device
        x = torch.empty((max(n, 1), MLP_FEATURES), dtype=torch.float32, device=dev)
        y = None
        nt = 0
        if inv_tau is not None:
            nt = int(inv_tau.shape[0])
            y = torch.empty((max(n, 1), nt), dtype=torch.float32, device=dev)
        st = lib().eph_mlp_features(self.ctx._h, n, _dptr(state_k), _dptr(energy.contiguous()),
                                    _dptr(vel.contiguous()), int(grid), float(mu),
                                    _dptr(inv_tau.contiguous()) if inv_tau is not None else None, nt,
                                    _dptr(x), _dptr(y), C.c_void_p(stream) if stream else None)
        self.ctx._check(st)
        return x[:n], (y[:n] if y is not None else None)

    def train(self, x, y, steps, batch=256, lr=1e-3, stream=None):
        loss = np.zeros(self.members, np.float32)
        st = lib().eph_mlp_train(self._h, int(x.shape[0]), _dptr(x), _dptr(y), int(steps), int(batch),
                                 float(lr), C.c_void_p(stream) if stream else None, _ptr(loss))
        self.ctx._check(st)
        return loss

    def gradient(self, x, y):
        g = np.zeros((self.members, self.n_params), np.float32)
        loss = np.zeros(self.members, np.float32)
        self.ctx._check(lib().eph_mlp_gradient(self._h, int(x.shape[0]), _dptr(x), _dptr(y), _ptr(g), _ptr(loss)))
        return loss, g

    def predict(self, x, stream=None):
        import torch
        n = int(x.shape[0])
        y = torch.empty((self.members, max(n, 1), self.n_out), dtype=torch.float32, device=x.device)
        self.ctx._check(lib().eph_mlp_predict(self._h, n, _dptr(x), _dptr(y), C.c_void_p(stream) if stream else None))
        return y[:, :n]

    def blend(self, y, threshold, stream=None):
        import torch
        n = int(y.shape[1])
        it = torch.empty((self.n_out, max(n, 1)), dtype=torch.float64, device=y.device)
        flag = torch.empty(max(n, 1), dtype=torch.int32, device=y.device)
        nf = C.c_int64()
        self.ctx._check(lib().eph_mlp_blend(self._h, n, _dptr(y.contiguous()), float(threshold), _dptr(it),
                                            _dptr(flag), C.byref(nf), C.c_void_p(stream) if stream else None))
        return it[:, :n], flag[:n], int(nf.value)


def merge_rates(ctx: Context, full_k, full_n, full_inv_tau, sub_k, sub_n, sub_inv_tau, stream=None):
    """full_inv_tau[:, i] <- sub_inv_tau[:, j] where the (k, n) match (in place)."""
    nt = int(full_inv_tau.shape[0])
    st = lib().eph_merge_rates(ctx._h, int(full_k.shape[0]), _dptr(full_k), _dptr(full_n), int(sub_k.shape[0]),
                               _dptr(sub_k), _dptr(sub_n), _dptr(sub_inv_tau.contiguous()), nt,
                               _dptr(full_inv_tau), C.c_void_p(stream) if stream else None)
    ctx._check(st)
