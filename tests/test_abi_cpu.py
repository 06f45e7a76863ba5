"""C-ABI checks that need no GPU: the library loads, exports every symbol
that include/eph.h declares, and rejects invalid models before touching a
device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from synth import make_system
import paper_2306_16493_amd as pkg
from paper_2306_16493_amd import eph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "eph.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eph_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = eph.lib()
    syms = header_symbols()
    assert set(syms) == set(eph.EXPORTS)
    for s in syms:
        assert hasattr(L, s), s


def _model(system):
    ctx = object.__new__(eph.Context)
    # build the struct exactly as Context does, without loading
    keep = dict(mass=np.ascontiguousarray(system.mass, np.float64),
                rh=np.ascontiguousarray(system.rh, np.int32), rh_w=np.ascontiguousarray(system.rh_w, np.float64),
                ham=np.ascontiguousarray(system.ham, np.complex128),
                rd=np.ascontiguousarray(system.rd, np.int32), rd_w=np.ascontiguousarray(system.rd_w, np.float64),
                ifc=np.ascontiguousarray(system.ifc, np.float64),
                re=np.ascontiguousarray(system.re, np.int32), rp=np.ascontiguousarray(system.rp, np.int32),
                gw=np.ascontiguousarray(system.gw, np.complex128))
    m = eph.Model()
    for i, v in enumerate(np.asarray(system.lattice, np.float64).ravel()):
        m.lattice[i] = float(v)
    m.n_atoms = keep["mass"].shape[0]
    m.mass_amu = eph._ptr(keep["mass"])
    m.n_wann = int(system.nw)
    m.n_rh, m.rh, m.rh_w, m.ham = keep["rh"].shape[0], eph._ptr(keep["rh"]), eph._ptr(keep["rh_w"]), \
        eph._ptr(keep["ham"])
    m.n_rd, m.rd, m.rd_w, m.ifc = keep["rd"].shape[0], eph._ptr(keep["rd"]), eph._ptr(keep["rd_w"]), \
        eph._ptr(keep["ifc"])
    m.n_re, m.re, m.n_rp, m.rp, m.gw = keep["re"].shape[0], eph._ptr(keep["re"]), keep["rp"].shape[0], \
        eph._ptr(keep["rp"]), eph._ptr(keep["gw"])
    return m, keep


def _load(m):
    h = C.c_void_p()
    st = eph.lib().eph_load_wannier(C.byref(m), 0, C.byref(h))
    msg = eph.lib().eph_last_error(None).decode()
    if h:
        eph.lib().eph_free(h)
    return st, msg


def test_rejects_non_hermitian_h():
    s = make_system("toy_sc")
    s.ham = s.ham.copy()
    s.ham[3, 0, 1] += 0.1
    m, keep = _model(s)
    st, msg = _load(m)
    assert st == eph.EPH_E_INVALID and "H" in msg


def test_rejects_unclosed_r_set():
    s = make_system("toy_sc")
    s.rh = s.rh.copy()
    s.rh[0] = [7, 7, 7]
    m, keep = _model(s)
    st, msg = _load(m)
    assert st == eph.EPH_E_INVALID


def test_rejects_asymmetric_phi_and_bad_mass():
    s = make_system("toy_sc")
    s.ifc = s.ifc.copy()
    s.ifc[5, 0, 1] += 1.0
    m, keep = _model(s)
    assert _load(m)[0] == eph.EPH_E_INVALID
    s = make_system("toy_sc")
    s.mass = np.array([-1.0])
    m, keep = _model(s)
    assert _load(m)[0] == eph.EPH_E_INVALID


def test_rejects_non_box_rp_and_too_many_orbitals():
    s = make_system("toy_sc")
    s.rp = s.rp.copy()
    s.rp[0] = [9, 9, 9]
    m, keep = _model(s)
    assert _load(m)[0] == eph.EPH_E_UNSUPPORTED
    m, keep = _model(make_system("toy_sc"))
    m.n_wann = 9
    assert _load(m)[0] == eph.EPH_E_UNSUPPORTED


def test_null_arguments():
    L = eph.lib()
    h = C.c_void_p()
    assert L.eph_load_wannier(None, 0, C.byref(h)) == eph.EPH_E_INVALID
    m, keep = _model(make_system("toy_sc"))
    assert L.eph_load_wannier(C.byref(m), 0, None) == eph.EPH_E_INVALID
    L.eph_free(None)  # NULL-safe
    assert L.eph_scattering_rates(None, None, 0, None, None, None, None, None, None) == eph.EPH_E_INVALID
    assert L.eph_conductivity(None, 0, None, None, None, 0.0, 1, None, 1, None, None) == eph.EPH_E_INVALID
    assert L.eph_transport(None, 0, None, None, None, 0.0, 1, None, 1, None, None, None, None) == eph.EPH_E_INVALID
    t = np.array([300.0])
    out = np.zeros(1)
    assert L.eph_carrier_density(None, 4, 0, 0, 0.0, 1, t.ctypes.data_as(C.c_void_p), None,
                                 out.ctypes.data_as(C.c_void_p)) == eph.EPH_E_INVALID
    assert L.eph_mobility(0, None, None, None) == eph.EPH_E_INVALID
    assert L.eph_mlp_create(None, 5, 1, 0, None) == eph.EPH_E_INVALID
    assert L.eph_mlp_params(None, None, None, 0) == eph.EPH_E_INVALID
    assert L.eph_mlp_train(None, 0, None, None, 0, 0, 0.0, None, None) == eph.EPH_E_INVALID
    assert L.eph_mlp_predict(None, 0, None, None, None) == eph.EPH_E_INVALID
    assert L.eph_mlp_blend(None, 0, None, 0.0, None, None, None, None) == eph.EPH_E_INVALID


def test_valid_model_without_gpu_reports_device_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    m, keep = _model(make_system("toy_sc"))
    st, msg = _load(m)
    assert st in (eph.EPH_E_DEVICE, eph.EPH_OK)


def test_mobility_host_arithmetic():
    """eph_mobility is host arithmetic: mu = sigma / (n e), in cm^2/(V s)."""
    from paper_2306_16493_amd import mobility
    from paper_2306_16493_amd.eph import EphError
    sig = np.arange(18, dtype=np.float64).reshape(2, 3, 3) * 1e5
    n = np.array([1e24, 2e25])
    mu = mobility(sig, n)
    ref = sig / (n[:, None, None] * 1.602176634e-19) * 1e4
    assert np.allclose(mu, ref, rtol=1e-15, atol=0)
    with pytest.raises(EphError):
        mobility(sig, np.array([1e24, 0.0]))
