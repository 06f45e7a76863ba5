"""Seeded synthetic model systems standing in for EPW Wannier data.

The paper runs on Quantum-ESPRESSO/EPW data for Al and Si (Sec. IV); that
data is not available, so these generators draw random model parameters with
the same shapes: the Wannier Hamiltonian H(R) (Sec. II.B, Wannier
interpolation of H), the interatomic force constants Phi(R) (dynamical-matrix
interpolation), and the el-ph vertex g_ij^mu(Re,Rp) in the Wannier basis
(interpolation formula of g).

Conventions (all arrays numpy, C order):
  lattice   [3][3]   rows a1,a2,a3 in Angstrom
  tau       [na][3]  atomic positions, Cartesian Angstrom
  mass      [na]     amu
  rh        [n_rh][3] int lattice coordinates of the H vectors, rh_w weights
  ham       [n_rh][nw][nw] complex128, eV;  H(-R) = H(R)^dagger
  rd, rd_w  D vectors and weights
  ifc       [n_rd][3na][3na] float64, eV/A^2, index (kappa*3+alpha);
            Phi(-R) = Phi(R)^T, built from springs so the acoustic sum rule
            holds exactly and every D(q) is positive semidefinite
  re, rp    [n][3] int lattice coordinates of the g vectors
  gw        [n_re][n_rp][3na][nw(i)][nw(j)] complex128, eV/A

Readings (also listed in the design notes):
  * g vectors: an n^3 box {-floor((n-1)/2) .. ceil((n-1)/2)}^3.
  * H and D vectors: {-n/2 .. n/2}^3 with weight 1/2 per coordinate at
    +-n/2, so the set is closed under R -> -R and sum(w) = n^3.
  * |R| in the decay factors is the Cartesian length in Angstrom.
  * The force-constant scale is set from a q-independent Gershgorin bound
    on the dynamical matrix, so that no phonon frequency exceeds 40 meV;
    the generator never diagonalises anything.
  * The chemical potential "at mid-band" of the metals is the band-energy
    centroid tr H(R=0) / nw, which equals the mean of all band energies on
    any full Gamma-centred grid.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Exact SI (2019) constants, used here only to set the force-constant scale.
_H_PLANCK = 6.62607015e-34
_E_CHARGE = 1.602176634e-19
_AMU = 1.66053906892e-27


def _c_phonon_ev() -> float:
    """hbar^2 / (amu * A^2) in eV, the (hbar omega)^2 unit of eV/(A^2 amu)."""
    hbar = _H_PLANCK / (2.0 * math.pi)
    return hbar * hbar / (_AMU * 1e-20) / _E_CHARGE


def lattice_block(n: int) -> np.ndarray:
    """n^3 integer vectors {-floor((n-1)/2) .. ceil((n-1)/2)}^3, first
    coordinate slowest."""
    lo = -((n - 1) // 2)
    r = np.arange(lo, lo + n)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.int32)


def lattice_box(n1: int, n2: int, n3: int) -> np.ndarray:
    """n1 x n2 x n3 integer vectors, each coordinate centred as in
    lattice_block, first coordinate slowest."""
    axes = [np.arange(-((n - 1) // 2), -((n - 1) // 2) + n) for n in (n1, n2, n3)]
    g = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, 3)
    return g.astype(np.int32)


def ws_block(n: int) -> Tuple[np.ndarray, np.ndarray]:
    """(n+1)^3 vectors {-n/2..n/2}^3 (n even) with weight 1/2 per boundary
    coordinate; closed under negation, weights sum to n^3."""
    assert n % 2 == 0
    h = n // 2
    r = np.arange(-h, h + 1)
    g = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    w = np.prod(np.where(np.abs(g) == h, 0.5, 1.0), axis=1)
    return g.astype(np.int32), w.astype(np.float64)


def _neg_index(vecs: np.ndarray) -> np.ndarray:
    lut = {tuple(v): i for i, v in enumerate(vecs.tolist())}
    return np.array([lut[tuple((-v).tolist())] for v in vecs], dtype=np.int64)


@dataclasses.dataclass
class System:
    name: str
    lattice: np.ndarray
    tau: np.ndarray
    mass: np.ndarray
    nw: int
    rh: np.ndarray
    rh_w: np.ndarray
    ham: np.ndarray
    rd: np.ndarray
    rd_w: np.ndarray
    ifc: np.ndarray
    re: np.ndarray
    rp: np.ndarray
    gw: np.ndarray
    mu_centroid: float

    @property
    def na(self) -> int:
        return int(self.mass.shape[0])

    @property
    def nmodes(self) -> int:
        return 3 * self.na

    @property
    def cell_volume(self) -> float:
        return float(abs(np.linalg.det(self.lattice)))


def _fcc(a: float) -> np.ndarray:
    h = 0.5 * a
    return np.array([[0.0, h, h], [h, 0.0, h], [h, h, 0.0]])


def _sc(a: float) -> np.ndarray:
    return np.diag([a, a, a]).astype(np.float64)


def _draw_ham(rng, lattice, rh, nw, onsite=None) -> np.ndarray:
    cart = rh @ lattice
    dist = np.linalg.norm(cart, axis=1)
    amp = rng.standard_normal((rh.shape[0], nw, nw)) * np.exp(-dist / 1.5)[:, None, None]
    neg = _neg_index(rh)
    ham = 0.5 * (amp + np.transpose(amp[neg], (0, 2, 1)))
    if onsite is not None:
        i0 = int(np.where((rh == 0).all(axis=1))[0][0])
        ham[i0] += np.diag(onsite)
    return ham.astype(np.complex128)


def _draw_ifc(rng, lattice, tau, mass, rd, rd_w, omega_scale_ev) -> np.ndarray:
    na = tau.shape[0]
    nd = rd.shape[0]
    ifc = np.zeros((nd, 3 * na, 3 * na))
    idx = {tuple(v): i for i, v in enumerate(rd.tolist())}
    i0 = idx[(0, 0, 0)]
    cart = rd @ lattice
    for ka in range(na):
        for kb in range(ka, na):
            for ir in range(nd):
                rv = tuple(rd[ir].tolist())
                if ka == kb and not (rv > (0, 0, 0)):
                    continue  # same-atom bonds: count R and -R once
                d = cart[ir] + tau[kb] - tau[ka]
                dn = float(np.linalg.norm(d))
                if dn == 0.0:
                    continue
                b = rng.standard_normal((3, 3))
                k = (b @ b.T) * math.exp(-dn / 1.5)
                w = rd_w[ir]
                jr = idx[tuple((-rd[ir]).tolist())]
                sa, sb = slice(3 * ka, 3 * ka + 3), slice(3 * kb, 3 * kb + 3)
                ifc[ir, sa, sb] -= k
                ifc[jr, sb, sa] -= k
                ifc[i0, sa, sa] += w * k
                ifc[i0, sb, sb] += w * k
    # q-independent Gershgorin bound on lambda_max of D(q)
    sq = np.sqrt(np.repeat(mass, 3))
    absd = np.abs(ifc) * rd_w[:, None, None] / (sq[:, None] * sq[None, :])
    bound = absd.sum(axis=(0, 2)).max()
    scale = omega_scale_ev ** 2 / (_c_phonon_ev() * bound)
    return ifc * scale


def _draw_g(rng, lattice, re, rp, nmodes, nw, real=False) -> np.ndarray:
    de = np.linalg.norm(re @ lattice, axis=1)
    dp = np.linalg.norm(rp @ lattice, axis=1)
    decay = np.exp(-(de[:, None] + dp[None, :]) / 1.5)
    shape = (re.shape[0], rp.shape[0], nmodes, nw, nw)
    sig = 0.1 / math.sqrt(2.0)
    gr = rng.standard_normal(shape) * sig
    gi = np.zeros(shape) if real else rng.standard_normal(shape) * sig
    g = (gr + 1j * gi) * decay[:, :, None, None, None]
    return g.astype(np.complex128)


def make_system(name: str, seed: Optional[int] = None, real_g: bool = False) -> System:
    """Build one of the named model systems.

    'toy_sc'  simple-cubic 1-atom toy, 4 orbitals, H/D on a 4^3 block,
              g on 4^3 x 4^3
    'al_fcc'  Al-like fcc metal, 4 orbitals, H/D on 6^3 blocks, g on
              6^3 x 6^3
    'si_fcc'  Si-like fcc 2-atom semiconductor, 8 orbitals (onsite -3 eV on
              1-4, +3 eV on 5-8), H on 8^3, D on 6^3, g on 8^3 x 6^3
    'mini_w1', 'mini_w8', 'mini_w2a2', 'mini_w4a2'
              small models covering the other (orbitals, modes) shapes:
              1 or 8 orbitals with 1 atom, 2 or 4 orbitals with 2 atoms;
              every block 4^3
    'box5_w4', 'box446_w2a2'
              small models whose Rp set is a 5^3 box (4 orbitals, 1 atom)
              or a 4 x 4 x 6 box (2 orbitals, 2 atoms)
    'chain_w2' 2 orbitals with hopping up to 7 cells along a1 (and nearest
              neighbours along a2, a3): an H(R) list whose bounding box is
              too long and too sparse for the separable Bloch sum
    'degen_w4', 'degen_w4_sym'
              exactly degenerate model: H(R) = h(R) (x) I_2 with a random
              2-orbital h (every band 2-fold), one atom with isotropic
              nearest-neighbour springs on a simple-cubic lattice (every
              phonon 3-fold); g random ('degen_w4') or g'(x) I_2
              ('degen_w4_sym', two identical decoupled copies)
    """
    defaults = {"toy_sc": 1649301, "al_fcc": 1649302, "si_fcc": 1649303,
                "mini_w1": 1649311, "mini_w2a2": 1649312, "mini_w8": 1649313, "mini_w4a2": 1649314,
                "box5_w4": 1649315, "box446_w2a2": 1649316, "degen_w4": 1649317, "degen_w4_sym": 1649317,
                "chain_w2": 1649318}
    if seed is None:
        seed = defaults[name]
    rng = np.random.default_rng(seed)
    if name == "toy_sc":
        lat, tau, mass, nw = _sc(3.0), np.zeros((1, 3)), np.array([26.98]), 4
        nh, nd, ne, npv, onsite = 4, 4, 4, 4, None
    elif name == "al_fcc":
        lat, tau, mass, nw = _fcc(4.05), np.zeros((1, 3)), np.array([26.98]), 4
        nh, nd, ne, npv, onsite = 6, 6, 6, 6, None
    elif name == "si_fcc":
        a = 5.43
        lat = _fcc(a)
        tau = np.array([[0.0, 0.0, 0.0], [0.25 * a, 0.25 * a, 0.25 * a]])
        mass, nw = np.array([28.0855, 28.0855]), 8
        nh, nd, ne, npv = 8, 6, 8, 6
        onsite = np.array([-3.0] * 4 + [3.0] * 4)
    elif name in ("mini_w1", "mini_w8"):
        # shape-coverage models: 1 atom with 1 or 8 orbitals, 4^3 blocks
        nw = 1 if name == "mini_w1" else 8
        lat = _sc(3.0) if nw == 1 else _fcc(4.0)
        tau, mass = np.zeros((1, 3)), np.array([26.98])
        nh, nd, ne, npv, onsite = 4, 4, 4, 4, None
    elif name in ("mini_w2a2", "mini_w4a2"):
        # shape-coverage models: 2 atoms (6 modes) with 2 or 4 orbitals
        a = 3.5
        lat = _sc(a)
        tau = np.array([[0.0, 0.0, 0.0], [0.5 * a, 0.5 * a, 0.5 * a]])
        mass = np.array([26.98, 40.0])
        nw = 2 if name == "mini_w2a2" else 4
        nh, nd, ne, npv, onsite = 4, 4, 4, 4, None
    elif name in ("box5_w4", "box446_w2a2"):
        if name == "box5_w4":
            lat, tau, mass, nw = _sc(3.0), np.zeros((1, 3)), np.array([26.98]), 4
        else:
            a = 3.5
            lat = _sc(a)
            tau = np.array([[0.0, 0.0, 0.0], [0.5 * a, 0.5 * a, 0.5 * a]])
            mass, nw = np.array([26.98, 40.0]), 2
        rh, rh_w = ws_block(4)
        rd, rd_w = ws_block(4)
        re = lattice_block(4)
        rp = lattice_block(5) if name == "box5_w4" else lattice_box(4, 4, 6)
        ham = _draw_ham(rng, lat, rh, nw)
        ifc = _draw_ifc(rng, lat, tau, mass, rd, rd_w, 0.040)
        gw = _draw_g(rng, lat, re, rp, 3 * mass.shape[0], nw)
        i0 = int(np.where((rh == 0).all(axis=1))[0][0])
        return System(name, lat, tau, mass, nw, rh, rh_w, ham, rd, rd_w, ifc, re, rp, gw,
                      float(np.real(np.trace(ham[i0]))) / nw)
    elif name == "chain_w2":
        lat, tau, mass, nw = _sc(3.0), np.zeros((1, 3)), np.array([26.98]), 2
        rh = np.array([[r, 0, 0] for r in range(-7, 8)] + [[0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                      dtype=np.int32)
        rh_w = np.ones(rh.shape[0])
        ham = _draw_ham(rng, _sc(1.0), rh, nw)  # decay over 1 A per cell: the long hops stay visible
        rd, rd_w = ws_block(4)
        ifc = _draw_ifc(rng, lat, tau, mass, rd, rd_w, 0.040)
        re, rp = lattice_block(4), lattice_block(4)
        gw = _draw_g(rng, lat, re, rp, 3, nw)
        i0 = int(np.where((rh == 0).all(axis=1))[0][0])
        return System(name, lat, tau, mass, nw, rh, rh_w, ham, rd, rd_w, ifc, re, rp, gw,
                      float(np.real(np.trace(ham[i0]))) / nw)
    elif name in ("degen_w4", "degen_w4_sym"):
        lat, tau, mass = _sc(3.0), np.zeros((1, 3)), np.array([26.98])
        rh, rh_w = ws_block(4)
        h = _draw_ham(rng, lat, rh, 2)
        ham = np.stack([np.kron(hr, np.eye(2)) for hr in h]).astype(np.complex128)
        # isotropic nearest-neighbour springs: Phi(+-a_i) = -K I, Phi(0) = 6K I
        rd = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], np.int32)
        rd_w = np.ones(rd.shape[0])
        K = 1.0
        ifc = np.stack([6 * K * np.eye(3)] + [-K * np.eye(3)] * 6)
        # scale so that the largest phonon energy (q = (1/2,1/2,1/2)) is 40 meV
        ifc = ifc * (0.040 ** 2 / (_c_phonon_ev() * 12 * K / mass[0]))
        re, rp = lattice_block(4), lattice_block(4)
        if name == "degen_w4":
            gw = _draw_g(rng, lat, re, rp, 3, 4)
        else:
            g2 = _draw_g(rng, lat, re, rp, 3, 2)
            gw = np.einsum("abmij,kl->abmikjl", g2, np.eye(2)).reshape(re.shape[0], rp.shape[0], 3, 4, 4)
        i0 = int(np.where((rh == 0).all(axis=1))[0][0])
        return System(name, lat, tau, mass, 4, rh, rh_w, ham, rd, rd_w, ifc.astype(np.float64), re, rp,
                      gw.astype(np.complex128), float(np.real(np.trace(ham[i0]))) / 4)
    else:
        raise KeyError(name)
    rh, rh_w = ws_block(nh)
    rd, rd_w = ws_block(nd)
    re, rp = lattice_block(ne), lattice_block(npv)
    ham = _draw_ham(rng, lat, rh, nw, onsite)
    ifc = _draw_ifc(rng, lat, tau, mass, rd, rd_w, 0.040)
    gw = _draw_g(rng, lat, re, rp, 3 * mass.shape[0], nw, real=real_g)
    i0 = int(np.where((rh == 0).all(axis=1))[0][0])
    mu = float(np.real(np.trace(ham[i0]))) / nw
    return System(name, lat, tau, mass, nw, rh, rh_w, ham, rd, rd_w, ifc,
                  re, rp, gw, mu)


@dataclasses.dataclass
class Workload:
    """A named transport run on one system: grid, smearing, temperatures,
    state window. Energies in eV, temperatures in K."""
    name: str
    system: str
    grid: int
    eta: float
    temps: Tuple[float, ...]
    window: Tuple[float, float]      # relative to mu unless absolute
    band_lo: int = 0
    band_hi: int = -1                # -1 = last band
    window_relative_to: str = "mu"   # 'mu' or 'cbm'
    mu_rule: str = "centroid"        # 'centroid' or 'cbm-0.25'
    note: str = ""


WORKLOADS = {
    "toy_sc_8": Workload("toy_sc_8", "toy_sc", 8, 0.050, (300.0,), (-1e3, 1e3),
                         note="all 2048 (n,k) states, 8^3 k x 8^3 q"),
    "al_fcc_100": Workload("al_fcc_100", "al_fcc", 100, 0.020,
                           (100.0, 300.0, 500.0), (-0.3, 0.3),
                           note="|e-mu| < 0.3 eV on 100^3 k, full 100^3 q"),
    "si_fcc_150": Workload("si_fcc_150", "si_fcc", 150, 0.010, (300.0,),
                           (0.0, 0.25), band_lo=4, band_hi=7,
                           window_relative_to="cbm", mu_rule="cbm-0.25",
                           note="conduction bands within 0.25 eV of the CBM"),
    "si_fcc_200": Workload("si_fcc_200", "si_fcc", 200, 0.010, (300.0,),
                           (0.0, 0.25), band_lo=4, band_hi=7,
                           window_relative_to="cbm", mu_rule="cbm-0.25"),
    "al_fcc_200": Workload("al_fcc_200", "al_fcc", 200, 0.020, (300.0,),
                           (-0.3, 0.3)),
}


def workload(name: str, grid: Optional[int] = None) -> Workload:
    w = dataclasses.replace(WORKLOADS[name])
    if grid is not None:
        w.grid = int(grid)
    return w
