// C ABI of the gfx950 EPWI transport library: model validation and upload,
// orchestration of the kernels of one scattering-rates call, conductivity.
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>

#include "internal.h"

namespace eph {

Units units() {
  Units u;
  const double hbar = kPlanck / (2.0 * kPi);
  u.hbar_evs = hbar / kCharge;
  u.kb_evk = kBoltz / kCharge;
  u.cph_ev = hbar * hbar / (kAmu * 1e-20) / kCharge;
  u.vel_unit = kCharge * 1e-10 / hbar;
  u.rate_pref = 2.0 * kPi / u.hbar_evs;
  return u;
}

// Electron tables (eps, V, v on the N^3 grid): the separable Bloch sum
// when the H(R) list has a dense box, else the direct sum over the list.
hipError_t electron_tables(eph_ctx *c, int N, const Units &U, hipStream_t st) {
  const int64_t NQ = (int64_t)N * N * N;
  if (c->hbox_n[0] > 0)
    return launch_bloch_lines(0, c->nw, N, c->hbox_lo, c->hbox_n, c->lattice, c->hbox.as<double2>(),
                              c->tab.as<double2>(), nullptr, U.cph_ev, 0.0, U.vel_unit, c->eps.as<double>(),
                              c->evec.as<double2>(), c->vel.as<double>(), nullptr, st);
  return launch_bloch_eig(0, c->nw, N, 0, NQ, c->nrh, c->rh.as<int>(), c->rh_w.as<double>(), c->rh_cart.as<double>(),
                          c->ham.as<double2>(), c->tab.as<double2>(), nullptr, U.cph_ev, 0.0, U.vel_unit,
                          c->eps.as<double>(), c->evec.as<double2>(), c->vel.as<double>(), nullptr, st);
}

// Phonon tables (hbar w, u on the N^3 grid), the same two forms.
hipError_t phonon_tables(eph_ctx *c, int N, const Units &U, double omega_cut, unsigned long long *n_excluded,
                         hipStream_t st) {
  const int64_t NQ = (int64_t)N * N * N;
  if (c->dbox_n[0] > 0)
    return launch_bloch_lines(1, c->nm, N, c->dbox_lo, c->dbox_n, c->lattice, c->dbox.as<double2>(),
                              c->tab.as<double2>(), c->mode_mass_d.as<double>(), U.cph_ev, omega_cut, U.vel_unit,
                              c->om.as<double>(), c->uu.as<double2>(), nullptr, n_excluded, st);
  return launch_bloch_eig(1, c->nm, N, 0, NQ, c->nrd, c->rd.as<int>(), c->rd_w.as<double>(), nullptr,
                          c->dyn.as<double2>(), c->tab.as<double2>(), c->mode_mass_d.as<double>(), U.cph_ev,
                          omega_cut, U.vel_unit, c->om.as<double>(), c->uu.as<double2>(), nullptr, n_excluded, st);
}

DevBuf::~DevBuf() {
  if (p) (void)hipFree(p);
}

hipError_t DevBuf::ensure(size_t n) {
  if (n <= bytes && p) return hipSuccess;
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
  if (n == 0) n = 8;
  hipError_t e = hipMalloc(&p, n);
  if (e == hipSuccess) bytes = n;
  else p = nullptr;
  return e;
}

}  // namespace eph

eph_gamma::~eph_gamma() {
  if (h_col) (void)hipHostFree(h_col);
  if (h_val) (void)hipHostFree(h_val);
}

using namespace eph;

static hipError_t scratch_address(int device, double **out);

namespace {

thread_local std::string g_load_error;

int fail(eph_ctx *c, int code, const std::string &msg) {
  c->err = msg;
  return code;
}

int hip_fail(eph_ctx *c, hipError_t e, const char *what) {
  (void)hipGetLastError();
  return fail(c, e == hipErrorOutOfMemory ? EPH_E_NOMEM : EPH_E_DEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define EPH_HIP(ctx, expr)                                 \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
  } while (0)

using Vec3 = std::tuple<int, int, int>;

// Event recorder for stage timing; a no-op unless profiling is on.
struct Timer {
  eph_ctx *c;
  hipStream_t st;
  int used = 0;
  hipError_t mark(int *slot) {
    *slot = -1;
    if (!c->profiling) return hipSuccess;
    if ((int)c->ev.size() <= used) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      c->ev.push_back(e);
    }
    *slot = used;
    return hipEventRecord(c->ev[used++], st);
  }
  float ms(int a, int b) const {
    float t = 0.f;
    if (a >= 0 && b >= 0) (void)hipEventElapsedTime(&t, c->ev[a], c->ev[b]);
    return t;
  }
};

template <class T>
hipError_t upload(DevBuf &b, const T *host, size_t n) {
  hipError_t e = b.ensure(sizeof(T) * n);
  if (e != hipSuccess) return e;
  return hipMemcpy(b.p, host, sizeof(T) * n, hipMemcpyHostToDevice);
}

// Device workspace of one rates call: grid tables and per-call lists
// (fixed), and the per-batch buffers per state of a batch.
struct Workspace {
  size_t fixed = 0;
  size_t per_state = 0;
};

Workspace plan_workspace(const eph_ctx *c, int N, int precision, int64_t nkl, int64_t ns, bool wave,
                         bool gamma = false) {
  const size_t NQ = (size_t)N * N * N, nw = c->nw, nm = c->nm;
  const bool red = precision != EPH_FP64;
  Workspace w;
  size_t t = 16 * (size_t)N + 64;                                   // phase table, counters
  t += NQ * nw * 8 + NQ * nw * nw * 16 + NQ * nw * 24;              // eps, eigenvectors, velocities
  t += NQ * nm * 8 + NQ * nm * nm * 16;                             // phonon energies, displacements
  if (red) t += NQ * nw * nw * 8 + NQ * nm * nm * 8;                // FP32 rotation tables
  if (red && wave) t += NQ * (nw + nm) * EPH_MAX_TEMPS * 4;         // FP32 occupation tables
  const size_t ncol = (size_t)c->box.count() * nm * nw, K = (size_t)c->nre * nw;
  if (precision == EPH_FP32) t += ncol * K * 8;                     // FP32 copy of g
  if (precision == EPH_BF16X3) t += 4 * bf16_w_elems(c->nre, c->nw, (int)ncol);  // bf16 hi/lo of g
  if (wave) {
    t += NQ * (nw + nm) * EPH_MAX_TEMPS * 8;                        // occupation tables
    t += NQ * nw * 4;                                               // float energies (prefilter)
  } else {
    t += NQ * nw * 10;                                              // energy-sorted lines
  }
  const size_t nl = (size_t)nkl + 1;
  t += 8 * (nl * 2 + scan_tmp_elems((int64_t)nl));                  // state counts and offsets
  t += 8 * (size_t)nkl;                                             // k subset
  const size_t nsl = (size_t)ns + 1;
  t += 8 * (3 * nsl + 2 * (size_t)ns + scan_tmp_elems((int64_t)nsl));  // groups, per-state counts
  if (gamma) t += NQ * nw * 4 + 16 * nsl;                           // state index table, counts, row starts
  w.fixed = t;
  w.per_state = (size_t)c->box.count() * nm * nw * (red ? 8 : 16);  // X row
  if (precision == EPH_BF16X3) w.per_state += 4 * bf16_a_elems(c->nre, c->nw);  // bf16 state operand
  return w;
}

// Checks that the R set is closed under negation with equal weights and
// that M(-R) = M(R)^dagger (herm=true, complex) or M(R)^T (real).
std::string check_pairs(int nr, const int32_t *R, const double *w, const double *M, int n, bool cplx) {
  std::map<Vec3, int> idx;
  for (int r = 0; r < nr; r++) {
    Vec3 v{R[3 * r], R[3 * r + 1], R[3 * r + 2]};
    if (idx.count(v)) return "duplicate lattice vector";
    idx[v] = r;
    if (!(w[r] > 0.0) || !std::isfinite(w[r])) return "weights must be positive";
  }
  const int es = cplx ? 2 : 1;
  double mx = 0.0;
  for (size_t e = 0; e < (size_t)nr * n * n * es; e++) {
    if (!std::isfinite(M[e])) return "non-finite matrix element";
    mx = std::max(mx, std::fabs(M[e]));
  }
  for (int r = 0; r < nr; r++) {
    Vec3 neg{-R[3 * r], -R[3 * r + 1], -R[3 * r + 2]};
    auto it = idx.find(neg);
    if (it == idx.end()) return "lattice-vector set not closed under R -> -R";
    int q = it->second;
    if (w[q] != w[r]) return "weights differ between R and -R";
    for (int i = 0; i < n; i++)
      for (int j = 0; j < n; j++) {
        // M(-R)_ij == conj(M(R)_ji)
        double ar = M[((size_t)q * n * n + i * n + j) * es];
        double br = M[((size_t)r * n * n + j * n + i) * es];
        double d = std::fabs(ar - br);
        if (cplx) {
          double ai = M[((size_t)q * n * n + i * n + j) * es + 1];
          double bi = M[((size_t)r * n * n + j * n + i) * es + 1];
          d = std::max(d, std::fabs(ai + bi));
        }
        if (d > 1e-12 * mx) return cplx ? "H(-R) != H(R)^dagger" : "Phi(-R) != Phi(R)^T";
      }
  }
  return "";
}

}  // namespace

extern "C" {

const char *eph_last_error(const eph_ctx *ctx) { return ctx ? ctx->err.c_str() : g_load_error.c_str(); }

void eph_free(eph_ctx *ctx) {
  if (!ctx) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(ctx->device);
  delete ctx;
  (void)hipSetDevice(cur);
}

int32_t eph_load_wannier(const eph_model *m, int32_t device, eph_ctx **out) {
  if (!out) {
    g_load_error = "out is NULL";
    return EPH_E_INVALID;
  }
  *out = nullptr;
  eph_ctx *c = new eph_ctx();
  auto bad = [&](int code, const std::string &msg) {
    g_load_error = msg;
    delete c;
    return code;
  };
  if (!m) return bad(EPH_E_INVALID, "model is NULL");
  if (m->n_wann < 1 || m->n_atoms < 1 || m->n_rh < 1 || m->n_rd < 1 || m->n_re < 1 || m->n_rp < 1)
    return bad(EPH_E_INVALID, "dimensions must be positive");
  if (!m->mass_amu || !m->rh || !m->rh_w || !m->ham || !m->rd || !m->rd_w || !m->ifc || !m->re || !m->rp || !m->gw)
    return bad(EPH_E_INVALID, "NULL model array");
  if (m->n_wann > EPH_MAX_WANN) return bad(EPH_E_UNSUPPORTED, "n_wann above EPH_MAX_WANN");
  if (3 * m->n_atoms > EPH_MAX_MODES) return bad(EPH_E_UNSUPPORTED, "3*n_atoms above EPH_MAX_MODES");
  const int nw = m->n_wann, na = m->n_atoms, nm = 3 * na;
  if (!(nw == 1 || nw == 2 || nw == 4 || nw == 8)) return bad(EPH_E_UNSUPPORTED, "n_wann must be 1, 2, 4 or 8");
  for (int a = 0; a < na; a++)
    if (!(m->mass_amu[a] > 0.0) || !std::isfinite(m->mass_amu[a])) return bad(EPH_E_INVALID, "masses must be positive");
  double vol = m->lattice[0] * (m->lattice[4] * m->lattice[8] - m->lattice[5] * m->lattice[7]) -
               m->lattice[1] * (m->lattice[3] * m->lattice[8] - m->lattice[5] * m->lattice[6]) +
               m->lattice[2] * (m->lattice[3] * m->lattice[7] - m->lattice[4] * m->lattice[6]);
  if (!(std::fabs(vol) > 0.0) || !std::isfinite(vol)) return bad(EPH_E_INVALID, "degenerate lattice");
  std::string why = check_pairs(m->n_rh, m->rh, m->rh_w, m->ham, nw, true);
  if (!why.empty()) return bad(EPH_E_INVALID, "H: " + why);
  why = check_pairs(m->n_rd, m->rd, m->rd_w, m->ifc, nm, false);
  if (!why.empty()) return bad(EPH_E_INVALID, "Phi: " + why);
  // Rp must be a full box
  int lo[3], hi[3];
  for (int a = 0; a < 3; a++) lo[a] = hi[a] = m->rp[a];
  for (int r = 0; r < m->n_rp; r++)
    for (int a = 0; a < 3; a++) {
      lo[a] = std::min(lo[a], m->rp[3 * r + a]);
      hi[a] = std::max(hi[a], m->rp[3 * r + a]);
    }
  RpBox box;
  for (int a = 0; a < 3; a++) {
    box.lo[a] = lo[a];
    box.n[a] = hi[a] - lo[a] + 1;
    if (box.n[a] > 16) return bad(EPH_E_UNSUPPORTED, "Rp box edge above 16");
  }
  if ((int64_t)box.count() != m->n_rp) return bad(EPH_E_UNSUPPORTED, "Rp vectors must form a full box");
  std::vector<int> rp_pos(m->n_rp);
  {
    std::vector<char> seen(box.count(), 0);
    for (int r = 0; r < m->n_rp; r++) {
      int p = ((m->rp[3 * r] - lo[0]) * box.n[1] + (m->rp[3 * r + 1] - lo[1])) * box.n[2] + (m->rp[3 * r + 2] - lo[2]);
      if (seen[p]) return bad(EPH_E_INVALID, "duplicate Rp vector");
      seen[p] = 1;
      rp_pos[r] = p;
    }
  }
  for (size_t e = 0; e < (size_t)m->n_re * m->n_rp * nm * nw * nw * 2; e++)
    if (!std::isfinite(m->gw[e])) return bad(EPH_E_INVALID, "non-finite g");

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return bad(EPH_E_DEVICE, "no HIP device");
  if (device < 0 || device >= ndev) return bad(EPH_E_INVALID, "device index out of range");
  DeviceGuard dg(device);
  if (!dg.ok) return bad(EPH_E_DEVICE, "hipSetDevice failed");
  {  // the static workspace of eph_conductivity_noalloc on this device
    hipError_t e = scratch_address(device, &c->scratch);
    if (e != hipSuccess) return bad(EPH_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }

  c->device = device;
  c->nw = nw;
  c->na = na;
  c->nm = nm;
  std::memcpy(c->lattice, m->lattice, sizeof(c->lattice));
  c->volume = std::fabs(vol);
  c->nrh = m->n_rh;
  c->nrd = m->n_rd;
  c->nre = m->n_re;
  c->nrp = m->n_rp;
  c->box = box;
  c->mode_mass.resize(nm);
  for (int mu = 0; mu < nm; mu++) c->mode_mass[mu] = m->mass_amu[mu / 3];

  // H: vectors, weights, Cartesian vectors, matrices
  std::vector<double> cart(3 * (size_t)m->n_rh);
  for (int r = 0; r < m->n_rh; r++)
    for (int a = 0; a < 3; a++)
      cart[3 * r + a] = m->rh[3 * r] * m->lattice[a] + m->rh[3 * r + 1] * m->lattice[3 + a] +
                        m->rh[3 * r + 2] * m->lattice[6 + a];
  // Phi / sqrt(M M') as complex
  std::vector<double> dyn(2 * (size_t)m->n_rd * nm * nm, 0.0);
  for (int r = 0; r < m->n_rd; r++)
    for (int a = 0; a < nm; a++)
      for (int b = 0; b < nm; b++)
        dyn[2 * (((size_t)r * nm + a) * nm + b)] =
            m->ifc[((size_t)r * nm + a) * nm + b] / std::sqrt(c->mode_mass[a] * c->mode_mass[b]);
  // g: Wt[(re, j)][(rp_box, mu, i)]
  const size_t ncol = (size_t)box.count() * nm * nw, K = (size_t)m->n_re * nw;
  std::vector<double> wt(2 * K * ncol);
  for (int r = 0; r < m->n_re; r++)
    for (int p = 0; p < m->n_rp; p++)
      for (int mu = 0; mu < nm; mu++)
        for (int i = 0; i < nw; i++)
          for (int j = 0; j < nw; j++) {
            size_t src = ((((size_t)r * m->n_rp + p) * nm + mu) * nw + i) * nw + j;
            size_t dst = ((size_t)r * nw + j) * ncol + ((size_t)rp_pos[p] * nm + mu) * nw + i;
            wt[2 * dst] = m->gw[2 * src];
            wt[2 * dst + 1] = m->gw[2 * src + 1];
          }
  // dense weighted boxes for the separable Bloch sum, when the R list fills
  // at least a quarter of its bounding box and the box is short along R1
  auto dense_box = [&](int nr, const int *R, const double *w, const double *M, int n, int *lo, int *nb,
                       std::vector<double> &box) {
    int hi[3];
    for (int a = 0; a < 3; a++) lo[a] = hi[a] = R[a];
    for (int r = 0; r < nr; r++)
      for (int a = 0; a < 3; a++) {
        lo[a] = std::min(lo[a], R[3 * r + a]);
        hi[a] = std::max(hi[a], R[3 * r + a]);
      }
    for (int a = 0; a < 3; a++) nb[a] = hi[a] - lo[a] + 1;
    const int64_t cells = (int64_t)nb[0] * nb[1] * nb[2];
    if (nb[0] > kBoxMaxR1 || cells > 4 * (int64_t)nr) {
      nb[0] = nb[1] = nb[2] = 0;
      return;
    }
    const size_t nn = (size_t)n * n;
    box.assign(2 * (size_t)cells * nn, 0.0);
    for (int r = 0; r < nr; r++) {
      const size_t cell = ((size_t)(R[3 * r] - lo[0]) * nb[1] + (R[3 * r + 1] - lo[1])) * nb[2] + (R[3 * r + 2] - lo[2]);
      for (size_t x = 0; x < 2 * nn; x++) box[2 * cell * nn + x] += w[r] * M[2 * (size_t)r * nn + x];
    }
  };
  std::vector<double> hb, db;
  dense_box(m->n_rh, m->rh, m->rh_w, m->ham, nw, c->hbox_lo, c->hbox_n, hb);
  dense_box(m->n_rd, m->rd, m->rd_w, dyn.data(), nm, c->dbox_lo, c->dbox_n, db);
  hipError_t e;
  if ((!hb.empty() && (e = upload(c->hbox, hb.data(), hb.size())) != hipSuccess) ||
      (!db.empty() && (e = upload(c->dbox, db.data(), db.size())) != hipSuccess)) {
    (void)hipGetLastError();
    return bad(e == hipErrorOutOfMemory ? EPH_E_NOMEM : EPH_E_DEVICE, std::string("upload: ") + hipGetErrorString(e));
  }
  if ((e = upload(c->rh, m->rh, 3 * (size_t)m->n_rh)) != hipSuccess ||
      (e = upload(c->rh_w, m->rh_w, (size_t)m->n_rh)) != hipSuccess ||
      (e = upload(c->rh_cart, cart.data(), cart.size())) != hipSuccess ||
      (e = upload(c->ham, m->ham, 2 * (size_t)m->n_rh * nw * nw)) != hipSuccess ||
      (e = upload(c->rd, m->rd, 3 * (size_t)m->n_rd)) != hipSuccess ||
      (e = upload(c->rd_w, m->rd_w, (size_t)m->n_rd)) != hipSuccess ||
      (e = upload(c->dyn, dyn.data(), dyn.size())) != hipSuccess ||
      (e = upload(c->re, m->re, 3 * (size_t)m->n_re)) != hipSuccess ||
      (e = upload(c->wt64, wt.data(), wt.size())) != hipSuccess ||
      (e = upload(c->mode_mass_d, c->mode_mass.data(), c->mode_mass.size())) != hipSuccess) {
    (void)hipGetLastError();
    return bad(e == hipErrorOutOfMemory ? EPH_E_NOMEM : EPH_E_DEVICE,
               std::string("upload: ") + hipGetErrorString(e));
  }
  *out = c;
  return EPH_OK;
}

// Transition rates requested from a rates call: count them only (memory
// estimate), or build them.
struct GammaReq {
  bool estimate_only = false;
  int64_t nnz = 0;
  int64_t bytes = 0;
  eph_gamma *out = nullptr;
};

static int32_t rates_impl(eph_ctx *c, const eph_rates_params *p, int64_t capacity, int32_t *state_k,
                          int32_t *state_n, double *energy_eV, double *vel_ms, double *inv_tau_s,
                          eph_counts *counts, bool states_only, GammaReq *gr = nullptr, int kbatch_q = 0) {
  if (!c) return EPH_E_INVALID;
  c->err.clear();
  if (!p) return fail(c, EPH_E_INVALID, "params is NULL");
  const int N = p->grid[0];
  if (N < 1 || p->grid[1] != N || p->grid[2] != N) return fail(c, EPH_E_INVALID, "grid must be N x N x N, N >= 1");
  if (N > EPH_MAX_GRID) return fail(c, EPH_E_UNSUPPORTED, "grid above EPH_MAX_GRID");
  if ((int64_t)N * c->nw > EPH_MAX_LINE) return fail(c, EPH_E_UNSUPPORTED, "N * n_wann above EPH_MAX_LINE");
  if (p->mem_budget_bytes < 0) return fail(c, EPH_E_INVALID, "mem_budget_bytes < 0");
  if (p->n_temps < 1 || p->n_temps > EPH_MAX_TEMPS || !p->temps_K)
    return fail(c, EPH_E_INVALID, "n_temps must be 1..EPH_MAX_TEMPS with temps_K given");
  for (int t = 0; t < p->n_temps; t++)
    if (!(p->temps_K[t] > 0.0) || !std::isfinite(p->temps_K[t])) return fail(c, EPH_E_INVALID, "temperatures must be > 0");
  if (!(p->eta_eV > 0.0) || !std::isfinite(p->eta_eV)) return fail(c, EPH_E_INVALID, "eta must be > 0");
  if (!(p->sieve_width > 0.0) || !std::isfinite(p->sieve_width)) return fail(c, EPH_E_INVALID, "sieve_width must be > 0");
  if (!(p->omega_cut_eV >= 0.0) || !std::isfinite(p->omega_cut_eV)) return fail(c, EPH_E_INVALID, "omega_cut must be >= 0");
  if (!std::isfinite(p->mu_eV) || std::isnan(p->win_lo_eV) || std::isnan(p->win_hi_eV))
    return fail(c, EPH_E_INVALID, "mu / window must be numbers");
  if (p->precision != EPH_FP64 && p->precision != EPH_FP32 && p->precision != EPH_BF16X3)
    return fail(c, EPH_E_INVALID, "unknown precision");
  const int blo = p->band_lo, bhi = p->band_hi < 0 ? c->nw - 1 : p->band_hi;
  if (blo < 0 || blo > bhi || bhi >= c->nw) return fail(c, EPH_E_INVALID, "band range outside 0..n_wann-1");
  if (capacity < 0) return fail(c, EPH_E_INVALID, "capacity < 0");
  if (capacity > 0 && (!state_k || !state_n || !energy_eV || !vel_ms || (!inv_tau_s && !states_only)))
    return fail(c, EPH_E_INVALID, "NULL output buffer");
  const int64_t NQ = (int64_t)N * N * N;
  std::vector<int64_t> klist;
  if (p->k_subset) {
    if (p->n_k_subset < 0) return fail(c, EPH_E_INVALID, "n_k_subset < 0");
    klist.assign(p->k_subset, p->k_subset + p->n_k_subset);
    for (int64_t k : klist)
      if (k < 0 || k >= NQ) return fail(c, EPH_E_INVALID, "k_subset index outside the grid");
    std::sort(klist.begin(), klist.end());
    klist.erase(std::unique(klist.begin(), klist.end()), klist.end());
  }
  const int nw = c->nw, nm = c->nm;
  const int gwave = rates_wave_group(nw, nm, c->box, N, p->precision);
  if (gwave == 0 && rates_smem_bytes(p->precision, N, nw, nm, c->box) > 160 * 1024)
    return fail(c, EPH_E_UNSUPPORTED, "Rp box too large for the workgroup rate kernel at this grid");
  if (kbatch_q > 0 && (gwave == 0 || p->precision != EPH_FP64))
    return fail(c, EPH_E_UNSUPPORTED, "the k-batch order needs FP64 and a cubic Rp box of edge 4 or 6");
  if (gr && (gwave == 0 || p->precision != EPH_FP64))
    return fail(c, EPH_E_UNSUPPORTED,
                "transition rates need FP64 and the wave rate kernel (cubic Rp box of edge 4 or 6)");
  const int64_t nkl = p->k_subset ? (int64_t)klist.size() : (int64_t)N * N * N;
  {  // the grid tables and lists alone must fit the budget (states not known yet)
    const Workspace w0 = plan_workspace(c, N, p->precision, nkl, 0, gwave > 0);
    if (p->mem_budget_bytes > 0 && w0.fixed > (size_t)p->mem_budget_bytes)
      return fail(c, EPH_E_NOMEM, "mem_budget_bytes below the grid tables and lists (" + std::to_string(w0.fixed) +
                                      " bytes)");
  }
  DeviceGuard dg(c->device);
  if (!dg.ok) return fail(c, EPH_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(p->stream);
  const Units U = units();
  Timer tm{c, st};
  int e_start, e_tables = -1, e_prep = -1, e_end;
  std::vector<int> e_batch;  // per batch: before transform, after transform, after rates
  for (auto &x : c->stage_ms) x = 0.0;
  c->launches[0] = c->launches[1] = 0;
  EPH_HIP(c, tm.mark(&e_start));

  // ---- grid tables: electrons and phonons on the full grid ----
  EPH_HIP(c, c->tab.ensure(sizeof(double2) * N));
  EPH_HIP(c, c->eps.ensure(sizeof(double) * NQ * nw));
  EPH_HIP(c, c->evec.ensure(sizeof(double2) * NQ * nw * nw));
  EPH_HIP(c, c->vel.ensure(sizeof(double) * NQ * nw * 3));
  EPH_HIP(c, c->om.ensure(sizeof(double) * NQ * nm));
  EPH_HIP(c, c->uu.ensure(sizeof(double2) * NQ * nm * nm));
  EPH_HIP(c, c->counters.ensure(sizeof(unsigned long long) * 8));
  unsigned long long *ctr = c->counters.as<unsigned long long>();
  // ctr: 0 n_excluded, 1 max omega bits, 2 n_kq, 3 sum n_q_valid, 4 sum n_terms, 5 n_zero,
  //      6 vertex contractions
  EPH_HIP(c, launch_zero(ctr, sizeof(unsigned long long) * 8, st));
  EPH_HIP(c, launch_phase_table(N, c->tab.as<double2>(), st));
  EPH_HIP(c, electron_tables(c, N, U, st));
  EPH_HIP(c, phonon_tables(c, N, U, p->omega_cut_eV, ctr + 0, st));
  const bool fp32 = p->precision != EPH_FP64;
  if (fp32) {  // FP32 copies of the rotation tables for the reduced-precision forms
    EPH_HIP(c, c->evec32.ensure(sizeof(float2) * NQ * nw * nw));
    EPH_HIP(c, c->uu32.ensure(sizeof(float2) * NQ * nm * nm));
    EPH_HIP(c, launch_to_f32(NQ * nw * nw, c->evec.as<double2>(), c->evec32.as<float2>(), st));
    EPH_HIP(c, launch_to_f32(NQ * nm * nm, c->uu.as<double2>(), c->uu32.as<float2>(), st));
    const size_t nwt = (size_t)c->nre * nw * c->box.count() * nm * nw;
    if (p->precision == EPH_FP32 && c->wt32.bytes < sizeof(float2) * nwt) {
      EPH_HIP(c, c->wt32.ensure(sizeof(float2) * nwt));
      EPH_HIP(c, launch_to_f32((int64_t)nwt, c->wt64.as<double2>(), c->wt32.as<float2>(), st));
    }
    const size_t nbf = 2 * bf16_w_elems(c->nre, nw, c->box.count() * nm * nw) * 2;  // hi + lo, 2 bytes each
    if (p->precision == EPH_BF16X3 && c->wtbf.bytes < nbf) {
      EPH_HIP(c, c->wtbf.ensure(nbf));
      EPH_HIP(c, launch_split_bf16(c->nre, nw, c->box.count() * nm * nw, c->wt64.as<double2>(), c->wtbf.p, st));
    }
  }
  EPH_HIP(c, tm.mark(&e_tables));

  // ---- states in the window ----
  const int64_t *d_klist = nullptr;
  if (p->k_subset) {
    EPH_HIP(c, c->subset.ensure(sizeof(int64_t) * std::max<int64_t>(1, nkl)));
    if (nkl > 0) EPH_HIP(c, hipMemcpyAsync(c->subset.p, klist.data(), sizeof(int64_t) * nkl, hipMemcpyHostToDevice, st));
    d_klist = c->subset.as<int64_t>();
  }
  EPH_HIP(c, c->cnt.ensure(sizeof(int64_t) * (nkl + 1)));
  EPH_HIP(c, c->offs.ensure(sizeof(int64_t) * (nkl + 1)));
  EPH_HIP(c, c->scan_tmp.ensure(sizeof(int64_t) * scan_tmp_elems(nkl + 1)));
  EPH_HIP(c, launch_zero(c->cnt.as<int64_t>() + nkl, sizeof(int64_t), st));
  EPH_HIP(c, launch_count_states(nkl, d_klist, nw, c->eps.as<double>(), blo, bhi, p->win_lo_eV, p->win_hi_eV,
                                 c->cnt.as<int64_t>(), st));
  EPH_HIP(c, launch_scan(nkl + 1, c->cnt.as<int64_t>(), c->offs.as<int64_t>(), c->scan_tmp.as<int64_t>(), st));
  int64_t ns = 0;
  EPH_HIP(c, hipMemcpyAsync(&ns, c->offs.as<int64_t>() + nkl, sizeof(int64_t), hipMemcpyDeviceToHost, st));
  EPH_HIP(c, hipStreamSynchronize(st));
  eph_counts cn;
  std::memset(&cn, 0, sizeof(cn));
  cn.n_states = ns;
  if (capacity < ns) {
    if (counts) *counts = cn;
    return fail(c, EPH_E_TRUNCATED, "capacity below the number of states");
  }
  EPH_HIP(c, launch_write_states(nkl, d_klist, nw, c->eps.as<double>(), c->vel.as<double>(), blo, bhi, p->win_lo_eV,
                                 p->win_hi_eV, c->offs.as<int64_t>(), state_k, state_n, energy_eV, vel_ms, st));
  if (states_only && !gr) {
    EPH_HIP(c, hipStreamSynchronize(st));
    if (counts) *counts = cn;
    return EPH_OK;
  }

  if (ns > 0) {
    // ---- groups of states sharing a k-line ----
    // the wave-autonomous kernel where it applies, else the workgroup form
    const int gmax = gwave > 0 ? gwave : rates_group_max(nw, nm);
    // state batches: the per-batch buffers (X) within the budget
    const Workspace ws = plan_workspace(c, N, p->precision, nkl, ns, gwave > 0, gr != nullptr);
    int64_t max_states;
    if (p->mem_budget_bytes > 0) {
      const size_t need = ws.fixed + ws.per_state * (size_t)gmax;
      if (need > (size_t)p->mem_budget_bytes)
        return fail(c, EPH_E_NOMEM, "mem_budget_bytes below the minimum of " + std::to_string(need) + " bytes (" +
                                        std::to_string(ws.fixed) + " bytes of tables and lists plus " +
                                        std::to_string(ws.per_state) + " bytes per state of a batch, " +
                                        std::to_string(gmax) + " states per group)");
      max_states = (int64_t)(((size_t)p->mem_budget_bytes - ws.fixed) / ws.per_state);
    } else {
      // automatic: the per-batch buffers take the free device memory less
      // 8 GiB, between 8 and 64 GiB (8 GiB when transition rates are built,
      // whose placement below assumes it), so that on a 288 GB part the
      // states of a large grid need few batches and few launch tails
      size_t xcap = (size_t)8 << 30;
      size_t freeb = 0, totalb = 0;
      if (!gr && hipMemGetInfo(&freeb, &totalb) == hipSuccess && freeb > ((size_t)16 << 30))
        xcap = std::min<size_t>(freeb - ((size_t)8 << 30), (size_t)64 << 30);
      (void)hipGetLastError();
      max_states = std::max<int64_t>(gmax, (int64_t)(xcap / ws.per_state));
    }
    EPH_HIP(c, c->grp_tmp.ensure(sizeof(int64_t) * 2 * (ns + 1)));
    int64_t *flag = c->grp_tmp.as<int64_t>(), *pos = flag + ns + 1;
    EPH_HIP(c, c->scan_tmp.ensure(sizeof(int64_t) * std::max(scan_tmp_elems(nkl + 1), scan_tmp_elems(ns))));
    EPH_HIP(c, launch_group_heads(ns, state_k, N, gmax, flag, st));
    EPH_HIP(c, launch_scan(ns, flag, pos, c->scan_tmp.as<int64_t>(), st));
    int64_t lastpf[2];
    EPH_HIP(c, hipMemcpyAsync(&lastpf[0], pos + ns - 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    EPH_HIP(c, hipMemcpyAsync(&lastpf[1], flag + ns - 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    EPH_HIP(c, hipStreamSynchronize(st));
    int64_t ng = lastpf[0] + lastpf[1];
    EPH_HIP(c, c->grp_start.ensure(sizeof(int64_t) * (ng + 1)));
    int64_t *gstart = c->grp_start.as<int64_t>();
    EPH_HIP(c, launch_group_starts(ns, flag, pos, gstart, st));
    std::vector<int64_t> hg(ng + 1);
    EPH_HIP(c, hipMemcpyAsync(hg.data(), gstart, sizeof(int64_t) * (ng + 1), hipMemcpyDeviceToHost, st));

    // ---- energy-sorted final-state lines (workgroup form) or occupation
    //      tables (wave form); largest phonon energy ----
    if (gwave == 0) {
      EPH_HIP(c, c->line_e.ensure(sizeof(double) * NQ * nw));
      EPH_HIP(c, c->line_key.ensure(sizeof(uint16_t) * NQ * nw));
      EPH_HIP(c, launch_line_sort(N, nw, c->eps.as<double>(), c->line_e.as<double>(), c->line_key.as<uint16_t>(),
                                  st));
    } else {
      double kts[EPH_MAX_TEMPS];
      for (int t = 0; t < p->n_temps; t++) kts[t] = U.kb_evk * p->temps_K[t];
      EPH_HIP(c, c->occ.ensure(sizeof(double) * NQ * (nw + nm) * EPH_MAX_TEMPS));
      EPH_HIP(c, launch_occupations(NQ, nw, nm, c->eps.as<double>(), c->om.as<double>(), p->mu_eV, p->n_temps, kts,
                                    p->omega_cut_eV, c->occ.as<double>(),
                                    c->occ.as<double>() + (size_t)NQ * nw * EPH_MAX_TEMPS, st));
    }
    EPH_HIP(c, launch_max_nonneg(NQ * nm, c->om.as<double>(), ctr + 1, st));
    EPH_HIP(c, tm.mark(&e_prep));
    unsigned long long wbits = 0;
    EPH_HIP(c, hipMemcpyAsync(&wbits, ctr + 1, sizeof(wbits), hipMemcpyDeviceToHost, st));
    EPH_HIP(c, hipStreamSynchronize(st));
    double wmax;
    std::memcpy(&wmax, &wbits, sizeof(wmax));

    // ---- per batch of groups: Re transform, then the fused rate kernel ----
    const size_t xrow = ws.per_state;
    EPH_HIP(c, c->state_cnt.ensure(sizeof(int64_t) * 2 * ns));
    RatesArgs a;
    std::memset(&a, 0, sizeof(a));
    a.N = N;
    a.nw = nw;
    a.nm = nm;
    a.nt = p->n_temps;
    a.box = c->box;
    a.mu = p->mu_eV;
    a.eta = p->eta_eV;
    a.sw = p->sieve_width;
    a.wcut = p->omega_cut_eV;
    a.wmax = wmax;
    for (int t = 0; t < p->n_temps; t++) a.temps_kt[t] = U.kb_evk * p->temps_K[t];
    a.pref = U.rate_pref / (double)NQ;
    a.sk = state_k;
    a.sn = state_n;
    a.eps = c->eps.as<double>();
    a.om = c->om.as<double>();
    a.evec = c->evec.as<double2>();
    a.uu = c->uu.as<double2>();
    a.line_e = c->line_e.as<double>();
    a.line_key = c->line_key.as<uint16_t>();
    a.tab = c->tab.as<double2>();
    a.inv_tau = inv_tau_s;
    a.ns_total = ns;
    a.st_counts = c->state_cnt.as<int64_t>();
    a.n_kq = ctr + 2;
    a.n_vertex = ctr + 6;
    a.evec32 = fp32 ? c->evec32.as<float2>() : nullptr;
    a.eps32 = nullptr;
    if (gwave > 0) {  // the wave kernel prefilters from a float copy of the energies
      EPH_HIP(c, c->eps32.ensure(sizeof(float) * NQ * nw));
      EPH_HIP(c, launch_real_to_f32(NQ * nw, c->eps.as<double>(), c->eps32.as<float>(), st));
      a.eps32 = c->eps32.as<float>();
    }
    a.uu32 = fp32 ? c->uu32.as<float2>() : nullptr;
    a.occ_f = c->occ.as<double>();
    a.occ_n = c->occ.as<double>() + (size_t)NQ * nw * EPH_MAX_TEMPS;
    a.occ32_f = a.occ32_n = nullptr;
    if (gwave > 0 && fp32) {  // FP32 copies of the occupation tables
      const size_t no = (size_t)NQ * (nw + nm) * EPH_MAX_TEMPS;
      EPH_HIP(c, c->occ32.ensure(sizeof(float) * no));
      EPH_HIP(c, launch_real_to_f32((int64_t)no, c->occ.as<double>(), c->occ32.as<float>(), st));
      a.occ32_f = c->occ32.as<float>();
      a.occ32_n = c->occ32.as<float>() + (size_t)NQ * nw * EPH_MAX_TEMPS;
    }
    const int ncol = c->box.count() * nm * nw;
    if (kbatch_q > 0) {  // ---- the k-batch order (ablation): q batches, all states each ----
      const int64_t per_q = (int64_t)c->nre * nm * nw * nw;
      EPH_HIP(c, c->kb_g.ensure(sizeof(double2) * per_q * kbatch_q));
      KBatchArgs kb;
      std::memset(&kb, 0, sizeof(kb));
      kb.N = N;
      kb.nw = nw;
      kb.nm = nm;
      kb.nt = p->n_temps;
      kb.nre = c->nre;
      kb.ns = ns;
      kb.eta = p->eta_eV;
      kb.sw = p->sieve_width;
      kb.wcut = p->omega_cut_eV;
      kb.pref = a.pref;
      kb.sk = state_k;
      kb.sn = state_n;
      kb.re = c->re.as<int>();
      kb.eps = c->eps.as<double>();
      kb.om = c->om.as<double>();
      kb.evec = c->evec.as<double2>();
      kb.tab = c->tab.as<double2>();
      kb.Gq = c->kb_g.as<double2>();
      kb.occ_f = a.occ_f;
      kb.occ_n = a.occ_n;
      kb.inv_tau = inv_tau_s;
      kb.st_counts = c->state_cnt.as<int64_t>();
      for (int64_t q0 = 0; q0 < NQ; q0 += kbatch_q) {
        const int nb = (int)std::min<int64_t>(kbatch_q, NQ - q0);
        int eb0, eb1, eb2;
        EPH_HIP(c, tm.mark(&eb0));
        EPH_HIP(c, launch_kbatch_step1(q0, nb, N, c->box, c->nre, nm, nw, ncol, c->wt64.as<double2>(),
                                       c->uu.as<double2>(), c->tab.as<double2>(), c->kb_g.as<double2>(), st));
        EPH_HIP(c, tm.mark(&eb1));
        kb.q0 = q0;
        kb.nb = nb;
        EPH_HIP(c, launch_kbatch_step2(kb, st));
        EPH_HIP(c, tm.mark(&eb2));
        e_batch.insert(e_batch.end(), {eb0, eb1, eb2});
        c->launches[0]++;
        c->launches[1]++;
      }
      ng = 0;  // the q-batch loop below has nothing left to do
    }
    // ---- transition rates: count pass, row starts, placement ----
    std::unique_ptr<eph_gamma> gam;
    std::vector<int64_t> hrow;
    bool spill = false;
    int64_t stage_cap = 0;
    const int nt = p->n_temps;
    if (gr) {
      EPH_HIP(c, c->stidx.ensure(sizeof(int32_t) * NQ * nw));
      EPH_HIP(c, launch_state_index(NQ, nw, ns, state_k, state_n, c->stidx.as<int32_t>(), st));
      EPH_HIP(c, c->gcur.ensure(sizeof(int64_t) * (ns + 1)));
      EPH_HIP(c, launch_zero(c->gcur.p, sizeof(int64_t) * (ns + 1), st));
      a.stidx = c->stidx.as<int32_t>();
      a.g_cursor = c->gcur.as<int64_t>();
      a.ng = ng;
      a.gstart = gstart;
      a.s_base = 0;
      a.X = nullptr;
      for (int q3 = 0; q3 < N; q3++) {
        a.q3_lo = q3;
        a.q3_hi = q3 + 1;
        a.q3_cur = q3;
        EPH_HIP(c, launch_rates_wave(EPH_FP64, a, st, kCount));
      }
      gam.reset(new eph_gamma());
      gam->ctx = c;
      EPH_HIP(c, gam->row.ensure(sizeof(int64_t) * (ns + 1)));
      EPH_HIP(c, c->scan_tmp.ensure(sizeof(int64_t) * scan_tmp_elems(ns + 1)));
      EPH_HIP(c, launch_scan(ns + 1, c->gcur.as<int64_t>(), gam->row.as<int64_t>(), c->scan_tmp.as<int64_t>(), st));
      hrow.resize(ns + 1);
      EPH_HIP(c, hipMemcpyAsync(hrow.data(), gam->row.p, sizeof(int64_t) * (ns + 1), hipMemcpyDeviceToHost, st));
      EPH_HIP(c, hipStreamSynchronize(st));
      const int64_t gnnz = hrow[ns];
      const size_t ebytes = 4 + 8 * (size_t)nt;  // one entry: column index and one value per temperature
      const size_t gbytes = (size_t)gnnz * ebytes + 8 * (size_t)(ns + 1);
      if (gr->estimate_only) {
        gr->nnz = gnnz;
        gr->bytes = (int64_t)gbytes;
        if (counts) *counts = cn;
        return EPH_OK;
      }
      // resident in device memory when it fits beside the other buffers,
      // else in pinned host memory, written through a staging buffer
      int64_t group_max = 0;  // most entries of one group
      for (int64_t g = 0; g < ng; g++) group_max = std::max(group_max, hrow[hg[g + 1]] - hrow[hg[g]]);
      if (p->mem_budget_bytes > 0) {
        const size_t rest = (size_t)p->mem_budget_bytes - ws.fixed;  // >= per_state * gmax (checked above)
        if (gbytes - 8 * (size_t)(ns + 1) + ws.per_state * (size_t)gmax <= rest) {
          max_states = (int64_t)((rest - (gbytes - 8 * (size_t)(ns + 1))) / ws.per_state);
        } else {
          spill = true;
          stage_cap = (int64_t)((rest - ws.per_state * (size_t)gmax) / 2 / ebytes);
          if (stage_cap < std::max<int64_t>(group_max, 1))
            return fail(c, EPH_E_NOMEM, "mem_budget_bytes leaves no room to stage the transition rates of one group (" +
                                            std::to_string(group_max * ebytes) + " bytes)");
          max_states = (int64_t)((rest - (size_t)stage_cap * ebytes) / ws.per_state);
        }
      } else {
        size_t freeb = 0, totalb = 0;
        EPH_HIP(c, hipMemGetInfo(&freeb, &totalb));
        const size_t xb = std::min<size_t>((size_t)8 << 30, ws.per_state * (size_t)ns);
        if (gbytes + xb + ((size_t)1 << 30) > freeb) {
          spill = true;
          stage_cap = std::max<int64_t>(group_max, std::min<int64_t>(gnnz, (int64_t)(((size_t)4 << 30) / ebytes)));
        }
      }
      gam->ns = ns;
      gam->nnz = gnnz;
      gam->nt = nt;
      for (int t = 0; t < nt; t++) gam->temps[t] = p->temps_K[t];
      gam->mu = p->mu_eV;
      gam->on_host = spill;
      gam->stage_nnz = stage_cap;
      if (spill) {
        hipError_t e1 = hipHostMalloc((void **)&gam->h_col, sizeof(int32_t) * std::max<int64_t>(gnnz, 1));
        hipError_t e2 = hipHostMalloc((void **)&gam->h_val, sizeof(double) * nt * std::max<int64_t>(gnnz, 1));
        if (e1 != hipSuccess || e2 != hipSuccess) {
          (void)hipGetLastError();
          return fail(c, EPH_E_NOMEM, "pinned host memory for the transition rates (" + std::to_string(gbytes) + " bytes)");
        }
        EPH_HIP(c, c->gstage_col.ensure(sizeof(int32_t) * stage_cap));
        EPH_HIP(c, c->gstage_val.ensure(sizeof(double) * nt * stage_cap));
      } else {
        EPH_HIP(c, gam->col.ensure(sizeof(int32_t) * std::max<int64_t>(gnnz, 1)));
        EPH_HIP(c, gam->val.ensure(sizeof(double) * nt * std::max<int64_t>(gnnz, 1)));
      }
      // every state's entries start at its row start
      EPH_HIP(c, hipMemcpyAsync(c->gcur.p, gam->row.p, sizeof(int64_t) * ns, hipMemcpyDeviceToDevice, st));
    }
    int64_t g0 = 0;
    while (g0 < ng) {
      int64_t g1 = g0 + 1;
      while (g1 < ng && hg[g1 + 1] - hg[g0] <= max_states &&
             (!spill || hrow[hg[g1 + 1]] - hrow[hg[g0]] <= stage_cap))
        g1++;
      const int64_t sa = hg[g0], sb = hg[g1];
      EPH_HIP(c, c->xbuf.ensure(xrow * (size_t)(sb - sa)));
      if (p->precision == EPH_BF16X3) EPH_HIP(c, c->abf.ensure(4 * bf16_a_elems(c->nre, nw) * (size_t)(sb - sa)));
      int eb0, eb1, eb2;
      EPH_HIP(c, tm.mark(&eb0));
      if (p->precision == EPH_BF16X3)
        EPH_HIP(c, launch_xform_bf16x3(sb - sa, state_k + sa, state_n + sa, N, nw, c->nre, c->re.as<int>(), ncol,
                                       c->wtbf.p, c->abf.p, c->evec.as<double2>(), c->tab.as<double2>(),
                                       c->xbuf.as<float2>(), st));
      else if (fp32)
        EPH_HIP(c, launch_xform32(sb - sa, state_k + sa, state_n + sa, N, nw, c->nre, c->re.as<int>(), ncol,
                                  c->wt32.as<float2>(), c->evec.as<double2>(), c->tab.as<double2>(),
                                  c->xbuf.as<float2>(), st));
      else
        EPH_HIP(c, launch_xform64(sb - sa, state_k + sa, state_n + sa, N, nw, c->nre, c->re.as<int>(), ncol,
                                  c->wt64.as<double2>(), c->evec.as<double2>(), c->tab.as<double2>(),
                                  c->xbuf.as<double2>(), st));
      a.ng = g1 - g0;
      a.gstart = gstart + g0;
      a.s_base = sa;
      a.X = c->xbuf.p;
      EPH_HIP(c, tm.mark(&eb1));
      if (gr) {
        a.g_base = spill ? hrow[sa] : 0;
        a.g_col = spill ? c->gstage_col.as<int32_t>() : gam->col.as<int32_t>();
        a.g_val = spill ? c->gstage_val.as<double>() : gam->val.as<double>();
        a.g_stride = spill ? stage_cap : gam->nnz;
      }
      if (gwave > 0) {
        // one launch per q3 plane: every resident wave then works on the same
        // plane, whose q-side tables stay in the XCD's L2
        for (int q3 = 0; q3 < N; q3++) {
          a.q3_lo = q3;
          a.q3_hi = q3 + 1;
          a.q3_cur = q3;
          EPH_HIP(c, launch_rates_wave(p->precision, a, st, gr ? kEmit : kRates));
        }
      } else
        EPH_HIP(c, launch_rates(p->precision, a, st));
      EPH_HIP(c, tm.mark(&eb2));
      if (gr && spill && hrow[sb] > hrow[sa]) {  // this batch's rows to pinned host memory
        const int64_t e0 = hrow[sa], ne = hrow[sb] - hrow[sa];
        EPH_HIP(c, hipMemcpyAsync(gam->h_col + e0, c->gstage_col.p, sizeof(int32_t) * ne, hipMemcpyDeviceToHost, st));
        for (int t = 0; t < nt; t++)
          EPH_HIP(c, hipMemcpyAsync(gam->h_val + (size_t)t * gam->nnz + e0, c->gstage_val.as<double>() + (size_t)t * stage_cap,
                                    sizeof(double) * ne, hipMemcpyDeviceToHost, st));
        EPH_HIP(c, hipStreamSynchronize(st));
      }
      e_batch.insert(e_batch.end(), {eb0, eb1, eb2});
      c->launches[0]++;
      c->launches[1] += gwave > 0 ? N : 1;
      g0 = g1;
    }
    EPH_HIP(c, launch_summarize(ns, c->state_cnt.as<int64_t>(), inv_tau_s, ctr + 3, st));
    if (gr) EPH_HIP(c, launch_check_rows(ns, c->gcur.as<int64_t>(), gam->row.as<int64_t>(), ctr + 7, st));
    if (gr) {
      gam->h_row = std::move(hrow);
      gr->out = gam.release();
    }
  } else if (gr) {  // no states: an empty set of rows
    std::unique_ptr<eph_gamma> gam(new eph_gamma());
    gam->ctx = c;
    gam->nt = p->n_temps;
    for (int t = 0; t < p->n_temps; t++) gam->temps[t] = p->temps_K[t];
    gam->mu = p->mu_eV;
    gam->h_row.assign(1, 0);
    EPH_HIP(c, gam->row.ensure(sizeof(int64_t)));
    EPH_HIP(c, launch_zero(gam->row.p, sizeof(int64_t), st));
    if (gr->estimate_only) {
      gr->nnz = 0;
      gr->bytes = 8;
    } else {
      gr->out = gam.release();
    }
  }
  unsigned long long hc[8];
  EPH_HIP(c, tm.mark(&e_end));
  EPH_HIP(c, hipMemcpyAsync(hc, ctr, sizeof(hc), hipMemcpyDeviceToHost, st));
  EPH_HIP(c, hipStreamSynchronize(st));
  if (c->profiling) {
    c->stage_ms[0] = tm.ms(e_start, e_tables);
    c->stage_ms[1] = tm.ms(e_tables, e_prep);
    for (size_t b = 0; b + 2 < e_batch.size(); b += 3) {
      c->stage_ms[2] += tm.ms(e_batch[b], e_batch[b + 1]);
      c->stage_ms[3] += tm.ms(e_batch[b + 1], e_batch[b + 2]);
    }
    c->stage_ms[4] = tm.ms(e_start, e_end);
  }
  cn.n_excluded_modes = (int64_t)hc[0];
  cn.n_kq = (int64_t)hc[2];
  cn.n_nkq = (int64_t)hc[3];
  cn.n_terms = (int64_t)hc[4];
  cn.n_zero_rate = (int64_t)hc[5];
  cn.n_vertex = (int64_t)hc[6];
  if (gr && gr->out && hc[7] != 0) {
    delete gr->out;
    gr->out = nullptr;
    return fail(c, EPH_E_DEVICE, "transition rates: " + std::to_string(hc[7]) + " rows not filled to their counted length");
  }
  if (counts) *counts = cn;
  return EPH_OK;
}

int32_t eph_scattering_rates(eph_ctx *c, const eph_rates_params *p, int64_t capacity, int32_t *state_k,
                             int32_t *state_n, double *energy_eV, double *vel_ms, double *inv_tau_s,
                             eph_counts *counts) {
  return rates_impl(c, p, capacity, state_k, state_n, energy_eV, vel_ms, inv_tau_s, counts, false);
}

int32_t eph_select_states(eph_ctx *c, const eph_rates_params *p, int64_t capacity, int32_t *state_k,
                          int32_t *state_n, double *energy_eV, double *vel_ms, eph_counts *counts) {
  return rates_impl(c, p, capacity, state_k, state_n, energy_eV, vel_ms, nullptr, counts, true);
}

int32_t eph_rates_kbatch(eph_ctx *c, const eph_rates_params *p, int64_t capacity, int32_t *state_k, int32_t *state_n,
                         double *energy_eV, double *vel_ms, double *inv_tau_s, eph_counts *counts, int32_t q_batch) {
  if (!c) return EPH_E_INVALID;
  if (q_batch < 1 || q_batch > (1 << 20)) return fail(c, EPH_E_INVALID, "q_batch must be 1 .. 2^20");
  return rates_impl(c, p, capacity, state_k, state_n, energy_eV, vel_ms, inv_tau_s, counts, false, nullptr, q_batch);
}

int32_t eph_gamma_estimate(eph_ctx *c, const eph_rates_params *p, int64_t capacity, int32_t *state_k,
                           int32_t *state_n, double *energy_eV, double *vel_ms, int64_t *nnz, int64_t *bytes) {
  if (!c) return EPH_E_INVALID;
  if (!nnz || !bytes) return fail(c, EPH_E_INVALID, "nnz / bytes output is NULL");
  GammaReq gr;
  gr.estimate_only = true;
  eph_counts cn;
  const int32_t r = rates_impl(c, p, capacity, state_k, state_n, energy_eV, vel_ms, nullptr, &cn, true, &gr);
  if (r != EPH_OK) return r;
  *nnz = gr.nnz;
  *bytes = gr.bytes;
  return EPH_OK;
}

int32_t eph_rates_gamma(eph_ctx *c, const eph_rates_params *p, int64_t capacity, int32_t *state_k, int32_t *state_n,
                        double *energy_eV, double *vel_ms, double *inv_tau_s, eph_counts *counts, eph_gamma **out) {
  if (!c) return EPH_E_INVALID;
  if (!out) return fail(c, EPH_E_INVALID, "gamma output is NULL");
  *out = nullptr;
  GammaReq gr;
  const int32_t r = rates_impl(c, p, capacity, state_k, state_n, energy_eV, vel_ms, inv_tau_s, counts, false, &gr);
  if (r != EPH_OK) {
    delete gr.out;
    return r;
  }
  *out = gr.out;
  return EPH_OK;
}

int32_t eph_gamma_info(const eph_gamma *g, int64_t *n_states, int64_t *nnz, int32_t *n_temps, int32_t *on_host,
                       int64_t *bytes) {
  if (!g) return EPH_E_INVALID;
  if (n_states) *n_states = g->ns;
  if (nnz) *nnz = g->nnz;
  if (n_temps) *n_temps = g->nt;
  if (on_host) *on_host = g->on_host ? 1 : 0;
  if (bytes) *bytes = g->nnz * (4 + 8 * (int64_t)g->nt) + 8 * (g->ns + 1);
  return EPH_OK;
}

int32_t eph_gamma_copy(const eph_gamma *g, int64_t *row_start, int32_t *col, double *val) {
  if (!g) return EPH_E_INVALID;
  eph_ctx *c = g->ctx;
  DeviceGuard dg(c->device);
  if (!dg.ok) return fail(c, EPH_E_DEVICE, "hipSetDevice failed");
  if (row_start) std::memcpy(row_start, g->h_row.data(), sizeof(int64_t) * (g->ns + 1));
  if (g->nnz == 0) return EPH_OK;
  if (g->on_host) {
    if (col) std::memcpy(col, g->h_col, sizeof(int32_t) * g->nnz);
    if (val) std::memcpy(val, g->h_val, sizeof(double) * g->nt * g->nnz);
    return EPH_OK;
  }
  if (col) EPH_HIP(c, hipMemcpy(col, g->col.p, sizeof(int32_t) * g->nnz, hipMemcpyDeviceToHost));
  if (val) EPH_HIP(c, hipMemcpy(val, g->val.p, sizeof(double) * g->nt * g->nnz, hipMemcpyDeviceToHost));
  return EPH_OK;
}

void eph_gamma_free(eph_gamma *g) {
  if (!g) return;
  DeviceGuard dg(g->ctx->device);
  delete g;
}

int32_t eph_set_profiling(eph_ctx *c, int32_t on) {
  if (!c) return EPH_E_INVALID;
  c->profiling = on != 0;
  return EPH_OK;
}

int32_t eph_stage_times(const eph_ctx *c, double *ms, int64_t *launches) {
  if (!c || !ms || !launches) return EPH_E_INVALID;
  for (int i = 0; i < 5; i++) ms[i] = c->stage_ms[i];
  launches[0] = c->launches[0];
  launches[1] = c->launches[1];
  return EPH_OK;
}

}  // extern "C"

namespace {
// Workspace of the conductivity reduction, in doubles: per-block partials
// [kSigBlocks][EPH_MAX_TEMPS * 9], the reduced moments [3][EPH_MAX_TEMPS * 9]
// and k_B T [EPH_MAX_TEMPS].
constexpr int kSigBlocks = 256;
constexpr size_t kSigWorkDoubles = (size_t)kSigBlocks * EPH_MAX_TEMPS * 9 + 3 * EPH_MAX_TEMPS * 9 + EPH_MAX_TEMPS;

// Static device workspace of eph_conductivity_noalloc: one copy per GPU,
// held until the process ends.  In host code `scratch` only names the
// symbol; its device address comes from hipGetSymbolAddress (per device).
static __device__ __align__(256) double scratch[kSigWorkDoubles];

std::mutex g_scratch_mu;
double *g_scratch_ptr[64] = {nullptr};

}  // namespace

// Device address of `scratch` on the current device, looked up once per
// device (the caller has made `device` current).
static hipError_t scratch_address(int device, double **out) {
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double *>(ptr);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

namespace {

// Moments 0..n_orders-1 of the SERTA sum on the device inputs, into host
// out[order][EPH_MAX_TEMPS * 9] (S/m times eV^order).  work is a device
// buffer of kSigWorkDoubles; every part of it is written before it is read.
int32_t moments(eph_ctx *c, int64_t n_states, const double *energy_eV, const double *vel_ms,
                const double *inv_tau_s, double mu_eV, int32_t n_temps, const double *temps_K, int64_t n_kpoints,
                void *stream, int n_orders, double (*out)[EPH_MAX_TEMPS * 9], double *work,
                const double *F = nullptr) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Units U = units();
  double *part = work;
  double *outd = part + (size_t)kSigBlocks * EPH_MAX_TEMPS * 9;
  double *kts = outd + 3 * EPH_MAX_TEMPS * 9;
  double hk[EPH_MAX_TEMPS] = {1.0, 1.0, 1.0, 1.0};
  for (int t = 0; t < n_temps; t++) hk[t] = U.kb_evk * temps_K[t];
  EPH_HIP(c, hipMemcpyAsync(kts, hk, sizeof(hk), hipMemcpyHostToDevice, st));
  const double pref = 2.0 * kCharge / ((double)n_kpoints * c->volume * 1e-30);
  for (int o = 0; o < n_orders; o++)
    EPH_HIP(c, launch_sigma(n_states, energy_eV, vel_ms, inv_tau_s, mu_eV, n_temps, kts, pref, part, kSigBlocks,
                            outd + o * EPH_MAX_TEMPS * 9, st, o, F));
  EPH_HIP(c, hipMemcpyAsync(out, outd, sizeof(double) * n_orders * EPH_MAX_TEMPS * 9, hipMemcpyDeviceToHost, st));
  EPH_HIP(c, hipStreamSynchronize(st));
  return EPH_OK;
}

// Argument checks shared by the conductivity and transport entry points.
int32_t check_moment_args(eph_ctx *c, int64_t n_states, const double *energy_eV, const double *vel_ms,
                          const double *inv_tau_s, double mu_eV, int32_t n_temps, const double *temps_K,
                          int64_t n_kpoints) {
  if (!c) return EPH_E_INVALID;
  c->err.clear();
  if (n_states < 0) return fail(c, EPH_E_INVALID, "n_states < 0");
  if (n_temps < 1 || n_temps > EPH_MAX_TEMPS || !temps_K) return fail(c, EPH_E_INVALID, "bad temperatures");
  for (int t = 0; t < n_temps; t++)
    if (!(temps_K[t] > 0.0) || !std::isfinite(temps_K[t])) return fail(c, EPH_E_INVALID, "temperatures must be > 0");
  if (n_kpoints < 1) return fail(c, EPH_E_INVALID, "n_kpoints must be >= 1");
  if (n_states > 0 && (!energy_eV || !vel_ms || !inv_tau_s)) return fail(c, EPH_E_INVALID, "NULL input buffer");
  if (!std::isfinite(mu_eV)) return fail(c, EPH_E_INVALID, "mu must be finite");
  return EPH_OK;
}

// moments() on the context's grow-only workspace (allocated on first use).
int32_t moments_ctx(eph_ctx *c, int64_t n_states, const double *energy_eV, const double *vel_ms,
                    const double *inv_tau_s, double mu_eV, int32_t n_temps, const double *temps_K, int64_t n_kpoints,
                    void *stream, int n_orders, double (*out)[EPH_MAX_TEMPS * 9]) {
  int32_t r = check_moment_args(c, n_states, energy_eV, vel_ms, inv_tau_s, mu_eV, n_temps, temps_K, n_kpoints);
  if (r != EPH_OK) return r;
  DeviceGuard dg(c->device);
  if (!dg.ok) return fail(c, EPH_E_DEVICE, "hipSetDevice failed");
  EPH_HIP(c, c->sig_part.ensure(sizeof(double) * kSigWorkDoubles));
  return moments(c, n_states, energy_eV, vel_ms, inv_tau_s, mu_eV, n_temps, temps_K, n_kpoints, stream, n_orders,
                 out, c->sig_part.as<double>());
}

void inv3(const double *a, double *r) {
  const double c00 = a[4] * a[8] - a[5] * a[7], c01 = a[5] * a[6] - a[3] * a[8], c02 = a[3] * a[7] - a[4] * a[6];
  const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  r[0] = c00 / det;
  r[3] = c01 / det;
  r[6] = c02 / det;
  r[1] = (a[2] * a[7] - a[1] * a[8]) / det;
  r[4] = (a[0] * a[8] - a[2] * a[6]) / det;
  r[7] = (a[1] * a[6] - a[0] * a[7]) / det;
  r[2] = (a[1] * a[5] - a[2] * a[4]) / det;
  r[5] = (a[2] * a[3] - a[0] * a[5]) / det;
  r[8] = (a[0] * a[4] - a[1] * a[3]) / det;
}
void mul3(const double *a, const double *b, double *r) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) r[i * 3 + j] = a[i * 3] * b[j] + a[i * 3 + 1] * b[3 + j] + a[i * 3 + 2] * b[6 + j];
}
}  // namespace

extern "C" {

int32_t eph_conductivity(eph_ctx *c, int64_t n_states, const double *energy_eV, const double *vel_ms,
                         const double *inv_tau_s, double mu_eV, int32_t n_temps, const double *temps_K,
                         int64_t n_kpoints, void *stream, double *sigma_S_per_m) {
  if (c && !sigma_S_per_m) return fail(c, EPH_E_INVALID, "sigma output is NULL");
  double m[1][EPH_MAX_TEMPS * 9];
  const int32_t r = moments_ctx(c, n_states, energy_eV, vel_ms, inv_tau_s, mu_eV, n_temps, temps_K, n_kpoints, stream, 1, m);
  if (r != EPH_OK) return r;
  for (int t = 0; t < n_temps; t++)
    for (int q = 0; q < 9; q++) sigma_S_per_m[t * 9 + q] = m[0][t * 9 + q];
  return EPH_OK;
}

int32_t eph_conductivity_noalloc(eph_ctx *c, int64_t n_states, const double *energy_eV, const double *vel_ms,
                                 const double *inv_tau_s, double mu_eV, int32_t n_temps, const double *temps_K,
                                 int64_t n_kpoints, void *stream, double *sigma_S_per_m) {
  int32_t r = check_moment_args(c, n_states, energy_eV, vel_ms, inv_tau_s, mu_eV, n_temps, temps_K, n_kpoints);
  if (r != EPH_OK) return r;
  if (!sigma_S_per_m) return fail(c, EPH_E_INVALID, "sigma output is NULL");
  if (!c->scratch) return fail(c, EPH_E_STATE, "no static workspace on this context's device");
  DeviceGuard dg(c->device);
  if (!dg.ok) return fail(c, EPH_E_DEVICE, "hipSetDevice failed");
  double m[1][EPH_MAX_TEMPS * 9];
  r = moments(c, n_states, energy_eV, vel_ms, inv_tau_s, mu_eV, n_temps, temps_K, n_kpoints, stream, 1, m, c->scratch);
  if (r != EPH_OK) return r;
  for (int t = 0; t < n_temps; t++)
    for (int q = 0; q < 9; q++) sigma_S_per_m[t * 9 + q] = m[0][t * 9 + q];
  return EPH_OK;
}

int32_t eph_transport(eph_ctx *c, int64_t n_states, const double *energy_eV, const double *vel_ms,
                      const double *inv_tau_s, double mu_eV, int32_t n_temps, const double *temps_K,
                      int64_t n_kpoints, void *stream, double *sigma_S_per_m, double *seebeck_V_per_K,
                      double *kappa_W_per_mK) {
  if (c && (!sigma_S_per_m || !seebeck_V_per_K || !kappa_W_per_mK))
    return fail(c, EPH_E_INVALID, "NULL output");
  double m[3][EPH_MAX_TEMPS * 9];
  const int32_t r = moments_ctx(c, n_states, energy_eV, vel_ms, inv_tau_s, mu_eV, n_temps, temps_K, n_kpoints, stream, 3, m);
  if (r != EPH_OK) return r;
  for (int t = 0; t < n_temps; t++) {
    const double *m0 = m[0] + t * 9, *m1 = m[1] + t * 9, *m2 = m[2] + t * 9;
    double i0[9], s1[9], k1[9];
    inv3(m0, i0);
    mul3(i0, m1, s1);
    mul3(m1, s1, k1);
    for (int q = 0; q < 9; q++) {
      sigma_S_per_m[t * 9 + q] = m0[q];
      seebeck_V_per_K[t * 9 + q] = -s1[q] / temps_K[t];
      kappa_W_per_mK[t * 9 + q] = (m2[q] - k1[q]) / temps_K[t];
    }
  }
  return EPH_OK;
}

int32_t eph_bte_iterate(eph_ctx *c, const eph_gamma *g, const double *energy_eV, const double *vel_ms,
                        const double *inv_tau_s, int64_t n_kpoints, int32_t max_iter, double tol, void *stream,
                        double *sigma_iter, int32_t *n_iter, double *F_out) {
  if (!c) return EPH_E_INVALID;
  c->err.clear();
  if (!g || g->ctx != c) return fail(c, EPH_E_INVALID, "transition rates of another context (or NULL)");
  if (max_iter < 0 || !(tol >= 0.0) || !sigma_iter) return fail(c, EPH_E_INVALID, "max_iter >= 0, tol >= 0, sigma_iter");
  const int64_t ns = g->ns;
  const int nt = g->nt;
  int32_t r = check_moment_args(c, ns, energy_eV, vel_ms, inv_tau_s, g->mu, nt, g->temps, n_kpoints);
  if (r != EPH_OK) return r;
  DeviceGuard dg(c->device);
  if (!dg.ok) return fail(c, EPH_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(stream);
  EPH_HIP(c, c->sig_part.ensure(sizeof(double) * kSigWorkDoubles));
  const size_t fsz = (size_t)nt * ns * 3;
  EPH_HIP(c, c->bte_f.ensure(sizeof(double) * 3 * std::max<size_t>(fsz, 1)));
  double *F0 = c->bte_f.as<double>(), *Fa = F0 + fsz, *Fb = Fa + fsz;
  EPH_HIP(c, launch_f0(ns, nt, vel_ms, inv_tau_s, F0, st));
  if (g->on_host && g->nnz > 0) {
    EPH_HIP(c, c->gstage_col.ensure(sizeof(int32_t) * g->stage_nnz));
    EPH_HIP(c, c->gstage_val.ensure(sizeof(double) * g->stage_nnz));
  }
  double m[1][EPH_MAX_TEMPS * 9];
  r = moments(c, ns, energy_eV, vel_ms, inv_tau_s, g->mu, nt, g->temps, n_kpoints, stream, 1, m, c->sig_part.as<double>(), F0);
  if (r != EPH_OK) return r;
  for (int q = 0; q < nt * 9; q++) sigma_iter[q] = m[0][q];
  const double *Fin = F0;
  double *Fout = Fa;
  int32_t done = 0;
  for (int32_t it = 1; it <= max_iter; it++) {
    for (int t = 0; t < nt; t++) {
      const double *itau = inv_tau_s + (size_t)t * ns;
      const size_t fo = (size_t)t * ns * 3;
      if (!g->on_host) {
        EPH_HIP(c, launch_bte_step(0, ns, g->row.as<int64_t>(), 0, g->col.as<int32_t>(),
                                   g->val.as<double>() + (size_t)t * g->nnz, itau, F0 + fo, Fin + fo, Fout + fo, st));
        continue;
      }
      // rows in batches whose entries fit the staging buffer
      int64_t r0 = 0;
      while (r0 < ns) {
        int64_t r1 = r0 + 1;
        while (r1 < ns && g->h_row[r1 + 1] - g->h_row[r0] <= g->stage_nnz) r1++;
        const int64_t e0 = g->h_row[r0], ne = g->h_row[r1] - e0;
        if (ne > 0) {
          EPH_HIP(c, hipMemcpyAsync(c->gstage_col.p, g->h_col + e0, sizeof(int32_t) * ne, hipMemcpyHostToDevice, st));
          EPH_HIP(c, hipMemcpyAsync(c->gstage_val.p, g->h_val + (size_t)t * g->nnz + e0, sizeof(double) * ne,
                                    hipMemcpyHostToDevice, st));
        }
        EPH_HIP(c, launch_bte_step(r0, r1, g->row.as<int64_t>(), e0, c->gstage_col.as<int32_t>(),
                                   c->gstage_val.as<double>(), itau, F0 + fo, Fin + fo, Fout + fo, st));
        r0 = r1;
      }
    }
    r = moments(c, ns, energy_eV, vel_ms, inv_tau_s, g->mu, nt, g->temps, n_kpoints, stream, 1, m,
                c->sig_part.as<double>(), Fout);
    if (r != EPH_OK) return r;
    double dmax = 0.0, smax = 0.0;
    for (int q = 0; q < nt * 9; q++) {
      sigma_iter[(size_t)it * nt * 9 + q] = m[0][q];
      dmax = std::max(dmax, std::fabs(m[0][q] - sigma_iter[(size_t)(it - 1) * nt * 9 + q]));
      smax = std::max(smax, std::fabs(m[0][q]));
    }
    done = it;
    Fin = Fout;
    Fout = (Fout == Fa) ? Fb : Fa;
    if (dmax <= tol * smax) break;
  }
  if (F_out && fsz > 0) EPH_HIP(c, hipMemcpyAsync(F_out, Fin, sizeof(double) * fsz, hipMemcpyDeviceToDevice, st));
  EPH_HIP(c, hipStreamSynchronize(st));
  if (n_iter) *n_iter = done;
  return EPH_OK;
}

int32_t eph_carrier_density(eph_ctx *c, int32_t grid, int32_t band_lo, int32_t band_hi, double mu_eV,
                            int32_t n_temps, const double *temps_K, void *stream, double *n_per_m3) {
  if (!c) return EPH_E_INVALID;
  c->err.clear();
  if (grid < 1 || grid > EPH_MAX_GRID) return fail(c, EPH_E_INVALID, "grid must be 1..EPH_MAX_GRID");
  if (band_lo < 0 || band_hi >= c->nw || band_lo > band_hi) return fail(c, EPH_E_INVALID, "bad band range");
  if (n_temps < 1 || n_temps > EPH_MAX_TEMPS || !temps_K) return fail(c, EPH_E_INVALID, "bad temperatures");
  for (int t = 0; t < n_temps; t++)
    if (!(temps_K[t] > 0.0) || !std::isfinite(temps_K[t])) return fail(c, EPH_E_INVALID, "temperatures must be > 0");
  if (!std::isfinite(mu_eV)) return fail(c, EPH_E_INVALID, "mu must be finite");
  if (!n_per_m3) return fail(c, EPH_E_INVALID, "output is NULL");
  DeviceGuard dg(c->device);
  if (!dg.ok) return fail(c, EPH_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Units U = units();
  const int N = grid, nw = c->nw;
  const int64_t NQ = (int64_t)N * N * N;
  // band energies on the full grid (the electron half of the grid tables)
  EPH_HIP(c, c->tab.ensure(sizeof(double2) * N));
  EPH_HIP(c, c->eps.ensure(sizeof(double) * NQ * nw));
  EPH_HIP(c, c->evec.ensure(sizeof(double2) * NQ * nw * nw));
  EPH_HIP(c, c->vel.ensure(sizeof(double) * NQ * nw * 3));
  EPH_HIP(c, launch_phase_table(N, c->tab.as<double2>(), st));
  EPH_HIP(c, electron_tables(c, N, U, st));
  const int nblk = 256;
  EPH_HIP(c, c->sig_part.ensure(sizeof(double) * ((size_t)nblk * EPH_MAX_TEMPS + 2 * EPH_MAX_TEMPS)));
  double *part = c->sig_part.as<double>();
  double *outd = part + (size_t)nblk * EPH_MAX_TEMPS;
  double *kts = outd + EPH_MAX_TEMPS;
  double hk[EPH_MAX_TEMPS] = {1.0, 1.0, 1.0, 1.0};
  for (int t = 0; t < n_temps; t++) hk[t] = U.kb_evk * temps_K[t];
  EPH_HIP(c, hipMemcpyAsync(kts, hk, sizeof(hk), hipMemcpyHostToDevice, st));
  const double pref = 2.0 / ((double)NQ * c->volume * 1e-30);
  EPH_HIP(c, launch_density(NQ, nw, c->eps.as<double>(), band_lo, band_hi, mu_eV, n_temps, kts, pref, part, nblk,
                            outd, st));
  double ho[EPH_MAX_TEMPS];
  EPH_HIP(c, hipMemcpyAsync(ho, outd, sizeof(ho), hipMemcpyDeviceToHost, st));
  EPH_HIP(c, hipStreamSynchronize(st));
  for (int t = 0; t < n_temps; t++) n_per_m3[t] = ho[t];
  return EPH_OK;
}

int32_t eph_mobility(int32_t n_temps, const double *sigma_S_per_m, const double *n_per_m3, double *mobility_cm2) {
  if (n_temps < 1 || n_temps > EPH_MAX_TEMPS || !sigma_S_per_m || !n_per_m3 || !mobility_cm2)
    return EPH_E_INVALID;
  for (int t = 0; t < n_temps; t++) {
    if (!(n_per_m3[t] > 0.0)) return EPH_E_INVALID;
    for (int q = 0; q < 9; q++) mobility_cm2[t * 9 + q] = sigma_S_per_m[t * 9 + q] / (n_per_m3[t] * kCharge) * 1e4;
  }
  return EPH_OK;
}

}  // extern "C"
