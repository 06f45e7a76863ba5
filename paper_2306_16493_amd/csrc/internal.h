// Internal declarations of the gfx950 EPWI library: context layout, device
// buffers and the host-side launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "eph.h"

namespace eph {

// Exact SI 2019 constants (amu: CODATA 2022).
constexpr double kPlanck = 6.62607015e-34;
constexpr double kCharge = 1.602176634e-19;
constexpr double kBoltz = 1.380649e-23;
constexpr double kAmu = 1.66053906892e-27;
constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxLine = EPH_MAX_LINE;

struct Units {
  double hbar_evs;   // hbar in eV s
  double kb_evk;     // k_B in eV/K
  double cph_ev;     // hbar^2/(amu A^2) in eV: (hbar w)^2 = cph * lambda
  double vel_unit;   // (1 eV A)/hbar in m/s
  double rate_pref;  // 2 pi / hbar in 1/(eV s)
};
Units units();

// Makes a device current for the lifetime of the guard and restores the
// caller's current device afterwards.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Grow-only device buffer.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  ~DevBuf();
  hipError_t ensure(size_t n);
  template <class T>
  T *as() const { return static_cast<T *>(p); }
};

struct RpBox {
  int lo[3];
  int n[3];
  int count() const { return n[0] * n[1] * n[2]; }
};

}  // namespace eph

struct eph_ctx {
  int device = 0;
  std::string err;
  // model
  int nw = 0, na = 0, nm = 0;
  double lattice[9];
  double volume = 0;  // A^3
  std::vector<double> mode_mass;  // [nm]
  int nrh = 0, nrd = 0, nre = 0, nrp = 0;
  eph::RpBox box;
  // device copies of the model
  eph::DevBuf rh, rh_w, rh_cart, ham;   // ham: [nrh][nw*nw] double2
  eph::DevBuf rd, rd_w, dyn;            // dyn: Phi/sqrt(MM') as double2 [nrd][nm*nm]
  // dense boxes of the weighted H(R) and D(R) for the separable Bloch sum
  // (empty when the R list does not fill its box well enough)
  eph::DevBuf hbox, dbox;
  int hbox_lo[3] = {0, 0, 0}, hbox_n[3] = {0, 0, 0}, dbox_lo[3] = {0, 0, 0}, dbox_n[3] = {0, 0, 0};
  eph::DevBuf re;                       // [nre][3] int
  eph::DevBuf wt64;                     // [nre*nw][box*nm*nw] double2 (K-major)
  eph::DevBuf wt32;                     // same in float2 (lazy)
  eph::DevBuf wtbf;                     // bf16 hi/lo split (lazy)
  eph::DevBuf mode_mass_d;              // [nm]
  // per-call workspaces (grow-only)
  eph::DevBuf tab;                      // e^{2 pi i m/N}, [N] double2
  eph::DevBuf eps, evec, vel, om, uu;   // grid tables
  eph::DevBuf evec32, uu32;             // FP32 copies for reduced forms
  eph::DevBuf eps32;                    // float band energies (prefilter of long lines)
  eph::DevBuf cnt, offs, scan_tmp, subset;
  eph::DevBuf grp_start, grp_tmp;
  eph::DevBuf line_e, line_key;         // energy-sorted p-lines
  eph::DevBuf xbuf;                     // X_s = Re transform + j rotation
  eph::DevBuf abf;                      // bf16 hi/lo state operand of the BF16x3 Re transform
  eph::DevBuf counters;                 // int64 counters
  eph::DevBuf sig_part;                 // sigma partial sums
  double *scratch = nullptr;            // device address of the static workspace (eph_conductivity_noalloc)
  eph::DevBuf state_cnt;                // per-state int64 counts
  eph::DevBuf stidx;                    // [N^3][nw] state index table (transition rates)
  eph::DevBuf gcur;                     // per-state transition-rate counts / cursors
  eph::DevBuf gstage_col, gstage_val;   // staging of spilled transition rates
  eph::DevBuf bte_f;                    // F0, F, F' of the iteration
  eph::DevBuf kb_g;                     // G_q of a q batch (k-batch order)
  eph::DevBuf occ;                      // Fermi and Bose factor tables
  eph::DevBuf occ32;                    // their FP32 copies (reduced-precision forms)
  // stage timing
  bool profiling = false;
  std::vector<hipEvent_t> ev;  // created on demand, reused across calls
  int64_t launches[2] = {0, 0};
  double stage_ms[5] = {0, 0, 0, 0, 0};
  ~eph_ctx() {
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

// Transition rates of the iterative BTE, row by row (CSR): row s holds the
// entries of state s, each a final-state index (into the same state list)
// and one value per temperature.  Kept in device memory, or in pinned host
// memory when it does not fit the device budget (streamed back in batches
// of rows for every iteration).
struct eph_gamma {
  eph_ctx *ctx = nullptr;
  int64_t ns = 0, nnz = 0;
  int nt = 0;
  double temps[EPH_MAX_TEMPS] = {0, 0, 0, 0};
  double mu = 0;
  bool on_host = false;
  std::vector<int64_t> h_row;   // [ns+1] row starts (host copy)
  eph::DevBuf row;              // [ns+1] row starts (device)
  eph::DevBuf col, val;         // device entries: col [nnz] int32, val [nt][nnz] (resident)
  int32_t *h_col = nullptr;     // pinned host entries (spilled)
  double *h_val = nullptr;      // [nt][nnz]
  int64_t stage_nnz = 0;        // entries per staging batch (spilled)
  ~eph_gamma();
};

namespace eph {

// ---- launchers (each returns the launch error) ----
// Bloch sum + Hermitian eigensolve on grid points [k0, k0+nk).
//  mode 0 (electrons): eval[k][n], evec[k][m][i] = V_im, vel[k][n][3] (m/s)
//  mode 1 (phonons):   eval[k][nu] = hbar w (eV), evec[k][nu][mu] = u_{mu nu}
//                      (A), zero for hbar w < omega_cut; counts excluded modes
hipError_t launch_bloch_eig(int mode, int n, int N, int64_t k0, int64_t nk, int nr, const int *R,
                            const double *w, const double *Rcart, const double2 *M, const double2 *tab,
                            const double *mode_mass, double cph, double omega_cut, double vel_unit,
                            double *eval, double2 *evec, double *vel, unsigned long long *n_excluded,
                            hipStream_t st);
hipError_t launch_phase_table(int N, double2 *tab, hipStream_t st);
// The same tables for all N^3 grid points from the separable form of the
// Bloch sum: Mb is the dense copy [nb0][nb1][nb2][n][n] of the weighted
// matrices on the box [lo, lo + nb) of R vectors (zero where the list has
// no vector), nb[0] <= kBoxMaxR1; lattice as rows a1, a2, a3 (Angstrom).
constexpr int kBoxMaxR1 = 12;
hipError_t launch_bloch_lines(int mode, int n, int N, const int *lo, const int *nb, const double *lattice,
                              const double2 *Mb, const double2 *tab, const double *mode_mass, double cph,
                              double omega_cut, double vel_unit, double *eval, double2 *evec, double *vel,
                              unsigned long long *n_excluded, hipStream_t st);

// State selection.  cnt/offs sized nklist+1.
hipError_t launch_count_states(int64_t nklist, const int64_t *klist, int nw, const double *eps, int blo,
                               int bhi, double wlo, double whi, int64_t *cnt, hipStream_t st);
hipError_t launch_scan(int64_t n, const int64_t *in, int64_t *out_excl, int64_t *tmp, hipStream_t st);
size_t scan_tmp_elems(int64_t n);
hipError_t launch_write_states(int64_t nklist, const int64_t *klist, int nw, const double *eps,
                               const double *vel, int blo, int bhi, double wlo, double whi,
                               const int64_t *offs, int32_t *sk, int32_t *sn, double *se, double *sv,
                               hipStream_t st);
// Group heads: states of one k-line (same i2,i3), chunks of at most gmax.
hipError_t launch_group_heads(int64_t ns, const int32_t *sk, int N, int gmax, int64_t *flag,
                              hipStream_t st);
hipError_t launch_group_starts(int64_t ns, const int64_t *flag, const int64_t *pos, int64_t *gstart,
                               hipStream_t st);
// Energy-sorted p-lines: for each line (i2,i3), entries key = i1*nw + m sorted by eps.
hipError_t launch_line_sort(int N, int nw, const double *eps, double *line_e, uint16_t *line_key,
                            hipStream_t st);

// Re transform fused with the j->n rotation:
//   X[s][rp][mu][i] = sum_{Re,j} Wt[(Re,j)][(rp,mu,i)] e^{i k_s.Re} V_{j n_s}(k_s)
hipError_t launch_xform64(int64_t ns, const int32_t *sk, const int32_t *sn, int N, int nw, int nre,
                          const int *re, int ncol, const double2 *wt, const double2 *evec,
                          const double2 *tab, double2 *X, hipStream_t st);
hipError_t launch_xform32(int64_t ns, const int32_t *sk, const int32_t *sn, int N, int nw, int nre,
                          const int *re, int ncol, const float2 *wt, const double2 *evec,
                          const double2 *tab, float2 *X, hipStream_t st);
hipError_t launch_real_to_f32(int64_t n, const double *in, float *out, hipStream_t st);
hipError_t launch_to_f32(int64_t n, const double2 *in, float2 *out, hipStream_t st);
// bf16 hi/lo split of the g operand in real form (2 * bf16_w_elems bf16 values)
size_t bf16_w_elems(int nre, int nw, int ncol);
// bf16 values per state of one half (hi or lo) of the state-side operand
size_t bf16_a_elems(int nre, int nw);
hipError_t launch_split_bf16(int nre, int nw, int ncol, const double2 *wt, void *out, hipStream_t st);
// abf: workspace of 2 * ns * bf16_a_elems bf16 values (the state operand, hi and lo)
hipError_t launch_xform_bf16x3(int64_t ns, const int32_t *sk, const int32_t *sn, int N, int nw, int nre,
                               const int *re, int ncol, const void *wbf, void *abf, const double2 *evec,
                               const double2 *tab, float2 *X, hipStream_t st);

struct RatesArgs {
  int N, nw, nm, nt;
  RpBox box;
  double mu, eta, sw, wcut, wmax;
  double temps_kt[EPH_MAX_TEMPS];  // k_B T in eV
  double pref;                     // 2 pi / hbar / N^3
  int64_t ng;                      // groups in this launch
  const int64_t *gstart;           // [ng+1] absolute state indices
  int64_t s_base;                  // state index of X row 0
  const int32_t *sk, *sn;
  const double *eps;               // [N^3][nw]
  const double *om;                // [N^3][nm]
  const double2 *evec;             // [N^3][nw][nw]
  const double2 *uu;               // [N^3][nm][nm]
  const float2 *evec32, *uu32;
  const float *eps32;              // float copy of eps (prefilter of lines longer than 512 energies)
  const double *line_e;
  const uint16_t *line_key;
  const double2 *tab;
  const void *X;                   // [ns][box][nm*nw] double2 or float2
  double *inv_tau;                 // [nt][ns_total]
  int64_t ns_total;
  int64_t *st_counts;              // [ns_total][2]: n_q_valid, n_terms
  unsigned long long *n_kq;
  unsigned long long *n_vertex;
  const double *occ_f;             // [N^3][nw][EPH_MAX_TEMPS] Fermi factors (wave kernel)
  const double *occ_n;             // [N^3][nm][EPH_MAX_TEMPS] Bose factors, 0 below omega_cut
  const float *occ32_f, *occ32_n;  // FP32 copies of occ_f, occ_n (reduced-precision forms)
  int q3_lo, q3_hi;                // q3 planes of this launch (wave kernel)
  int q3_cur;                      // the plane (wave kernel launches one plane at a time)
  // transition rates of the iterative BTE (wave kernel, FP64, count and emit modes)
  const int32_t *stidx;            // [N^3][nw] index of state (k, m) in the list, -1 if none
  int64_t *g_cursor;               // [ns_total] per-state count (count mode) or next position (emit)
  int32_t *g_col;                  // emitted final-state indices, position - g_base
  double *g_val;                   // emitted values [t][g_stride], 1/s
  int64_t g_stride;                // temperature stride of g_val
  int64_t g_base;                  // position of g_col[0] / g_val[0]
};
// rate-kernel modes (wave kernel)
constexpr int kRates = 0, kCount = 1, kEmit = 2;
hipError_t launch_rates(int precision, const RatesArgs &a, hipStream_t st);
// Wave-autonomous rate kernel; rates_wave_group gives its states per group
// (0 when the shape is not served and launch_rates must be used).
int rates_wave_group(int nw, int nm, RpBox box, int N, int precision);
hipError_t launch_rates_wave(int precision, const RatesArgs &a, hipStream_t st, int mode = kRates);
// k-batch order of the vertex (k_kbatch.hip): step 1 forms G_q for a batch
// of q, step 2 runs one wave per state over that batch.
struct KBatchArgs {
  int N, nw, nm, nt, nre, nb;
  int64_t q0, ns;
  double eta, sw, wcut, pref;
  const int32_t *sk, *sn;
  const int *re;
  const double *eps, *om;
  const double2 *evec, *tab, *Gq;
  const double *occ_f, *occ_n;
  double *inv_tau;
  int64_t *st_counts;
};
hipError_t launch_kbatch_step1(int64_t q0, int nb, int N, RpBox box, int nre, int nm, int nw, int ncol,
                               const double2 *wt, const double2 *uu, const double2 *tab, double2 *Gq, hipStream_t st);
hipError_t launch_kbatch_step2(const KBatchArgs &a, hipStream_t st);
// Occupation tables: occ_f[k][n][t] = 1/(exp((eps-mu)/kT_t)+1),
// occ_n[q][nu][t] = 1/expm1(hbar w/kT_t) (0 when hbar w < wcut).
hipError_t launch_occupations(int64_t nq, int nw, int nm, const double *eps, const double *om, double mu,
                              int nt, const double *kts_host, double wcut, double *occ_f, double *occ_n,
                              hipStream_t st);

// sigma partial sums per block, then out[T*9 + ab] = pref * sum of partials
// (partials: [nblk][EPH_MAX_TEMPS*9], out: [EPH_MAX_TEMPS*9], kts: device [nt]).
// order n weights each state by (eps - mu)^n (n = 0: sigma)
// F (optional, [nt][ns][3]) replaces v_b tau by the mean free path F_b.
hipError_t launch_sigma(int64_t ns, const double *e, const double *v, const double *inv_tau, double mu,
                        int nt, const double *kts, double pref, double *partials, int nblk, double *out,
                        hipStream_t st, int order = 0, const double *F = nullptr);
// iterative BTE (k_bte.hip)
hipError_t launch_state_index(int64_t nq, int nw, int64_t ns, const int32_t *sk, const int32_t *sn, int32_t *stidx,
                              hipStream_t st);
hipError_t launch_f0(int64_t ns, int nt, const double *vel, const double *inv_tau, double *F0, hipStream_t st);
hipError_t launch_bte_step(int64_t r0, int64_t r1, const int64_t *row_start, int64_t base, const int32_t *col,
                           const double *val, const double *inv_tau, const double *F0, const double *Fin, double *Fout,
                           hipStream_t st);
hipError_t launch_check_rows(int64_t ns, const int64_t *cursor, const int64_t *row_start, unsigned long long *bad,
                             hipStream_t st);
// out[t] = pref * sum_{k, blo <= n <= bhi} f(eps_nk) (partials: [nblk][EPH_MAX_TEMPS])
hipError_t launch_density(int64_t nk, int nw, const double *eps, int blo, int bhi, double mu, int nt,
                          const double *kts, double pref, double *partials, int nblk, double *out, hipStream_t st);
int rates_group_max(int nw, int nm);
hipError_t launch_zero(void *p, size_t bytes, hipStream_t st);
hipError_t launch_max_nonneg(int64_t n, const double *x, unsigned long long *out, hipStream_t st);
hipError_t launch_summarize(int64_t ns, const int64_t *st_counts, const double *inv_tau0,
                            unsigned long long *out, hipStream_t st);
size_t rates_smem_bytes(int precision, int N, int nw, int nm, RpBox box);

}  // namespace eph
