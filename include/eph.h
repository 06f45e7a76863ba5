/*
 * eph.h -- C ABI of the MI355X (gfx950) electron-phonon Wannier interpolation
 * (EPWI) SERTA transport library.
 *
 * The library computes, on one GPU, the quantities of arXiv 2306.16493:
 *   - Bloch Hamiltonian H(k) = sum_R w_R e^{ik.R} H(R), its eigenpairs and
 *     band velocities (Sec. II.B, Wannier interpolation of H; velocities are
 *     a preprocessing quantity of Sec. III.A);
 *   - dynamical matrix D(q) = sum_R w_R Phi(R)/sqrt(m m') e^{iq.R}, phonon
 *     energies hbar w and displacements u_{mu nu} = (hbar/2 m_mu w)^{1/2} e
 *     (Sec. II.B);
 *   - the interpolated vertex g_mn^nu(k,q) (Sec. II.B), in the bracket order
 *     of the q-batch algorithm (Sec. III.C);
 *   - SERTA scattering rates 1/tau_nk (Sec. II.C) over energy-conserving
 *     processes (the energy-conservation sieve of Sec. III.A);
 *   - the conductivity tensor sigma (Sec. II.C).
 *
 * Conventions shared by every call
 *   - Units: Angstrom, amu, eV, K, seconds; velocities m/s; sigma S/m.
 *   - Complex arrays are interleaved (re, im) doubles.
 *   - Lattice vectors are integer lattice coordinates (n1,n2,n3), R = sum n_i a_i.
 *   - The k and q grids are the same Gamma-centred N x N x N grid; grid point
 *     (i1,i2,i3) has reduced coordinates i/N and linear index
 *     i1 + N*(i2 + N*i3).  k+q is the grid point (i_k + i_q) mod N.
 *   - Eigenvectors: H V = V diag(eps), U = V^dagger, so the vertex reads
 *     g_mn^nu(k,q) = sum conj(V_im(k+q)) V_jn(k) e^{i(k.Re+q.Rp)}
 *                    g_ij^mu(Re,Rp) u_{mu nu}(q).
 *   - delta_eta(x) = exp(-x^2/eta^2) / (sqrt(pi) eta); a (q, m, nu, +-)
 *     term enters 1/tau when |eps_nk +- hbar w_qnu - eps_m,k+q| <=
 *     sieve_width*eta and hbar w_qnu >= omega_cut.
 *   - 1/tau carries the Brillouin-zone average 1/N^3 over q.
 *   - Every call returns an eph_status and never throws.  On an error the
 *     outputs are left untouched (except *counts on EPH_E_TRUNCATED) and
 *     eph_last_error() describes it.
 *   - A context is used by one host thread at a time.  Calls enqueue their
 *     work on the given HIP stream (NULL = the default stream) and
 *     synchronise that stream before they return host results.
 *   - Calls make the context's device current while they run and restore
 *     the caller's current device before they return.
 */
#ifndef EPH_H
#define EPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eph_ctx eph_ctx;

typedef enum {
  EPH_OK = 0,
  EPH_E_INVALID = 1,     /* bad argument, dimension or model property */
  EPH_E_NOMEM = 2,       /* device allocation failed */
  EPH_E_DEVICE = 3,      /* HIP runtime error (message in eph_last_error) */
  EPH_E_STATE = 4,       /* call on a context in an unusable state */
  EPH_E_TRUNCATED = 5,   /* output capacity too small; counts->n_states set */
  EPH_E_UNSUPPORTED = 6  /* valid input outside the implemented shapes */
} eph_status;

typedef enum {
  EPH_FP64 = 0,   /* every step in FP64 */
  EPH_FP32 = 1,   /* Re and Rp transforms and rotations in FP32 (FP32 tables);
                     eigensolves, energies, the sieve and the 1/tau and sigma
                     accumulations in FP64 */
  EPH_BF16X3 = 2  /* as EPH_FP32, but the Re transform on bf16 MFMA with the
                     split x = hi + lo and three products hi*hi + hi*lo +
                     lo*hi accumulated in FP32 */
} eph_precision;

/* Limits of this implementation (EPH_E_UNSUPPORTED beyond them). */
#define EPH_MAX_WANN 8    /* Wannier orbitals: 1, 2, 4 or 8 */
#define EPH_MAX_MODES 6   /* phonon modes 3*n_atoms: 3 or 6 */
#define EPH_MAX_TEMPS 4   /* temperatures per rates call */
#define EPH_MAX_GRID 512  /* N of the N x N x N grid */
#define EPH_MAX_LINE 2048 /* N * n_wann: energies on one final-state line */

/* The Wannier-basis model.  All pointers are HOST pointers; the data is
 * copied to the device by eph_load_wannier and the caller keeps ownership.
 *   lattice   rows a1, a2, a3 (Angstrom)
 *   mass_amu  [n_atoms]
 *   rh, rh_w  [n_rh][3] lattice coordinates and weights of H(R); the set
 *             must be closed under R -> -R with w(-R) = w(R)
 *   ham       [n_rh][n_wann][n_wann] complex, eV; H(-R) = H(R)^dagger
 *   rd, rd_w  [n_rd][3], weights; same closure rule
 *   ifc       [n_rd][3 n_atoms][3 n_atoms] real, eV/A^2, index 3*atom+axis;
 *             Phi(-R) = Phi(R)^T
 *   re        [n_re][3] electron lattice vectors of g (any set)
 *   rp        [n_rp][3] phonon lattice vectors of g; must form a full box
 *             {lo_i .. lo_i + n_i - 1} per coordinate (n_i <= 16), any order
 *   gw        [n_re][n_rp][3 n_atoms][n_wann(i)][n_wann(j)] complex, eV/A
 *             (g_ij^mu(Re, Rp)); i pairs with k+q, j with k.            */
typedef struct {
  double lattice[9];
  int32_t n_atoms;
  const double *mass_amu;
  int32_t n_wann;
  int32_t n_rh;
  const int32_t *rh;
  const double *rh_w;
  const double *ham;
  int32_t n_rd;
  const int32_t *rd;
  const double *rd_w;
  const double *ifc;
  int32_t n_re;
  const int32_t *re;
  int32_t n_rp;
  const int32_t *rp;
  const double *gw;
} eph_model;

/* Validate the model (Hermiticity of H(R) and Phi(R) pairs to 1e-12 of the
 * largest element, closure of the R sets, positive weights and masses,
 * dimensions), select HIP device `device`, copy the model to it and return
 * a new context in *out.  Errors: EPH_E_INVALID, EPH_E_UNSUPPORTED,
 * EPH_E_NOMEM, EPH_E_DEVICE; *out is set to NULL on error.  The paper's
 * input stage (Sec. III.A) reads these Wannier-basis quantities from EPW. */
int32_t eph_load_wannier(const eph_model *model, int32_t device, eph_ctx **out);

/* Release a context and all its device memory.  NULL is accepted. */
void eph_free(eph_ctx *ctx);

/* Message of the last failed call on ctx (or of the last failed
 * eph_load_wannier in this thread when ctx is NULL).  Valid until the next
 * call on the same context. */
const char *eph_last_error(const eph_ctx *ctx);

typedef struct {
  int32_t grid[3];          /* N, N, N (all three equal, 1..EPH_MAX_GRID) */
  double mu_eV;             /* chemical potential */
  int32_t n_temps;          /* 1..EPH_MAX_TEMPS */
  const double *temps_K;    /* host [n_temps], each > 0 */
  double eta_eV;            /* Gaussian smearing, > 0 */
  double sieve_width;       /* keep |x| <= sieve_width*eta; > 0 (6 is usual) */
  double win_lo_eV;         /* state window on eps_nk (inclusive) */
  double win_hi_eV;
  int32_t band_lo;          /* initial-state bands band_lo..band_hi */
  int32_t band_hi;          /* < 0 means the last band */
  double omega_cut_eV;      /* phonon modes below are dropped (>= 0) */
  int32_t precision;        /* eph_precision */
  const int64_t *k_subset;  /* optional host list of k indices whose window
                               states are computed (duplicates ignored);
                               NULL = every k of the grid */
  int64_t n_k_subset;
  int64_t mem_budget_bytes; /* device workspace this call may use (grid
                               tables, state lists, per-batch buffers);
                               the states are processed in batches sized
                               to fit.  0 = automatic (per-batch buffers up
                               to the free device memory less 8 GiB, at
                               least 8 and at most 64 GiB; 8 GiB when
                               transition rates are built; the context
                               keeps them for later calls until
                               eph_free).  EPH_E_NOMEM, with the required
                               size in eph_last_error, when the tables and
                               one group of states do not fit. */
  void *stream;             /* hipStream_t, NULL = default stream */
} eph_rates_params;

typedef struct {
  int64_t n_states;          /* initial states (n,k) selected */
  int64_t n_kq;              /* (k,q) pairs with >= 1 kept term for a state at k */
  int64_t n_nkq;             /* (n,k,q) with >= 1 kept term */
  int64_t n_terms;           /* kept (n,k,q,m,nu,+-) terms */
  int64_t n_zero_rate;       /* states whose 1/tau is 0 at the first temperature */
  int64_t n_excluded_modes;  /* (q,nu) with hbar w < omega_cut on the grid */
  int64_t n_vertex;          /* (n,k,q,m) vertex contractions evaluated: final
                                bands m with >= 1 kept (nu, +-) term */
} eph_counts;

/* SERTA scattering rates (Sec. II.C) of every selected state.
 * States are the (n,k) with band_lo <= n <= band_hi and
 * win_lo_eV <= eps_nk <= win_hi_eV (k restricted to k_subset if given),
 * ordered by k index, then n.
 * Outputs are caller-owned DEVICE buffers on the context's device:
 *   state_k [capacity] int32, state_n [capacity] int32,
 *   energy_eV [capacity], vel_ms [capacity][3],
 *   inv_tau_s [n_temps][n_states] (packed with stride n_states), 1/s.
 * counts is a host pointer (may be NULL).
 * If capacity < n_states nothing is written except *counts (n_states set,
 * the other counts 0) and EPH_E_TRUNCATED is returned; calling with
 * capacity 0 is the way to size the outputs.
 * Every grid quantity (eigenpairs, velocities, phonons) is recomputed from
 * the Wannier model by each call. */
int32_t eph_scattering_rates(eph_ctx *ctx, const eph_rates_params *params, int64_t capacity,
                             int32_t *state_k, int32_t *state_n, double *energy_eV,
                             double *vel_ms, double *inv_tau_s, eph_counts *counts);

/* The state selection of eph_scattering_rates alone: the same grid tables
 * and window, the same outputs except inv_tau, no rates (all counts other
 * than n_states and n_excluded_modes are 0).  Used by callers that compute
 * rates for a part of the states only (k_subset) or estimate them. */
int32_t eph_select_states(eph_ctx *ctx, const eph_rates_params *params, int64_t capacity, int32_t *state_k,
                          int32_t *state_n, double *energy_eV, double *vel_ms, eph_counts *counts);

/* Conductivity tensor (Sec. II.C) from per-state data, in S/m:
 *   sigma_ab(T) = 2 e^2/(n_kpoints V) sum_s v_a v_b tau_s f(1-f)/(k_B T),
 * tau_s = 1/inv_tau_s(T); states with inv_tau = 0 are skipped.  V is the
 * cell volume of the loaded lattice.
 * energy_eV [n_states], vel_ms [n_states][3], inv_tau_s [n_temps][n_states]
 * are DEVICE pointers (e.g. the outputs of eph_scattering_rates, a
 * surrogate's rates, or a constant-tau test); temps_K and sigma_S_per_m
 * ([n_temps][3][3]) are HOST pointers.  The reduction is FP64 in a fixed
 * order, so repeated calls give bit-identical results. */
int32_t eph_conductivity(eph_ctx *ctx, int64_t n_states, const double *energy_eV,
                         const double *vel_ms, const double *inv_tau_s, double mu_eV,
                         int32_t n_temps, const double *temps_K, int64_t n_kpoints,
                         void *stream, double *sigma_S_per_m);

/* eph_conductivity for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same kernels and the same bit-identical
 * result, but the reduction's workspace is a static device array of
 * 9,328 doubles (74,624 bytes) per GPU, set up by eph_load_wannier and held
 * until the process ends; the call itself allocates nothing.  The workspace
 * does not grow with n_states, so the only size limit is n_temps <=
 * EPH_MAX_TEMPS (EPH_E_INVALID beyond it).  Every call on one GPU shares
 * that GPU's array: calls that overlap in time on one GPU (several host
 * threads or streams) race and must be serialised by the caller.
 * EPH_E_STATE if the context has no workspace address. */
int32_t eph_conductivity_noalloc(eph_ctx *ctx, int64_t n_states, const double *energy_eV,
                                 const double *vel_ms, const double *inv_tau_s, double mu_eV,
                                 int32_t n_temps, const double *temps_K, int64_t n_kpoints,
                                 void *stream, double *sigma_S_per_m);

/* Transport coefficients (Sec. II.C, the coefficients built from the same
 * relaxation-time sums as sigma).  With energies in eV and
 *   M_n,ab(T) = 2 e^2/(n_kpoints V) sum_s v_a v_b tau_s f(1-f)/(k_B T)
 *               (eps_s - mu)^n,          n = 0, 1, 2,
 * the outputs ([n_temps][3][3], HOST) are
 *   sigma_S_per_m   = M_0,
 *   seebeck_V_per_K = -M_0^-1 M_1 / T          (carriers of charge -e),
 *   kappa_W_per_mK  = (M_2 - M_1 M_0^-1 M_1) / T (electronic thermal
 *                     conductivity at zero electric current).
 * Inputs as eph_conductivity (DEVICE state arrays, HOST temperatures); the
 * three moments are fixed-order FP64 device reductions, the 3x3 algebra is
 * done on the host.  A singular sigma gives non-finite S and kappa. */
int32_t eph_transport(eph_ctx *ctx, int64_t n_states, const double *energy_eV, const double *vel_ms,
                      const double *inv_tau_s, double mu_eV, int32_t n_temps, const double *temps_K,
                      int64_t n_kpoints, void *stream, double *sigma_S_per_m, double *seebeck_V_per_K,
                      double *kappa_W_per_mK);

/* ------------------------------------------------------------------------
 * Iterative solution of the linearised BTE (Sec. II.C, iteration equation;
 * Sec. III.E, compressed storage).  The transition rates of a state
 * s = (n,k) to a final state (m, k+q) are
 *   Gamma_s(q,m) = (2 pi/hbar)(1/N^3) sum_nu |g_mn^nu(k,q)|^2
 *                  [(N_qnu + f_m,k+q) delta(x+) + (1 + N_qnu - f_m,k+q) delta(x-)],
 * the terms of 1/tau_s before they are summed over (q, m), so that
 * sum_{q,m} Gamma_s(q,m) = 1/tau_s; they carry the same sieve and factors
 * as the rates.  Only entries whose final state is itself a selected state
 * are stored (any other final state is not part of the solution and carries
 * F = 0).  Storage is by rows (CSR): row s holds, for each entry, the index
 * of the final state in the state list (int32) and one FP64 value per
 * temperature, values laid out [n_temps][nnz].  The iteration is
 *   F^{i+1}_s = F0_s + tau_s sum_e Gamma_e F^i_{col_e},  F0 = v tau,
 * and sigma after each iteration is
 *   sigma_ab = 2 e^2/(n_kpoints V k_B T) sum_s v_a F_b f(1-f)
 * (iteration 0 is the SERTA sigma of eph_conductivity).  States with
 * 1/tau = 0 keep F = 0.  Available for FP64 on the Rp boxes served by the
 * wave rate kernel (cubic, edge 4 or 6); EPH_E_UNSUPPORTED otherwise.
 * ------------------------------------------------------------------------ */
typedef struct eph_gamma eph_gamma;

/* Memory estimate of the transition rates before they are computed (the
 * preprocessing estimate of Sec. III.A): runs the state selection and the
 * energy-conservation sieve only, and returns the number of stored entries
 * (*nnz) and their bytes (*bytes = nnz (4 + 8 n_temps) + 8 (n_states + 1)).
 * State outputs as eph_select_states (DEVICE buffers, capacity in states;
 * EPH_E_TRUNCATED with capacity < n_states). */
int32_t eph_gamma_estimate(eph_ctx *ctx, const eph_rates_params *params, int64_t capacity, int32_t *state_k,
                           int32_t *state_n, double *energy_eV, double *vel_ms, int64_t *nnz, int64_t *bytes);

/* eph_scattering_rates (same arguments and outputs) that also builds the
 * transition rates into *gamma (free with eph_gamma_free).  A counting pass
 * (the sieve only) sizes the rows first.  The rows stay in device memory
 * when they fit mem_budget_bytes beside the call's other buffers (with
 * mem_budget_bytes = 0: when they fit the free device memory with 1 GiB to
 * spare); otherwise they are written batch by batch, through a device
 * staging buffer, to pinned host memory (the host spill of Sec. III.E), and
 * eph_bte_iterate streams them back.  The rows of a state follow the order
 * in which the kernel evaluates its vertices, which is fixed, so repeated
 * calls give identical rows.  EPH_E_NOMEM when neither fits. */
int32_t eph_rates_gamma(eph_ctx *ctx, const eph_rates_params *params, int64_t capacity, int32_t *state_k,
                        int32_t *state_n, double *energy_eV, double *vel_ms, double *inv_tau_s, eph_counts *counts,
                        eph_gamma **gamma);

/* Size and placement: states (rows), entries, temperatures, 1 if the rows
 * are in pinned host memory, bytes.  Any output may be NULL. */
int32_t eph_gamma_info(const eph_gamma *gamma, int64_t *n_states, int64_t *nnz, int32_t *n_temps, int32_t *on_host,
                       int64_t *bytes);

/* Copy the rows to HOST arrays (any may be NULL): row_start [n_states+1],
 * col [nnz] (final-state index in the state list), val [n_temps][nnz] (1/s). */
int32_t eph_gamma_copy(const eph_gamma *gamma, int64_t *row_start, int32_t *col, double *val);

void eph_gamma_free(eph_gamma *gamma); /* NULL-safe */

/* Iterate from F0 = v tau until the largest change of sigma is <= tol times
 * its largest element, or max_iter iterations.  energy_eV [n_states],
 * vel_ms [n_states][3] and inv_tau_s [n_temps][n_states] are the DEVICE
 * outputs of the eph_rates_gamma call that built gamma (temperatures and mu
 * are those of that call).  sigma_iter (HOST, [max_iter+1][n_temps][3][3])
 * receives sigma after iterations 0..*n_iter; F_out (DEVICE
 * [n_temps][n_states][3], may be NULL) the final mean free paths in m.  The
 * iteration step is FP64 with a fixed summation order. */
int32_t eph_bte_iterate(eph_ctx *ctx, const eph_gamma *gamma, const double *energy_eV, const double *vel_ms,
                        const double *inv_tau_s, int64_t n_kpoints, int32_t max_iter, double tol, void *stream,
                        double *sigma_iter, int32_t *n_iter, double *F_out);

/* Carrier density for mobilities (Sec. II.C, mobility = sigma / (n e)):
 *   n(T) = 2/(N^3 V) sum_{all k of the N^3 grid} sum_{band_lo <= n <= band_hi} f(eps_nk)
 * in m^-3 into n_per_m3 [n_temps] (HOST).  The band energies are computed on
 * the full grid on the device (the electron half of the grid tables).
 * EPH_E_INVALID for a bad grid (1..EPH_MAX_GRID), band range or
 * temperature. */
int32_t eph_carrier_density(eph_ctx *ctx, int32_t grid, int32_t band_lo, int32_t band_hi, double mu_eV,
                            int32_t n_temps, const double *temps_K, void *stream, double *n_per_m3);

/* Mobility tensor mu_ab = sigma_ab / (n e) in cm^2/(V s), from HOST arrays
 * sigma_S_per_m [n_temps][3][3] and n_per_m3 [n_temps] into mobility_cm2
 * [n_temps][3][3].  EPH_E_INVALID when a density is not positive. */
int32_t eph_mobility(int32_t n_temps, const double *sigma_S_per_m, const double *n_per_m3, double *mobility_cm2);

/* The same SERTA rates (same arguments and outputs as eph_scattering_rates)
 * computed in the other association of the vertex sum, the k-batch order of
 * Sec. III.D, kept to measure the comparison of that section on this GPU:
 * for each batch of q_batch wave vectors q, G_q(Re; nu, i, j) =
 * sum_{Rp,mu} e^{iq.Rp} g(Re, Rp) u_{mu nu}(q) is formed, then every state
 * takes sum_Re e^{ik.Re} G_q and the band rotations at each q of the batch.
 * Its volume per (k,q) pair is N_w^2 N_Re N_nu complex multiply-adds, against
 * N_w N_nu N_Rp per (n,k,q) of the q-batch order.  FP64 only, on the Rp
 * boxes the wave kernel serves (EPH_E_UNSUPPORTED otherwise); counts->n_kq
 * and n_vertex are not counted (0).  With profiling on, eph_stage_times
 * reports step 1 as ms[2] and step 2 as ms[3], and the number of q batches. */
int32_t eph_rates_kbatch(eph_ctx *ctx, const eph_rates_params *params, int64_t capacity, int32_t *state_k,
                         int32_t *state_n, double *energy_eV, double *vel_ms, double *inv_tau_s, eph_counts *counts,
                         int32_t q_batch);

/* Stage timing.  With profiling on, eph_scattering_rates records HIP events
 * on its stream around its stages; eph_stage_times then returns their GPU
 * durations in milliseconds for the last call:
 *   ms[0] grid tables (Bloch sums, eigensolves, velocities, phonons)
 *   ms[1] state selection, grouping, energy-sorted lines
 *   ms[2] Re transform (all launches)
 *   ms[3] rate kernel (all launches)
 *   ms[4] whole call (first to last event)
 * and in launches[0] / launches[1] the number of Re-transform and
 * rate-kernel launches.  ms needs 5 doubles, launches 2 int64 (host).
 * Profiling is off by default; it adds event records but no
 * synchronisation beyond the one each call already does. */
int32_t eph_set_profiling(eph_ctx *ctx, int32_t on);
int32_t eph_stage_times(const eph_ctx *ctx, double *ms, int64_t *launches);

/* ------------------------------------------------------------------------
 * Learned form: an ensemble of multilayer perceptrons that predicts
 * log(1/tau) of a state from its features, trained on rates that
 * eph_scattering_rates computed on a subset of k points.  Where the members
 * disagree the caller recomputes the rates with eph_scattering_rates
 * (k_subset) and merges them with eph_merge_rates.  This form is not in the
 * paper; it stands beside the SERTA rates of Sec. II.C.
 * Network: features (10) -> 128 -> 128 -> 128 -> n_out, SiLU, FP32; Adam on
 * the mean squared error of normalised log(1/tau); n_out = temperatures.
 * Parameter layout per member (row-major W[out][in]):
 *   W1[128][10] b1[128] W2[128][128] b2 W3[128][128] b3 W4[n_out][128] b4.
 * All array arguments are DEVICE pointers unless marked host.
 * ------------------------------------------------------------------------ */
typedef struct eph_mlp eph_mlp;

/* Create n_members (1..64) networks with n_out (1..EPH_MAX_TEMPS) outputs,
 * weights drawn from a counter-based hash of seed.  Errors: EPH_E_INVALID,
 * EPH_E_NOMEM, EPH_E_DEVICE. */
int32_t eph_mlp_create(eph_ctx *ctx, int32_t n_members, int32_t n_out, uint64_t seed, eph_mlp **out);
void eph_mlp_free(eph_mlp *mlp); /* NULL-safe */

/* Parameter count per member in *n_params; with host_params non-NULL, copy
 * all members' parameters ([n_members][n_params] floats) out (set = 0) or
 * in (set = 1). */
int32_t eph_mlp_params(eph_mlp *mlp, float *host_params, int64_t *n_params, int32_t set);

/* Features x[n][10] = (sin 2pi k1/N, cos 2pi k1/N, the same for k2 and k3,
 * eps - mu [eV], v [1e6 m/s] x3) of states (state_k, energy_eV, vel_ms as
 * returned by eph_scattering_rates): the reduced k coordinates enter through
 * periodic functions, as the rates are periodic over the zone.  With
 * inv_tau_s ([n_temps][n]) also the targets y[n][n_temps] = log(inv_tau).
 * Enqueued on stream. */
int32_t eph_mlp_features(eph_ctx *ctx, int64_t n, const int32_t *state_k, const double *energy_eV,
                         const double *vel_ms, int32_t grid, double mu_eV, const double *inv_tau_s,
                         int32_t n_temps, float *x, float *y, void *stream);

/* Train every member for `steps` Adam steps (lr, beta 0.9/0.999) on
 * minibatches of `batch` samples (multiple of 32) drawn independently per
 * member from the n samples.  The first call fixes the input/target
 * normalisation from its data.  loss (host, may be NULL) receives each
 * member's last minibatch loss.  Synchronises the stream. */
int32_t eph_mlp_train(eph_mlp *mlp, int64_t n, const float *x, const float *y, int32_t steps,
                      int32_t batch, float lr, void *stream, float *loss);

/* Gradient of the loss over all n samples (multiple of 32, taken as already
 * normalised) w.r.t. every parameter, into grad (host, [n_members][n_params]);
 * loss (host, may be NULL) per member.  For checking the backward kernels. */
int32_t eph_mlp_gradient(eph_mlp *mlp, int64_t n, const float *x, const float *y, float *grad, float *loss);

/* y[n_members][n][n_out] = each member's prediction of log(1/tau). */
int32_t eph_mlp_predict(eph_mlp *mlp, int64_t n, const float *x, float *y, void *stream);

/* Ensemble mean of exp(y) into inv_tau_s [n_out][n]; flag[s] = 1 where the
 * relative spread (std / mean over members, largest over outputs) exceeds
 * threshold; *n_flagged (host) counts them.  Synchronises the stream. */
int32_t eph_mlp_blend(eph_mlp *mlp, int64_t n, const float *y, double threshold, double *inv_tau_s,
                      int32_t *flag, int64_t *n_flagged, void *stream);

/* Overwrite full_inv_tau [n_temps][n_full] at the states (k, n) of the sub
 * list with sub_inv_tau [n_temps][n_sub]; both lists sorted by k then n, as
 * eph_scattering_rates returns them.  Sub states absent from the full list
 * are ignored. */
int32_t eph_merge_rates(eph_ctx *ctx, int64_t n_full, const int32_t *full_k, const int32_t *full_n,
                        int64_t n_sub, const int32_t *sub_k, const int32_t *sub_n, const double *sub_inv_tau,
                        int32_t n_temps, double *full_inv_tau, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* EPH_H */
