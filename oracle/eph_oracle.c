/*
 * Plain FP64 CPU oracle for the electron-phonon Wannier interpolation (EPWI)
 * SERTA transport path of arXiv 2306.16493.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP library is checked against.  Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or table with the HIP library.
 *
 * Every routine evaluates the paper's equations literally, in FP64:
 *   electrons   H(k) = sum_R w_R e^{ik.R} H(R), Hermitian eigensolve
 *               (Sec. II.B, Wannier interpolation of H); band velocities by
 *               the Hellmann-Feynman diagonal of dH/dk (the paper computes
 *               velocities in preprocessing, Sec. III.A, without a formula).
 *   phonons     D(q) = sum_R Phi(R)/sqrt(m m') e^{iq.R}, D e = w^2 e
 *               (Sec. II.B, dynamical-matrix equations);
 *               u_{mu nu} = (hbar / 2 m_mu w_nu)^{1/2} e^nu_mu.
 *   vertex      g_mn^nu(k,q) = sum_{ij mu Re Rp} U_mi(k+q) U+_jn(k)
 *               e^{i(k.Re+q.Rp)} g_ij^mu(Re,Rp) u_mu nu(q)
 *               (Sec. II.B, interpolation of g), associated in the q-batch
 *               bracket order of Sec. III.C: first the Re sum at fixed k,
 *               then the Rp sum at each q, then the band/mode rotations.
 *   rates       SERTA 1/tau (Sec. II.C), Gaussian delta, 1/N_q BZ average.
 *   sigma       sigma = 2 e^2/(N_k V) sum v v tau f(1-f)/(k_B T) (Sec. II.C).
 *   transport   sigma, Seebeck and electronic thermal conductivity from the
 *               (eps - mu)^n moments of the same sum (Sec. II.C);
 *               carrier density for mobilities.
 *   iteration   transition rates Gamma_nm(k,k+q) (the terms of 1/tau before
 *               the sum over final states) and the iterative solution
 *               F^{i+1} = F^0 + tau sum Gamma F^i with sigma per iteration
 *               (Sec. II.C iteration equation, Sec. III.E).
 * Loop order is the paper's CPU algorithm (Sec. III.A): outer loop over the
 * k points that carry states, inner loop over all q; OpenMP over k points.
 *
 * Readings where the paper is silent (listed in the design notes):
 *   U = V^dagger with H V = V diag(eps), so U_mi(k+q) = conj(V_im(k+q)) and
 *   U+_jn(k) = V_jn(k);  phases e^{+i k.R};  delta_eta(x) =
 *   exp(-x^2/eta^2)/(sqrt(pi) eta);  a term is kept when |x| <= sw*eta;
 *   phonon modes with hbar w < omega_cut are dropped;  states with
 *   1/tau = 0 are left out of sigma.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <complex.h>

typedef double complex cplx;

/* ---- constants: exact SI 2019 values (amu: CODATA 2022) ---- */
#define ORC_H 6.62607015e-34
#define ORC_E 1.602176634e-19
#define ORC_KB 1.380649e-23
#define ORC_AMU 1.66053906892e-27
#define ORC_PI 3.14159265358979323846

static double hbar_js(void) { return ORC_H / (2.0 * ORC_PI); }
double orc_hbar_evs(void) { return hbar_js() / ORC_E; }
double orc_kb_evk(void) { return ORC_KB / ORC_E; }
/* (hbar w)^2 [eV^2] = C * lambda [eV/(A^2 amu)];  C = hbar^2/(amu A^2) in eV */
double orc_cph_ev(void) { return hbar_js() * hbar_js() / (ORC_AMU * 1e-20) / ORC_E; }
/* 1 eV*A / hbar in m/s */
double orc_vel_unit(void) { return ORC_E * 1e-10 / hbar_js(); }

typedef struct {
  double lattice[9];
  int32_t na;
  const double *mass;
  int32_t nw;
  int32_t nrh;
  const int32_t *rh;
  const double *rh_w;
  const double *ham; /* [nrh][nw][nw] complex interleaved */
  int32_t nrd;
  const int32_t *rd;
  const double *rd_w;
  const double *ifc; /* [nrd][3na][3na] */
  int32_t nre;
  const int32_t *re;
  int32_t nrp;
  const int32_t *rp;
  const double *gw; /* [nre][nrp][3na][nw][nw] complex interleaved */
} orc_model;

/* e^{i 2 pi (k.n)/N} with the argument reduced exactly in integers */
static cplx phase(const int64_t k[3], const int32_t n[3], int64_t N) {
  int64_t s = 0;
  for (int a = 0; a < 3; a++) {
    int64_t t = (k[a] * (int64_t)n[a]) % N;
    s = (s + t) % N;
  }
  if (s < 0) s += N;
  double ang = 2.0 * ORC_PI * (double)s / (double)N;
  return cos(ang) + I * sin(ang);
}

static void grid_coords(int64_t idx, int64_t N, int64_t k[3]) {
  /* linear index = k1 + N*(k2 + N*k3), k1 fastest */
  k[0] = idx % N;
  k[1] = (idx / N) % N;
  k[2] = idx / (N * N);
}

static int64_t grid_index(const int64_t k[3], int64_t N) {
  int64_t a = ((k[0] % N) + N) % N, b = ((k[1] % N) + N) % N, c = ((k[2] % N) + N) % N;
  return a + N * (b + N * c);
}

/* ---------------------------------------------------------------------
 * Hermitian eigensolver: cyclic complex Jacobi.  A (n x n, row-major) is
 * destroyed; on return w[] holds eigenvalues ascending and V (row-major,
 * V[i*n+m] = component i of eigenvector m) the orthonormal eigenvectors.
 * Each rotation first removes the phase of a_pq, then applies the real
 * symmetric Jacobi rotation that annihilates it (Rutishauser's formulas).
 * -------------------------------------------------------------------*/
void orc_heevj(int n, cplx *A, double *w, cplx *V) {
  for (int i = 0; i < n; i++)
    for (int j = 0; j < n; j++) V[i * n + j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; sweep++) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; i++)
      for (int j = 0; j < n; j++) {
        double a2 = creal(A[i * n + j]) * creal(A[i * n + j]) + cimag(A[i * n + j]) * cimag(A[i * n + j]);
        tot += a2;
        if (i != j) off += a2;
      }
    if (off == 0.0 || off <= 1e-33 * tot) break;
    for (int p = 0; p < n - 1; p++)
      for (int q = p + 1; q < n; q++) {
        cplx apq = A[p * n + q];
        double g = cabs(apq);
        if (g == 0.0) continue;
        cplx eph = apq / g; /* e^{i phi} */
        double app = creal(A[p * n + p]), aqq = creal(A[q * n + q]);
        double theta = (aqq - app) / (2.0 * g);
        double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        /* J (on columns p,q): J_pp = c, J_pq = s e^{i phi}, J_qp = -s e^{-i phi}... written out:
           new column p = c*col_p - s*conj(eph)*col_q,  new column q = s*eph*col_p + c*col_q  */
        cplx jpp = c, jqp = -s * conj(eph), jpq = s * eph, jqq = c;
        for (int i = 0; i < n; i++) { /* A <- A J */
          cplx ap = A[i * n + p], aq = A[i * n + q];
          A[i * n + p] = ap * jpp + aq * jqp;
          A[i * n + q] = ap * jpq + aq * jqq;
        }
        for (int j = 0; j < n; j++) { /* A <- J^H A */
          cplx ap = A[p * n + j], aq = A[q * n + j];
          A[p * n + j] = conj(jpp) * ap + conj(jqp) * aq;
          A[q * n + j] = conj(jpq) * ap + conj(jqq) * aq;
        }
        A[p * n + q] = 0.0;
        A[q * n + p] = 0.0;
        A[p * n + p] = creal(A[p * n + p]);
        A[q * n + q] = creal(A[q * n + q]);
        for (int i = 0; i < n; i++) { /* V <- V J */
          cplx vp = V[i * n + p], vq = V[i * n + q];
          V[i * n + p] = vp * jpp + vq * jqp;
          V[i * n + q] = vp * jpq + vq * jqq;
        }
      }
  }
  for (int i = 0; i < n; i++) w[i] = creal(A[i * n + i]);
  /* selection sort ascending, permuting eigenvector columns */
  for (int i = 0; i < n - 1; i++) {
    int m = i;
    for (int j = i + 1; j < n; j++)
      if (w[j] < w[m]) m = j;
    if (m != i) {
      double tw = w[i]; w[i] = w[m]; w[m] = tw;
      for (int r = 0; r < n; r++) {
        cplx tv = V[r * n + i]; V[r * n + i] = V[r * n + m]; V[r * n + m] = tv;
      }
    }
  }
}

/* ---------------------------------------------------------------------
 * Electrons on grid points: eps[k][n], evec[k][m][i] = V_im(k) (row m is
 * eigenvector m), vel[k][n][3] in m/s.  Any pointer may be NULL.
 * -------------------------------------------------------------------*/
void orc_electrons(const orc_model *md, int64_t N, int64_t nk, const int64_t *kidx,
                   double *eps, double *evec, double *vel) {
  const int nw = md->nw;
  const double vu = orc_vel_unit();
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nk; t++) {
    cplx H[32 * 32], dH[3][32 * 32], V[32 * 32];
    double w[32];
    int64_t k[3];
    grid_coords(kidx[t], N, k);
    for (int e = 0; e < nw * nw; e++) {
      H[e] = 0;
      dH[0][e] = dH[1][e] = dH[2][e] = 0;
    }
    for (int r = 0; r < md->nrh; r++) {
      const int32_t *n = md->rh + 3 * r;
      cplx ph = md->rh_w[r] * phase(k, n, N);
      double Rc[3];
      for (int a = 0; a < 3; a++)
        Rc[a] = n[0] * md->lattice[0 * 3 + a] + n[1] * md->lattice[1 * 3 + a] + n[2] * md->lattice[2 * 3 + a];
      const double *h = md->ham + (size_t)r * nw * nw * 2;
      for (int e = 0; e < nw * nw; e++) {
        cplx he = h[2 * e] + I * h[2 * e + 1];
        H[e] += ph * he;
        for (int a = 0; a < 3; a++) dH[a][e] += I * Rc[a] * ph * he;
      }
    }
    cplx A[32 * 32];
    memcpy(A, H, sizeof(cplx) * nw * nw);
    orc_heevj(nw, A, w, V);
    if (eps)
      for (int n = 0; n < nw; n++) eps[t * nw + n] = w[n];
    if (evec)
      for (int m = 0; m < nw; m++)
        for (int i = 0; i < nw; i++) {
          cplx v = V[i * nw + m];
          evec[((t * nw + m) * nw + i) * 2] = creal(v);
          evec[((t * nw + m) * nw + i) * 2 + 1] = cimag(v);
        }
    if (vel)
      for (int n = 0; n < nw; n++)
        for (int a = 0; a < 3; a++) {
          cplx s = 0;
          for (int i = 0; i < nw; i++)
            for (int j = 0; j < nw; j++) s += conj(V[i * nw + n]) * dH[a][i * nw + j] * V[j * nw + n];
          vel[(t * nw + n) * 3 + a] = creal(s) * vu;
        }
  }
}

/* ---------------------------------------------------------------------
 * Phonons on grid points: omega[q][nu] = hbar w in eV (ascending; lambda<0
 * from rounding is clamped to 0), u[q][nu][mu] = u_{mu nu}(q) in Angstrom
 * (zero for modes below omega_cut), complex interleaved.
 * -------------------------------------------------------------------*/
void orc_phonons(const orc_model *md, int64_t N, int64_t nq, const int64_t *qidx, double omega_cut,
                 double *omega, double *u, double *lambda_out) {
  const int nm = 3 * md->na;
  const double C = orc_cph_ev();
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t t = 0; t < nq; t++) {
    cplx D[256], V[256];
    double w[16];
    int64_t q[3];
    grid_coords(qidx[t], N, q);
    for (int e = 0; e < nm * nm; e++) D[e] = 0;
    for (int r = 0; r < md->nrd; r++) {
      cplx ph = md->rd_w[r] * phase(q, md->rd + 3 * r, N);
      const double *f = md->ifc + (size_t)r * nm * nm;
      for (int a = 0; a < nm; a++)
        for (int b = 0; b < nm; b++)
          D[a * nm + b] += ph * f[a * nm + b] / sqrt(md->mass[a / 3] * md->mass[b / 3]);
    }
    orc_heevj(nm, D, w, V);
    for (int nu = 0; nu < nm; nu++) {
      double lam = w[nu];
      if (lambda_out) lambda_out[t * nm + nu] = lam;
      double hw = sqrt(C * (lam > 0 ? lam : 0.0));
      if (omega) omega[t * nm + nu] = hw;
      for (int mu = 0; mu < nm; mu++) {
        cplx val = 0;
        if (hw >= omega_cut) val = V[mu * nm + nu] * sqrt(C / (2.0 * md->mass[mu / 3] * hw));
        if (u) {
          u[((t * nm + nu) * nm + mu) * 2] = creal(val);
          u[((t * nm + nu) * nm + mu) * 2 + 1] = cimag(val);
        }
      }
    }
  }
}

/* delta_eta(x) of the Gaussian reading */
double orc_delta(double x, double eta) { return exp(-(x * x) / (eta * eta)) / (sqrt(ORC_PI) * eta); }

static double fermi(double e, double mu, double kt) { return 1.0 / (exp((e - mu) / kt) + 1.0); }
static double bose(double w, double kt) { return 1.0 / (exp(w / kt) - 1.0); }

/* ---------------------------------------------------------------------
 * The vertex at one (k,q) for all (m, n, nu):
 *   gout[(m*nw + n)*nm + nu] = g_mn^nu(k,q)   (complex interleaved)
 * using full-grid tables evec (electrons) and u (phonons).  Gk is the Re
 * sum at this k, [nrp][nm][nw][nw] complex (computed by orc_re_sum).
 * -------------------------------------------------------------------*/
static void re_sum(const orc_model *md, int64_t N, const int64_t k[3], cplx *Gk) {
  const int nw = md->nw, nm = 3 * md->na;
  const size_t blk = (size_t)md->nrp * nm * nw * nw;
  for (size_t e = 0; e < blk; e++) Gk[e] = 0;
  for (int r = 0; r < md->nre; r++) {
    cplx ph = phase(k, md->re + 3 * r, N);
    const double *g = md->gw + (size_t)r * blk * 2;
    for (size_t e = 0; e < blk; e++) Gk[e] += ph * (g[2 * e] + I * g[2 * e + 1]);
  }
}

static void rp_sum(const orc_model *md, int64_t N, const int64_t q[3], const cplx *Gk, cplx *Gq) {
  const int nw = md->nw, nm = 3 * md->na;
  const size_t blk = (size_t)nm * nw * nw;
  for (size_t e = 0; e < blk; e++) Gq[e] = 0;
  for (int r = 0; r < md->nrp; r++) {
    cplx ph = phase(q, md->rp + 3 * r, N);
    const cplx *g = Gk + (size_t)r * blk;
    for (size_t e = 0; e < blk; e++) Gq[e] += ph * g[e];
  }
}

/* vertex for band pair (m,n), mode nu from Gq [nm][nw(i)][nw(j)] */
static cplx rotate(int nw, int nm, const cplx *Gq, const double *evp, const double *evk, const double *uq, int m,
                   int n, int nu) {
  cplx s = 0;
  for (int mu = 0; mu < nm; mu++) {
    cplx umn = uq[(nu * nm + mu) * 2] + I * uq[(nu * nm + mu) * 2 + 1];
    if (umn == 0) continue;
    cplx t = 0;
    for (int i = 0; i < nw; i++) {
      cplx vim = evp[(m * nw + i) * 2] - I * evp[(m * nw + i) * 2 + 1]; /* conj(V_im(k+q)) */
      cplx ti = 0;
      for (int j = 0; j < nw; j++) {
        cplx vjn = evk[(n * nw + j) * 2] + I * evk[(n * nw + j) * 2 + 1]; /* V_jn(k) */
        ti += Gq[(mu * nw + i) * nw + j] * vjn;
      }
      t += vim * ti;
    }
    s += t * umn;
  }
  return s;
}

void orc_vertex(const orc_model *md, int64_t N, int64_t kidx, int64_t qidx, const double *evec_k,
                const double *evec_p, const double *u_q, double *gout) {
  const int nw = md->nw, nm = 3 * md->na;
  int64_t k[3], q[3];
  grid_coords(kidx, N, k);
  grid_coords(qidx, N, q);
  cplx *Gk = malloc(sizeof(cplx) * (size_t)md->nrp * nm * nw * nw);
  cplx *Gq = malloc(sizeof(cplx) * (size_t)nm * nw * nw);
  re_sum(md, N, k, Gk);
  rp_sum(md, N, q, Gk, Gq);
  for (int m = 0; m < nw; m++)
    for (int n = 0; n < nw; n++)
      for (int nu = 0; nu < nm; nu++) {
        cplx g = rotate(nw, nm, Gq, evec_p, evec_k, u_q, m, n, nu);
        gout[((m * nw + n) * nm + nu) * 2] = creal(g);
        gout[((m * nw + n) * nm + nu) * 2 + 1] = cimag(g);
      }
  free(Gk);
  free(Gq);
}

/* ---------------------------------------------------------------------
 * SERTA scattering rates for a list of states (state_k[s], state_n[s]).
 * States must be sorted by k (states of one k are contiguous).
 * Tables cover the full N^3 grid: eps[N^3][nw], evec[N^3][nw][nw] c,
 * omega[N^3][nm], u[N^3][nm][nm] c.
 * Outputs: inv_tau[t][s] (1/s), nq_valid[s] = #q with a kept term,
 * nterms[s] = #(q,m,nu,sign) kept, nkq[0] = #(k,q) with a kept term for
 * any state at k.  sw = sieve width in units of eta.
 * -------------------------------------------------------------------*/
void orc_rates(const orc_model *md, int64_t N, const double *eps, const double *evec, const double *omega,
               const double *u, int64_t ns, const int32_t *state_k, const int32_t *state_n, double mu,
               int32_t nt, const double *temps, double eta, double sw, double omega_cut, double *inv_tau,
               int64_t *nq_valid, int64_t *nterms, int64_t *nkq) {
  const int nw = md->nw, nm = 3 * md->na;
  const int64_t NQ = N * N * N;
  const double pref = 2.0 * ORC_PI / orc_hbar_evs() / (double)NQ;
  const double kb = orc_kb_evk();
  /* group boundaries */
  int64_t ng = 0;
  int64_t *gs = malloc(sizeof(int64_t) * (ns + 1));
  for (int64_t s = 0; s < ns; s++)
    if (s == 0 || state_k[s] != state_k[s - 1]) gs[ng++] = s;
  gs[ng] = ns;
  int64_t total_kq = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total_kq)
  for (int64_t gi = 0; gi < ng; gi++) {
    const int64_t s0 = gs[gi], s1 = gs[gi + 1];
    const int64_t kidx = state_k[s0];
    int64_t k[3];
    grid_coords(kidx, N, k);
    cplx *Gk = malloc(sizeof(cplx) * (size_t)md->nrp * nm * nw * nw);
    cplx *Gq = malloc(sizeof(cplx) * (size_t)nm * nw * nw);
    re_sum(md, N, k, Gk);
    for (int64_t s = s0; s < s1; s++) {
      for (int t = 0; t < nt; t++) inv_tau[t * ns + s] = 0.0;
      nq_valid[s] = 0;
      nterms[s] = 0;
    }
    for (int64_t qi = 0; qi < NQ; qi++) {
      int64_t q[3], p[3];
      grid_coords(qi, N, q);
      for (int a = 0; a < 3; a++) p[a] = k[a] + q[a];
      const int64_t pidx = grid_index(p, N);
      const double *ep = eps + pidx * nw, *wq = omega + qi * nm;
      /* energy-conservation sieve over all states at this k */
      int any = 0;
      for (int64_t s = s0; s < s1 && !any; s++) {
        const double en = eps[kidx * nw + state_n[s]];
        for (int m = 0; m < nw && !any; m++)
          for (int nu = 0; nu < nm && !any; nu++) {
            if (wq[nu] < omega_cut) continue;
            for (int sg = -1; sg <= 1; sg += 2)
              if (fabs(en + sg * wq[nu] - ep[m]) <= sw * eta) any = 1;
          }
      }
      if (!any) continue;
      total_kq++;
      rp_sum(md, N, q, Gk, Gq);
      for (int64_t s = s0; s < s1; s++) {
        const int n = state_n[s];
        const double en = eps[kidx * nw + n];
        int hit = 0;
        for (int m = 0; m < nw; m++)
          for (int nu = 0; nu < nm; nu++) {
            if (wq[nu] < omega_cut) continue;
            double xp = en + wq[nu] - ep[m], xm = en - wq[nu] - ep[m];
            int kp = fabs(xp) <= sw * eta, km = fabs(xm) <= sw * eta;
            if (!kp && !km) continue;
            cplx g = rotate(nw, nm, Gq, evec + (size_t)pidx * nw * nw * 2, evec + (size_t)kidx * nw * nw * 2,
                            u + (size_t)qi * nm * nm * 2, m, n, nu);
            double g2 = creal(g) * creal(g) + cimag(g) * cimag(g);
            for (int t = 0; t < nt; t++) {
              double kt = kb * temps[t];
              double Nq = bose(wq[nu], kt), f = fermi(ep[m], mu, kt);
              double acc = 0.0;
              if (kp) acc += (Nq + f) * orc_delta(xp, eta);
              if (km) acc += (1.0 + Nq - f) * orc_delta(xm, eta);
              inv_tau[t * ns + s] += pref * g2 * acc;
            }
            nterms[s] += kp + km;
            hit = 1;
          }
        nq_valid[s] += hit;
      }
    }
    free(Gk);
    free(Gq);
  }
  free(gs);
  nkq[0] = total_kq;
}

/* ---------------------------------------------------------------------
 * Transition rates of the iterative solution (Sec. II.C, the iteration
 * equation; Sec. III.E stores their sum over modes and both phonon terms):
 * for a state s = (n,k) and a final state (m, p = k+q) with a kept term,
 *   Gamma_s(p,m)[t] = (2 pi/hbar)(1/N_q) sum_nu |g_mn^nu|^2
 *                     [(N_qnu + f_mp) delta(x+) + (1 + N_qnu - f_mp) delta(x-)],
 * the terms of 1/tau_s before they are summed over (q, m), so that
 * sum_{q,m} Gamma_s(q,m) = 1/tau_s.  Same sieve, vertex and factors as
 * orc_rates.  Entries are written state by state (rows in list order), q
 * ascending, then m ascending: row_start[s] .. row_start[s+1]-1 hold
 * fin[e] = p*nw + m and val[e*nt + t].  With fin == NULL only row_start is
 * filled (entry counts, then the prefix sum); the return value is the number
 * of entries.  States must be sorted by k.
 * -------------------------------------------------------------------*/
static int64_t gamma_state_terms(const orc_model *md, int64_t N, const double *eps, const double *omega,
                                 int64_t kidx, int n, double eta, double sw, double omega_cut) {
  /* number of (q, m) with at least one kept (nu, sign) term */
  const int nw = md->nw, nm = 3 * md->na;
  const int64_t NQ = N * N * N;
  int64_t k[3], q[3], p[3], cnt = 0;
  grid_coords(kidx, N, k);
  const double en = eps[kidx * nw + n];
  for (int64_t qi = 0; qi < NQ; qi++) {
    grid_coords(qi, N, q);
    for (int a = 0; a < 3; a++) p[a] = k[a] + q[a];
    const int64_t pidx = grid_index(p, N);
    for (int m = 0; m < nw; m++) {
      int kept = 0;
      for (int nu = 0; nu < nm && !kept; nu++) {
        const double w = omega[qi * nm + nu];
        if (w < omega_cut) continue;
        if (fabs(en + w - eps[pidx * nw + m]) <= sw * eta || fabs(en - w - eps[pidx * nw + m]) <= sw * eta) kept = 1;
      }
      cnt += kept;
    }
  }
  return cnt;
}

int64_t orc_gamma(const orc_model *md, int64_t N, const double *eps, const double *evec, const double *omega,
                  const double *u, int64_t ns, const int32_t *state_k, const int32_t *state_n, double mu, int32_t nt,
                  const double *temps, double eta, double sw, double omega_cut, int64_t *row_start, int64_t *fin,
                  double *val) {
  const int nw = md->nw, nm = 3 * md->na;
  const int64_t NQ = N * N * N;
  const double pref = 2.0 * ORC_PI / orc_hbar_evs() / (double)NQ;
  const double kb = orc_kb_evk();
  if (!fin) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < ns; s++)
      row_start[s + 1] = gamma_state_terms(md, N, eps, omega, state_k[s], state_n[s], eta, sw, omega_cut);
    row_start[0] = 0;
    for (int64_t s = 0; s < ns; s++) row_start[s + 1] += row_start[s];
    return row_start[ns];
  }
  int64_t ng = 0;
  int64_t *gs = malloc(sizeof(int64_t) * (ns + 1));
  for (int64_t s = 0; s < ns; s++)
    if (s == 0 || state_k[s] != state_k[s - 1]) gs[ng++] = s;
  gs[ng] = ns;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t gi = 0; gi < ng; gi++) {
    const int64_t s0 = gs[gi], s1 = gs[gi + 1];
    const int64_t kidx = state_k[s0];
    int64_t k[3];
    grid_coords(kidx, N, k);
    cplx *Gk = malloc(sizeof(cplx) * (size_t)md->nrp * nm * nw * nw);
    cplx *Gq = malloc(sizeof(cplx) * (size_t)nm * nw * nw);
    int64_t *cur = malloc(sizeof(int64_t) * (s1 - s0));
    for (int64_t s = s0; s < s1; s++) cur[s - s0] = row_start[s];
    re_sum(md, N, k, Gk);
    for (int64_t qi = 0; qi < NQ; qi++) {
      int64_t q[3], p[3];
      grid_coords(qi, N, q);
      for (int a = 0; a < 3; a++) p[a] = k[a] + q[a];
      const int64_t pidx = grid_index(p, N);
      const double *ep = eps + pidx * nw, *wq = omega + qi * nm;
      int gq_done = 0;
      for (int64_t s = s0; s < s1; s++) {
        const int n = state_n[s];
        const double en = eps[kidx * nw + n];
        for (int m = 0; m < nw; m++) {
          int any = 0;
          double acc[8] = {0};
          for (int nu = 0; nu < nm; nu++) {
            if (wq[nu] < omega_cut) continue;
            double xp = en + wq[nu] - ep[m], xm = en - wq[nu] - ep[m];
            int kp = fabs(xp) <= sw * eta, km = fabs(xm) <= sw * eta;
            if (!kp && !km) continue;
            if (!gq_done) {
              rp_sum(md, N, q, Gk, Gq);
              gq_done = 1;
            }
            any = 1;
            cplx g = rotate(nw, nm, Gq, evec + (size_t)pidx * nw * nw * 2, evec + (size_t)kidx * nw * nw * 2,
                            u + (size_t)qi * nm * nm * 2, m, n, nu);
            double g2 = creal(g) * creal(g) + cimag(g) * cimag(g);
            for (int t = 0; t < nt; t++) {
              double kt = kb * temps[t];
              double Nq = bose(wq[nu], kt), f = fermi(ep[m], mu, kt);
              double a = 0.0;
              if (kp) a += (Nq + f) * orc_delta(xp, eta);
              if (km) a += (1.0 + Nq - f) * orc_delta(xm, eta);
              acc[t] += pref * g2 * a;
            }
          }
          if (!any) continue;
          const int64_t e = cur[s - s0]++;
          fin[e] = pidx * nw + m;
          for (int t = 0; t < nt; t++) val[e * nt + t] = acc[t];
        }
      }
    }
    free(Gk);
    free(Gq);
    free(cur);
  }
  free(gs);
  return row_start[ns];
}

/* ---------------------------------------------------------------------
 * Iterative solution of the linearised BTE (Sec. II.C): with the mean free
 * paths F0_s = v_s tau_s,
 *   F^{i+1}_s = F0_s + tau_s sum_e Gamma_e F^i_{state(fin_e)},
 * where final states that are not in the state list carry F = 0.  States
 * with 1/tau = 0 are left out (F = 0).  sigma after every iteration (i = 0
 * is the SERTA value):
 *   sigma_ab = 2 e^2/(N_k V k_B T) sum_s v_a F_b f(1-f)
 * into sigma[(n_iter+1)][nt][9]; the final F into F[nt][ns][3].  Rows and
 * entries as written by orc_gamma (val[e*nt + t]).  Plain left-to-right sums.
 * -------------------------------------------------------------------*/
void orc_bte(int64_t N, int nw, int64_t ns, const int32_t *state_k, const int32_t *state_n, const double *energy,
             const double *vel, const double *inv_tau, const int64_t *row_start, const int64_t *fin,
             const double *val, double mu, int32_t nt, const double *temps, int64_t nk_total, double volume_a3,
             int32_t n_iter, double *sigma, double *F) {
  const int64_t NQ = N * N * N;
  const double kb = orc_kb_evk();
  const double vol = volume_a3 * 1e-30;
  int64_t *sidx = malloc(sizeof(int64_t) * NQ * nw);
  for (int64_t i = 0; i < NQ * nw; i++) sidx[i] = -1;
  for (int64_t s = 0; s < ns; s++) sidx[(int64_t)state_k[s] * nw + state_n[s]] = s;
  double *F0 = malloc(sizeof(double) * ns * 3), *Fo = malloc(sizeof(double) * ns * 3);
  for (int t = 0; t < nt; t++) {
    const double kt = kb * temps[t];
    for (int64_t s = 0; s < ns; s++) {
      const double it = inv_tau[t * ns + s];
      for (int a = 0; a < 3; a++) F0[s * 3 + a] = it == 0.0 ? 0.0 : vel[s * 3 + a] / it;
    }
    memcpy(Fo, F0, sizeof(double) * ns * 3);
    double *Fn = F + (size_t)t * ns * 3;
    for (int32_t i = 0; i <= n_iter; i++) {
      if (i > 0) {
        for (int64_t s = 0; s < ns; s++) {
          const double it = inv_tau[t * ns + s];
          double acc[3] = {0.0, 0.0, 0.0};
          if (it != 0.0)
            for (int64_t e = row_start[s]; e < row_start[s + 1]; e++) {
              const int64_t j = sidx[fin[e]];
              if (j < 0) continue;
              for (int a = 0; a < 3; a++) acc[a] += val[e * nt + t] * Fo[j * 3 + a];
            }
          for (int a = 0; a < 3; a++) Fn[s * 3 + a] = it == 0.0 ? 0.0 : F0[s * 3 + a] + acc[a] / it;
        }
        memcpy(Fo, Fn, sizeof(double) * ns * 3);
      } else {
        memcpy(Fn, F0, sizeof(double) * ns * 3);
      }
      double acc[9] = {0};
      for (int64_t s = 0; s < ns; s++) {
        if (inv_tau[t * ns + s] == 0.0) continue;
        const double f = fermi(energy[s], mu, kt);
        const double w = f * (1.0 - f) / kt;
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) acc[a * 3 + b] += vel[s * 3 + a] * Fo[s * 3 + b] * w;
      }
      for (int e = 0; e < 9; e++) sigma[((size_t)i * nt + t) * 9 + e] = 2.0 * ORC_E / ((double)nk_total * vol) * acc[e];
    }
  }
  free(sidx);
  free(F0);
  free(Fo);
}

/* ---------------------------------------------------------------------
 * Conductivity sigma[t][3][3] in S/m:
 *   sigma_ab(T) = 2 e^2/(N_k V) sum_s v_a v_b tau_s f(1-f)/(k_B T)
 * with V in m^3, v in m/s, tau = 1/inv_tau; states with inv_tau = 0 are
 * skipped.  Plain left-to-right summation over states.
 * -------------------------------------------------------------------*/
void orc_sigma(int64_t ns, const double *energy, const double *vel, const double *inv_tau, double mu,
               int32_t nt, const double *temps, int64_t nk_total, double volume_a3, double *sigma) {
  const double kb = orc_kb_evk();
  const double vol = volume_a3 * 1e-30;
  for (int t = 0; t < nt; t++) {
    double kt = kb * temps[t];
    double acc[9] = {0};
    for (int64_t s = 0; s < ns; s++) {
      double it = inv_tau[t * ns + s];
      if (it == 0.0) continue;
      double f = fermi(energy[s], mu, kt);
      double w = f * (1.0 - f) / kt / it; /* tau f(1-f)/kT in s/eV */
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) acc[a * 3 + b] += vel[s * 3 + a] * vel[s * 3 + b] * w;
    }
    /* e^2 * [1/eV -> 1/J] = e^2/(e) = e */
    for (int e = 0; e < 9; e++) sigma[t * 9 + e] = 2.0 * ORC_E / ((double)nk_total * vol) * acc[e];
  }
}

/* ---------------------------------------------------------------------
 * Transport coefficients from the same SERTA sums (Sec. II.C, the
 * coefficient definitions): with
 *   M_n,ab(T) = 2e/(N_k V) sum_s v_a v_b tau f(1-f)/(k_B T) (eps_s - mu)^n
 * (energies in eV, so M_0 = sigma in S/m),
 *   sigma = M_0,
 *   S     = -M_0^-1 M_1 / T                  (V/K, carriers of charge -e),
 *   kappa = (M_2 - M_1 M_0^-1 M_1) / T       (W/(m K), zero electric current).
 * Plain left-to-right sums; 3x3 inverse by cofactors.
 * -------------------------------------------------------------------*/
static void inv3(const double *a, double *r) {
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
static void mul3(const double *a, const double *b, double *r) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) r[i * 3 + j] = a[i * 3] * b[j] + a[i * 3 + 1] * b[3 + j] + a[i * 3 + 2] * b[6 + j];
}

void orc_transport(int64_t ns, const double *energy, const double *vel, const double *inv_tau, double mu,
                   int32_t nt, const double *temps, int64_t nk_total, double volume_a3, double *sigma,
                   double *seebeck, double *kappa) {
  const double kb = orc_kb_evk();
  const double vol = volume_a3 * 1e-30;
  for (int t = 0; t < nt; t++) {
    const double kt = kb * temps[t];
    double m[3][9] = {{0}};
    for (int64_t s = 0; s < ns; s++) {
      const double it = inv_tau[t * ns + s];
      if (it == 0.0) continue;
      const double f = fermi(energy[s], mu, kt), de = energy[s] - mu;
      const double w = f * (1.0 - f) / kt / it;
      for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) {
          const double x = vel[s * 3 + a] * vel[s * 3 + b] * w;
          m[0][a * 3 + b] += x;
          m[1][a * 3 + b] += x * de;
          m[2][a * 3 + b] += x * de * de;
        }
    }
    const double pref = 2.0 * ORC_E / ((double)nk_total * vol);
    for (int n = 0; n < 3; n++)
      for (int e = 0; e < 9; e++) m[n][e] *= pref;
    double i0[9], s1[9], k1[9];
    inv3(m[0], i0);
    mul3(i0, m[1], s1);
    mul3(m[1], s1, k1);
    for (int e = 0; e < 9; e++) {
      sigma[t * 9 + e] = m[0][e];
      seebeck[t * 9 + e] = -s1[e] / temps[t];
      kappa[t * 9 + e] = (m[2][e] - k1[e]) / temps[t];
    }
  }
}

/* carrier density n_c(T) = 2/(N_k V) sum_{band_lo<=n<=band_hi, all k} f(eps) in m^-3 */
void orc_carrier_density(int64_t nk, int nw, const double *eps, int band_lo, int band_hi, double mu, int32_t nt,
                         const double *temps, double volume_a3, double *nc) {
  const double kb = orc_kb_evk();
  for (int t = 0; t < nt; t++) {
    double kt = kb * temps[t], acc = 0.0;
    for (int64_t k = 0; k < nk; k++)
      for (int n = band_lo; n <= band_hi; n++) acc += fermi(eps[k * nw + n], mu, kt);
    nc[t] = 2.0 * acc / ((double)nk * volume_a3 * 1e-30);
  }
}

#ifdef _OPENMP
#include <omp.h>
#endif
/* threads an OpenMP region of the oracle uses */
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
