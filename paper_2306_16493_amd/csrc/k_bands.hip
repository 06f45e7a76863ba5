// Bloch sums and Hermitian eigensolves on the fine grid (gfx950).
//
// Electrons: H(k) = sum_R w_R e^{ik.R} H(R) and dH/dk_a = sum_R w_R i R_a
// e^{ik.R} H(R) (Sec. II.B, Wannier interpolation of H); eigenpairs
// H V = V diag(eps); velocities v_n = Re(V^+ dH V)_nn / hbar (Hellmann-Feynman
// form of the velocities of the preprocessing step, Sec. III.A).
// Phonons: D(q) = sum_R w_R Phi(R)/sqrt(M M') e^{iq.R}, (hbar w)^2 = C lambda,
// u_{mu nu} = e_{mu nu} sqrt(C/(2 M_mu hbar w_nu)) (Sec. II.B).
//
// Layout on the chip: one wave64 per workgroup; a matrix of padded size NP
// (1, 2, 4 or 8) occupies NP*NP lanes, one element (i,j) per lane, so a wave
// holds 64/(NP*NP) matrices.  Each lane accumulates its own element of the
// Bloch sum (and of the three derivatives) in registers; the eigensolve is a
// parallel cyclic Jacobi with round-robin pairing: every round applies
// NP/2 disjoint complex rotations at once, each lane updating its element of
// A and V from the (at most four) elements of the two rows/columns it mixes,
// staged in LDS.  Everything stays in FP64.
#include "dev_util.h"
#include "internal.h"

namespace eph {
namespace {

constexpr int kMaxSweeps = 40;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// Partner of index x in round r of the round-robin (circle) schedule of NP
// indices; NP-1 rounds cover every pair once.
template <int NP>
__device__ __forceinline__ int rr_partner(int x, int r) {
  if (NP == 1) return x;
  constexpr int M = NP - 1;
  int pos = (x == 0) ? 0 : ((x - 1 - r + 2 * M) % M) + 1;
  int ppos = NP - 1 - pos;
  return (ppos == 0) ? 0 : ((ppos - 1 + r) % M) + 1;
}

// element (row a, col b) of the block rotation J of this round.
struct Rot {
  double c;
  double2 se;  // s e^{i phi}
};

// Outputs of the eigensolve, shared by both Bloch-sum forms.
struct EigOut {
  int mode, n;
  const double *mode_mass;
  double cph, omega_cut, vel_unit;
  double *eval;
  double2 *evec;
  double *vel;
  unsigned long long *n_excluded;
};

// Parallel cyclic Jacobi on the matrices of one wave (element (i, j) of
// matrix mloc in each lane, acc its value, d0..d2 its k-derivatives), then
// eigenvalues sorted ascending, eigenvectors (or mode amplitudes) and
// velocities written for grid point kl.  The wave is the whole workgroup.
template <int NP>
__device__ __forceinline__ void eig_store(const EigOut &o, bool live, int64_t kl, double2 acc, double2 d0,
                                          double2 d1, double2 d2, double2 *sA, double2 *sV, Rot *sR, double *sW) {
  constexpr int L = NP * NP;
  const int mode = o.mode, n = o.n;
  const int lane = threadIdx.x;
  const int e = lane % L;
  const int i = e / NP, j = e % NP;
  const bool valid_ij = (i < n) && (j < n);
  const int base = (lane / L) * L;
    sA[lane] = valid_ij ? acc : make_double2(0.0, 0.0);
    sV[lane] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    __syncthreads();

    // ---- parallel cyclic Jacobi ----
    for (int sweep = 0; sweep < kMaxSweeps; sweep++) {
      double2 a = sA[lane];
      double a2 = valid_ij ? (a.x * a.x + a.y * a.y) : 0.0;
      double off = (i != j) ? a2 : 0.0, tot = a2;
#pragma unroll
      for (int m = 1; m < L; m <<= 1) {
        off += __shfl_xor(off, m, 64);
        tot += __shfl_xor(tot, m, 64);
      }
      bool done = (off == 0.0) || (off <= 1e-33 * tot) || !live;
      if (__all(done)) break;
      for (int r = 0; r < NP - 1; r++) {
        // rotation parameters: lane (p,q) with p<q, q = partner(p)
        if (valid_ij && i < j && rr_partner<NP>(i, r) == j) {
          double2 apq = sA[base + i * NP + j];
          double g = sqrt(apq.x * apq.x + apq.y * apq.y);
          Rot ro;
          if (g == 0.0) {
            ro.c = 1.0;
            ro.se = make_double2(0.0, 0.0);
          } else {
            double app = sA[base + i * NP + i].x, aqq = sA[base + j * NP + j].x;
            double theta = (aqq - app) / (2.0 * g);
            double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
            ro.c = c;
            ro.se = make_double2(s * apq.x / g, s * apq.y / g);
          }
          sR[base + i] = ro;  // indexed by the smaller index of the pair
        }
        __syncthreads();
        // J entries: J_pp = c, J_pq = s e, J_qp = -s conj(e), J_qq = c (p<q)
        const int pi = rr_partner<NP>(i, r), pj = rr_partner<NP>(j, r);
        const bool roti = (i < n) && (pi < n) && (pi != i);
        const bool rotj = (j < n) && (pj < n) && (pj != j);
        // column factors J_{b j} for b in {j, pj}
        double2 Jjj = make_double2(1.0, 0.0), Jpj = make_double2(0.0, 0.0);
        if (rotj) {
          Rot ro = sR[base + min(j, pj)];
          Jjj = make_double2(ro.c, 0.0);
          if (j > pj) Jpj = ro.se;                                  // J_{p q} with p=pj<q=j
          else Jpj = make_double2(-ro.se.x, ro.se.y);               // J_{q p} = -conj(se)
        }
        double2 Jii = make_double2(1.0, 0.0), Jpi = make_double2(0.0, 0.0);
        if (roti) {
          Rot ro = sR[base + min(i, pi)];
          Jii = make_double2(ro.c, 0.0);
          if (i > pi) Jpi = ro.se;
          else Jpi = make_double2(-ro.se.x, ro.se.y);
        }
        double2 nA = make_double2(0.0, 0.0), nV = make_double2(0.0, 0.0);
        if (valid_ij) {
          // (J^H A J)_ij = sum_{a in {i,pi}} sum_{b in {j,pj}} conj(J_ai) A_ab J_bj
          double2 Aij = sA[base + i * NP + j];
          double2 col_i = cmul(Aij, Jjj);
          if (rotj) col_i = cadd(col_i, cmul(sA[base + i * NP + pj], Jpj));
          nA = cmul(cconj(Jii), col_i);
          if (roti) {
            double2 col_p = cmul(sA[base + pi * NP + j], Jjj);
            if (rotj) col_p = cadd(col_p, cmul(sA[base + pi * NP + pj], Jpj));
            nA = cadd(nA, cmul(cconj(Jpi), col_p));
          }
          nV = cmul(sV[base + i * NP + j], Jjj);
          if (rotj) nV = cadd(nV, cmul(sV[base + i * NP + pj], Jpj));
          if (i != j && pi == j && roti) nA = make_double2(0.0, 0.0);  // annihilated pair
          if (i == j) nA.y = 0.0;
        } else {
          nV = sV[lane];
        }
        __syncthreads();
        sA[lane] = nA;
        sV[lane] = nV;
        __syncthreads();
      }
    }

    // ---- sort eigenvalues ascending; lane (i,j) carries column j ----
    if (lane < 64 && i == 0) sW[base + j] = (j < n) ? sA[base + j * NP + j].x : 0.0;
    __syncthreads();
    int rank = 0;
    double wj = sW[base + j];
    for (int jj = 0; jj < n; jj++) {
      double wo = sW[base + jj];
      rank += (wo < wj) || (wo == wj && jj < j);
    }
    if (live && valid_ij) {
      const int64_t kk = kl;
      double2 v = sV[base + i * NP + j];
      if (mode == 0) {
        if (i == 0) o.eval[kk * n + rank] = wj;
        o.evec[(kk * n + rank) * n + i] = v;
      } else {
        double hw = sqrt(o.cph * fmax(wj, 0.0));
        if (i == 0) {
          o.eval[kk * n + rank] = hw;
          if (hw < o.omega_cut) atomicAdd(o.n_excluded, 1ull);
        }
        double2 u = make_double2(0.0, 0.0);
        if (hw >= o.omega_cut) {
          double f = sqrt(o.cph / (2.0 * o.mode_mass[i] * hw));
          u = make_double2(v.x * f, v.y * f);
        }
        o.evec[(kk * n + rank) * n + i] = u;  // evec[q][nu][mu] = u_{mu nu}
      }
    }
    if (mode == 0) {
      // velocities: v_col = Re sum_ij conj(V_i,col) dH_ij V_j,col, butterfly over the matrix lanes
      for (int col = 0; col < n; col++) {
        double c0 = 0.0, c1 = 0.0, c2 = 0.0;
        if (valid_ij) {
          double2 vi = sV[base + i * NP + col], vj = sV[base + j * NP + col];
          double2 pr = cmul(cconj(vi), vj);  // conj(V_i) V_j
          c0 = pr.x * d0.x - pr.y * d0.y;
          c1 = pr.x * d1.x - pr.y * d1.y;
          c2 = pr.x * d2.x - pr.y * d2.y;
        }
#pragma unroll
        for (int m = 1; m < L; m <<= 1) {
          c0 += __shfl_xor(c0, m, 64);
          c1 += __shfl_xor(c1, m, 64);
          c2 += __shfl_xor(c2, m, 64);
        }
        int rk = 0;
        double wc = sW[base + col];
        for (int jj = 0; jj < n; jj++) {
          double wo = sW[base + jj];
          rk += (wo < wc) || (wo == wc && jj < col);
        }
        if (live && e == 0) {
          double *vo = o.vel + (kl * n + rk) * 3;
          vo[0] = c0 * o.vel_unit;
          vo[1] = c1 * o.vel_unit;
          vo[2] = c2 * o.vel_unit;
        }
      }
    }
  __syncthreads();
}

template <int NP>
__global__ __launch_bounds__(64) void bloch_eig_kernel(EigOut o, int N, int64_t k0, int64_t nk, int nr,
                                                       const int *__restrict__ R, const double *__restrict__ w,
                                                       const double *__restrict__ Rcart,
                                                       const double2 *__restrict__ M,
                                                       const double2 *__restrict__ tab) {
  constexpr int L = NP * NP;
  constexpr int MPW = 64 / L;
  __shared__ double2 sA[64];
  __shared__ double2 sV[64];
  __shared__ Rot sR[64];
  __shared__ double sW[64];
  const int mode = o.mode, n = o.n;
  const int lane = threadIdx.x;
  const int mloc = lane / L;
  const int e = lane % L;
  const int i = e / NP, j = e % NP;
  const bool valid_ij = (i < n) && (j < n);

  const int64_t ngroups = (nk + MPW - 1) / MPW;
  for (int64_t gidx = blockIdx.x; gidx < ngroups; gidx += gridDim.x) {
    const int64_t kl = gidx * MPW + mloc;
    const bool live = kl < nk;
    const int64_t kg = k0 + (live ? kl : 0);
    const int64_t k1 = kg % N, k2 = (kg / N) % N, k3 = kg / ((int64_t)N * N);

    // ---- Bloch sum (and derivatives for electrons), direct over the R list ----
    double2 acc = make_double2(0.0, 0.0);
    double2 d0 = acc, d1 = acc, d2 = acc;
    if (valid_ij) {
      for (int r = 0; r < nr; r++) {
        int64_t s = (k1 * R[3 * r] + k2 * R[3 * r + 1] + k3 * R[3 * r + 2]) % N;
        if (s < 0) s += N;
        double2 ph = tab[s];
        double wr = w[r];
        ph.x *= wr;
        ph.y *= wr;
        double2 t = cmul(ph, M[(size_t)r * n * n + i * n + j]);
        acc = cadd(acc, t);
        if (mode == 0) {
          // i * R_a * t
          double2 it = make_double2(-t.y, t.x);
          double r0 = Rcart[3 * r], r1 = Rcart[3 * r + 1], r2 = Rcart[3 * r + 2];
          d0.x += r0 * it.x; d0.y += r0 * it.y;
          d1.x += r1 * it.x; d1.y += r1 * it.y;
          d2.x += r2 * it.x; d2.y += r2 * it.y;
        }
      }
    }
    eig_store<NP>(o, live, kl, acc, d0, d1, d2, sA, sV, sR, sW);
  }
}

// Separable form of the same Bloch sum for R lists that fill a box
// [lo, lo + nb) (missing vectors are zero in the dense copy Mb, weights
// folded in).  One wave per k-line (k2, k3): every lane first sums its
// element over the (R2, R3) planes for each R1,
//   T0(R1) = sum_{R2,R3} e^{i2pi(k2 R2 + k3 R3)/N} M(R),  T2, T3 the same
//   weighted by R2, R3 (electrons),
// in registers, then per k1 on the line
//   M(k) = sum_R1 e^{i2pi k1 R1/N} T0(R1),  S1 = sum_R1 R1 e^{..} T0(R1),
//   S2, S3 = sum_R1 e^{..} T2,3(R1),  dM/dk_a = i sum_b L_ba S_b
// (L the lattice vectors as rows), which is the direct sum associated
// differently.  NR1 bounds the box length along R1.
struct BoxArgs {
  int lo[3], nb[3];
  double lat[9];
};

template <int NP, int NR1, int MODE>
__global__ __launch_bounds__(64) void bloch_line_kernel(EigOut o, int N, BoxArgs bx, const double2 *__restrict__ Mb,
                                                        const double2 *__restrict__ tab) {
  constexpr int NRD = MODE == 0 ? NR1 : 1;  // derivative planes only for electrons
  constexpr int L = NP * NP;
  constexpr int MPW = 64 / L;
  __shared__ double2 sA[64];
  __shared__ double2 sV[64];
  __shared__ Rot sR[64];
  __shared__ double sW[64];
  constexpr int mode = MODE;
  const int n = o.n;
  const int lane = threadIdx.x;
  const int mloc = lane / L;
  const int e = lane % L;
  const int i = e / NP, j = e % NP;
  const bool valid_ij = (i < n) && (j < n);
  const int n1 = bx.nb[0], n2 = bx.nb[1], n3 = bx.nb[2];
  const size_t nn = (size_t)n * n;
  const int64_t nlines = (int64_t)N * N;
  for (int64_t line = blockIdx.x; line < nlines; line += gridDim.x) {
    const int k2 = (int)(line % N), k3 = (int)(line / N);
    double2 T0[NR1], T2[NRD], T3[NRD];
#pragma unroll
    for (int b = 0; b < NR1; b++) T0[b] = make_double2(0.0, 0.0);
#pragma unroll
    for (int b = 0; b < NRD; b++) T2[b] = T3[b] = make_double2(0.0, 0.0);
    if (valid_ij) {
      int i2 = imod(k2 * bx.lo[1], N);
      const int i3s = imod(k3 * bx.lo[2], N);
      for (int b2 = 0; b2 < n2; b2++) {
        const double r2 = (double)(bx.lo[1] + b2);
        int i23 = i2 + i3s;
        i23 -= (i23 >= N) ? N : 0;
        for (int b3 = 0; b3 < n3; b3++) {
          const double2 ph = tab[i23];
          const double r3 = (double)(bx.lo[2] + b3);
          const double2 *m = Mb + ((size_t)b2 * n3 + b3) * nn + i * n + j;
#pragma unroll
          for (int b1 = 0; b1 < NR1; b1++) {
            if (b1 < n1) {
              const double2 t = cmul(ph, m[(size_t)b1 * n2 * n3 * nn]);
              T0[b1] = cadd(T0[b1], t);
              if constexpr (MODE == 0) {
                T2[b1].x = fma(r2, t.x, T2[b1].x);
                T2[b1].y = fma(r2, t.y, T2[b1].y);
                T3[b1].x = fma(r3, t.x, T3[b1].x);
                T3[b1].y = fma(r3, t.y, T3[b1].y);
              }
            }
          }
          i23 += k3;
          i23 -= (i23 >= N) ? N : 0;
        }
        i2 += k2;
        i2 -= (i2 >= N) ? N : 0;
      }
    }
    for (int kb = 0; kb < N; kb += MPW) {
      const int k1r = kb + mloc;
      const bool live = k1r < N;
      const int k1 = live ? k1r : 0;
      double2 acc = make_double2(0.0, 0.0), s1 = acc, s2 = acc, s3 = acc;
      if (valid_ij) {
        int i1 = imod(k1 * bx.lo[0], N);
#pragma unroll
        for (int b1 = 0; b1 < NR1; b1++) {
          if (b1 < n1) {
            const double2 ph = tab[i1];
            const double2 t = cmul(ph, T0[b1]);
            acc = cadd(acc, t);
            if constexpr (MODE == 0) {
              const double r1 = (double)(bx.lo[0] + b1);
              s1.x = fma(r1, t.x, s1.x);
              s1.y = fma(r1, t.y, s1.y);
              s2 = cadd(s2, cmul(ph, T2[b1]));
              s3 = cadd(s3, cmul(ph, T3[b1]));
            }
            i1 += k1;
            i1 -= (i1 >= N) ? N : 0;
          }
        }
      }
      double2 d[3];
#pragma unroll
      for (int a = 0; a < 3; a++) {
        // i * sum_b L_ba S_b
        const double re = bx.lat[a] * s1.x + bx.lat[3 + a] * s2.x + bx.lat[6 + a] * s3.x;
        const double im = bx.lat[a] * s1.y + bx.lat[3 + a] * s2.y + bx.lat[6 + a] * s3.y;
        d[a] = make_double2(-im, re);
      }
      const int64_t kl = (int64_t)k1 + (int64_t)N * line;
      eig_store<NP>(o, live, kl, acc, d[0], d[1], d[2], sA, sV, sR, sW);
    }
  }
}

__global__ void phase_table_kernel(int N, double2 *tab) {
  int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < N) {
    double s, c;
    sincospi(2.0 * (double)m / (double)N, &s, &c);
    tab[m] = make_double2(c, s);
  }
}

}  // namespace

hipError_t launch_phase_table(int N, double2 *tab, hipStream_t st) {
  hipLaunchKernelGGL(phase_table_kernel, dim3((N + 255) / 256), dim3(256), 0, st, N, tab);
  return hipGetLastError();
}

hipError_t launch_bloch_eig(int mode, int n, int N, int64_t k0, int64_t nk, int nr, const int *R,
                            const double *w, const double *Rcart, const double2 *M, const double2 *tab,
                            const double *mode_mass, double cph, double omega_cut, double vel_unit,
                            double *eval, double2 *evec, double *vel, unsigned long long *n_excluded,
                            hipStream_t st) {
  if (nk <= 0) return hipSuccess;
  const EigOut o{mode, n, mode_mass, cph, omega_cut, vel_unit, eval, evec, vel, n_excluded};
  int NP = n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : 8;
  int mpw = 64 / (NP * NP);
  int64_t ngroups = (nk + mpw - 1) / mpw;
  int grid = (int)(ngroups < 262144 ? ngroups : 262144);
#define EPH_LAUNCH_BE(NPV) \
  hipLaunchKernelGGL(bloch_eig_kernel<NPV>, dim3(grid), dim3(64), 0, st, o, N, k0, nk, nr, R, w, Rcart, M, tab)
  switch (NP) {
    case 1: EPH_LAUNCH_BE(1); break;
    case 2: EPH_LAUNCH_BE(2); break;
    case 4: EPH_LAUNCH_BE(4); break;
    default: EPH_LAUNCH_BE(8); break;
  }
#undef EPH_LAUNCH_BE
  return hipGetLastError();
}

hipError_t launch_bloch_lines(int mode, int n, int N, const int *lo, const int *nb, const double *lattice,
                              const double2 *Mb, const double2 *tab, const double *mode_mass, double cph,
                              double omega_cut, double vel_unit, double *eval, double2 *evec, double *vel,
                              unsigned long long *n_excluded, hipStream_t st) {
  const EigOut o{mode, n, mode_mass, cph, omega_cut, vel_unit, eval, evec, vel, n_excluded};
  if (nb[0] > kBoxMaxR1) return hipErrorInvalidValue;
  BoxArgs bx;
  for (int a = 0; a < 3; a++) {
    bx.lo[a] = lo[a];
    bx.nb[a] = nb[a];
  }
  for (int a = 0; a < 9; a++) bx.lat[a] = lattice[a];
  const int NP = n <= 1 ? 1 : n <= 2 ? 2 : n <= 4 ? 4 : 8;
  const int64_t nlines = (int64_t)N * N;
  const int grid = (int)(nlines < 262144 ? nlines : 262144);
#define EPH_LAUNCH_BL(NPV, R1)                                                                               \
  if (mode == 0) hipLaunchKernelGGL((bloch_line_kernel<NPV, R1, 0>), dim3(grid), dim3(64), 0, st, o, N, bx, Mb, tab); \
  else hipLaunchKernelGGL((bloch_line_kernel<NPV, R1, 1>), dim3(grid), dim3(64), 0, st, o, N, bx, Mb, tab);       \
  return hipGetLastError();
#define EPH_LAUNCH_NP(R1)        \
  switch (NP) {                  \
    case 1: EPH_LAUNCH_BL(1, R1) \
    case 2: EPH_LAUNCH_BL(2, R1) \
    case 4: EPH_LAUNCH_BL(4, R1) \
    default: EPH_LAUNCH_BL(8, R1) \
  }
  if (nb[0] <= 7) EPH_LAUNCH_NP(7)
  if (nb[0] <= 9) EPH_LAUNCH_NP(9)
  EPH_LAUNCH_NP(kBoxMaxR1)
#undef EPH_LAUNCH_NP
#undef EPH_LAUNCH_BL
}

}  // namespace eph
