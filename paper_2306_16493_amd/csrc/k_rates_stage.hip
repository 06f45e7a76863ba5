// SERTA scattering rates, staged q-line form (gfx950).
//
// Arithmetic as in the other rate kernels (separable Rp box: Y per q3, Z per
// q-line, G per q; vertex contracted onto a final band m, then onto the
// modes; energy-conservation sieve, occupations, Gaussian delta; Sec. II.B,
// II.C, III.A, III.C).  Organisation:
//   * a 512-thread workgroup owns up to SG initial states of one k-line and
//     walks the q-lines (q2, q3) in lockstep;
//   * Y_s(p1, p2; q3) of all its states lives in registers, NSLOT
//     (state, p1, channel) slots per thread; Z_s(p1; q2, q3) goes to LDS;
//   * every q needs the q-side record (hbar w, Bose factors, u) and every
//     final state p = k + q the p-side record (energy, Fermi factors, V row);
//     both come from packed per-call tables in which one q-line (resp. one
//     final-state line) is a contiguous chunk.  The next line's two chunks
//     are loaded into registers while the current line is processed and then
//     written to LDS, so the candidates never wait on global memory;
//   * candidates (state, p1, final-band mask) are compacted state-major with
//     ballots and a prefix over the per-state counts; per-candidate partial
//     rates are summed per state in index order, so results are
//     bit-reproducible.
#include "dev_util.h"
#include "internal.h"

namespace eph {
namespace {

constexpr int kThreads = 512;
constexpr int kRound = 1024;  // candidates per round (2 per thread)
constexpr int kStageSG = 21;  // states per group: 3 Y slots per thread

// Record layouts (in doubles); complex members start on 16-byte boundaries.
__host__ __device__ inline int qoff_u(int nm, int nt) { return (nm + nm * nt + 1) & ~1; }
__host__ __device__ inline int qrec(int nm, int nt) { return qoff_u(nm, nt) + 2 * nm * nm; }
__host__ __device__ inline int poff_v(int nt) { return (1 + nt + 1) & ~1; }
__host__ __device__ inline int prec(int nw, int nt) { return poff_v(nt) + 2 * nw; }

template <int NW, int NM, int NB, int SG>
struct StageLayout {
  static constexpr int C = NW * NM;
  static constexpr int SMX = SG + NW;  // members + shadows
  size_t tab, z, qt, pt, cand, contrib, acc, mask, misc, total;
  __host__ __device__ StageLayout(int N, int nt) {
    size_t o = 0;
    tab = o; o = align16(o + 16 * (size_t)N);
    z = o; o = align16(o + 16 * (size_t)SG * NB * C);
    qt = o; o = align16(o + 8 * (size_t)N * qrec(NM, nt));
    pt = o; o = align16(o + 8 * (size_t)N * NW * prec(NW, nt));
    cand = o; o = align16(o + 4 * (size_t)SMX * N);
    contrib = o; o = align16(o + 8 * (size_t)kRound * nt);
    acc = o; o = align16(o + 8 * (size_t)SG * nt);
    mask = o; o = align16(o + 8 * (size_t)SMX * ((N + 63) / 64));
    misc = o; o = align16(o + 4 * (3 * SMX + 2) + 8 * SMX + 64);
    total = o;
  }
};

template <int NW, int NM, int NB, int SG, int NSLOT, int LPF>
__global__ __launch_bounds__(kThreads) void rates_stage_kernel(RatesArgs a, const double *__restrict__ qtab,
                                                              const double *__restrict__ ptab) {
  constexpr int C = NW * NM;
  constexpr int SMX = SG + NW;
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = a.N, nt = a.nt;
  const int QR = qrec(NM, nt), PR = prec(NW, nt);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int MW = (N + 63) >> 6;
  const StageLayout<NW, NM, NB, SG> L(N, nt);
  double2 *sTab = reinterpret_cast<double2 *>(smem + L.tab);
  double2 *sZ = reinterpret_cast<double2 *>(smem + L.z);
  double *sQT = reinterpret_cast<double *>(smem + L.qt);
  double *sPT = reinterpret_cast<double *>(smem + L.pt);
  uint32_t *sCand = reinterpret_cast<uint32_t *>(smem + L.cand);
  double *sContrib = reinterpret_cast<double *>(smem + L.contrib);
  double *sAcc = reinterpret_cast<double *>(smem + L.acc);
  unsigned long long *sMask = reinterpret_cast<unsigned long long *>(smem + L.mask);
  int *sCnt = reinterpret_cast<int *>(smem + L.misc);
  int *sK1 = sCnt + SMX;
  int *sTerms = sK1 + SMX;
  unsigned long long *sCtr = reinterpret_cast<unsigned long long *>(sTerms + SMX + 2 - (SMX & 1));
  double *sEps = reinterpret_cast<double *>(sCtr + 2 + (SMX > 0 ? 0 : 0));

  // XCD-aware group order
  const int64_t per_xcd = (a.ng + 7) / 8;
  const int64_t g = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (g >= a.ng) return;  // uniform over the workgroup
  const int64_t s0 = a.gstart[g];
  const int S = (int)(a.gstart[g + 1] - s0);
  const int64_t kfirst = a.sk[s0];
  int SH = 0;
  {
    const int64_t klast = a.sk[s0 + S - 1];
    while (SH < NW - 1 && s0 + S + SH < a.ns_total && a.sk[s0 + S + SH] == klast) SH++;
  }
  const int ST = S + SH;
  const bool cont = (s0 > 0) && (a.sk[s0 - 1] == kfirst);
  const int k2 = (int)((kfirst / N) % N), k3 = (int)(kfirst / ((int64_t)N * N));
  const double W = a.wmax + a.sw * a.eta;
  const double cut = a.sw * a.eta;
  const double inv_eta = 1.0 / a.eta;
  const double dnorm = 1.0 / (1.7724538509055160273 * a.eta);
  const int lo1 = a.box.lo[0], lo2 = a.box.lo[1], lo3 = a.box.lo[2];

  for (int t = tid; t < N; t += kThreads) sTab[t] = a.tab[t];
  if (tid < SMX) {
    if (tid < ST) {
      const int64_t k = a.sk[s0 + tid];
      sK1[tid] = (int)(k % N);
      sEps[tid] = a.eps[k * NW + a.sn[s0 + tid]];
    } else {
      sK1[tid] = 0;
      sEps[tid] = 0.0;
    }
    sTerms[tid] = 0;
  }
  if (tid < 2) sCtr[tid] = 0ull;
  for (int t = tid; t < SG * nt; t += kThreads) sAcc[t] = 0.0;
  for (int t = tid; t < SMX * MW; t += kThreads) sMask[t] = 0ull;
  // staged tables of the first q-line (q2 = q3 = 0)
  {
    const double *qs = qtab + (size_t)0 * N * QR;
    const double *ps = ptab + (size_t)(k2 + N * k3) * N * NW * PR;
    for (int t = tid; t < N * QR; t += kThreads) sQT[t] = qs[t];
    for (int t = tid; t < N * NW * PR; t += kThreads) sPT[t] = ps[t];
  }
  unsigned long long my_nq = 0, my_nt = 0, my_nkq = 0, my_nv = 0;

  double yr[NSLOT][NB], yi[NSLOT][NB];
  const double2 *Xg = reinterpret_cast<const double2 *>(a.X);
  const int64_t xrow = (int64_t)NB * NB * NB * C;
  const int nq_chunk = N * QR, np_chunk = N * NW * PR;
  const int qsl = (nq_chunk + kThreads - 1) / kThreads;
  double pf[LPF];

  for (int q3 = 0; q3 < N; q3++) {
    __syncthreads();
    // ---- Y_s(p1, p2; q3) into registers ----
#pragma unroll
    for (int j = 0; j < NSLOT; j++)
#pragma unroll
      for (int p2 = 0; p2 < NB; p2++) yr[j][p2] = yi[j][p2] = 0.0;
    {
      int i3 = imod(q3 * lo3, N);
#pragma unroll 1
      for (int p3 = 0; p3 < NB; p3++) {
        const double2 ph = sTab[i3];
        i3 += q3;
        i3 -= (i3 >= N) ? N : 0;
#pragma unroll
        for (int j = 0; j < NSLOT; j++) {
          const int P = tid + kThreads * j;
          const int s = P / (NB * C), p1 = (P / C) % NB, c = P % C;
          if (s < S) {
            const double2 *xs = Xg + (s0 + s - a.s_base) * xrow + (int64_t)p1 * NB * NB * C + p3 * C + c;
#pragma unroll
            for (int p2 = 0; p2 < NB; p2++) {
              const double2 x = xs[p2 * NB * C];
              yr[j][p2] += ph.x * x.x - ph.y * x.y;
              yi[j][p2] += ph.x * x.y + ph.y * x.x;
            }
          }
        }
      }
    }
    const int p3line = (k3 + q3 >= N) ? k3 + q3 - N : k3 + q3;
    for (int q2 = 0; q2 < N; q2++) {
      // ---- prefetch the next q-line's staged tables into registers ----
      {
        int nq2 = q2 + 1, nq3 = q3;
        if (nq2 == N) {
          nq2 = 0;
          nq3 = (q3 + 1 == N) ? 0 : q3 + 1;
        }
        const int n2l = (k2 + nq2 >= N) ? k2 + nq2 - N : k2 + nq2;
        const int n3l = (k3 + nq3 >= N) ? k3 + nq3 - N : k3 + nq3;
        const double *qs = qtab + (size_t)(nq2 + N * nq3) * nq_chunk;
        const double *ps = ptab + (size_t)(n2l + N * n3l) * np_chunk;
        // slots [0, qsl) carry the q-side chunk, [qsl, LPF) the p-side chunk
#pragma unroll
        for (int i = 0; i < LPF; i++) {
          if (i < qsl) {
            const int e = tid + kThreads * i;
            pf[i] = (e < nq_chunk) ? qs[e] : 0.0;
          } else {
            const int e = tid + kThreads * (i - qsl);
            pf[i] = (e < np_chunk) ? ps[e] : 0.0;
          }
        }
      }
      // ---- Z_s(p1; q2, q3) -> LDS ----
      {
        double2 ph2[NB];
        int i2 = imod(q2 * lo2, N);
#pragma unroll
        for (int p = 0; p < NB; p++) {
          ph2[p] = sTab[i2];
          i2 += q2;
          i2 -= (i2 >= N) ? N : 0;
        }
#pragma unroll
        for (int j = 0; j < NSLOT; j++) {
          const int P = tid + kThreads * j;
          if (P < SG * NB * C) {
            double r = 0, i = 0;
#pragma unroll
            for (int p2 = 0; p2 < NB; p2++) {
              r += ph2[p2].x * yr[j][p2] - ph2[p2].y * yi[j][p2];
              i += ph2[p2].x * yi[j][p2] + ph2[p2].y * yr[j][p2];
            }
            sZ[P] = make_double2(r, i);
          }
        }
      }
      const int p2line = (k2 + q2 >= N) ? k2 + q2 - N : k2 + q2;
      const int line = p2line + N * p3line;
      // ---- candidate counts per state (wave w: states w, w+8, ...) ----
      for (int s = wave; s < ST; s += 8) {
        int cnt = 0;
        const double es = sEps[s];
        for (int c0 = 0; c0 < N; c0 += 64) {
          const int p1 = c0 + lane;
          bool any = false;
          if (p1 < N) {
#pragma unroll
            for (int m = 0; m < NW; m++) any |= fabs(sPT[(p1 * NW + m) * PR] - es) <= W;
          }
          cnt += __popcll(__ballot(any));
        }
        if (lane == 0) sCnt[s] = cnt;
      }
      __syncthreads();
      int pre_me = 0, total = 0;
      // prefix over states (every thread)
      for (int s = 0; s < ST; s++) total += sCnt[s];
      for (int s = wave; s < ST; s += 8) {
        int base = 0;
        for (int s2 = 0; s2 < s; s2++) base += sCnt[s2];
        const double es = sEps[s];
        for (int c0 = 0; c0 < N; c0 += 64) {
          const int p1 = c0 + lane;
          unsigned mm = 0;
          if (p1 < N) {
#pragma unroll
            for (int m = 0; m < NW; m++) mm |= (fabs(sPT[(p1 * NW + m) * PR] - es) <= W) ? (1u << m) : 0u;
          }
          const unsigned long long bits = __ballot(mm != 0);
          if (mm) {
            const int pos = base + __popcll(bits & ((1ull << lane) - 1ull));
            sCand[pos] = (uint32_t)p1 | (mm << 10) | ((uint32_t)s << 18);
          }
          base += __popcll(bits);
        }
      }
      (void)pre_me;
      __syncthreads();
      // ---- rounds of candidates ----
      for (int r0 = 0; r0 < total; r0 += kRound) {
        for (int ii = 0; ii < kRound / kThreads; ii++) {
          const int li = tid + kThreads * ii;
          const int i = r0 + li;
          double contrib[EPH_MAX_TEMPS] = {0.0, 0.0, 0.0, 0.0};
          if (i < total) {
            const uint32_t d = sCand[i];
            const int p1 = (int)(d & 1023u), s = (int)(d >> 18);
            unsigned mm = (d >> 10) & 255u;
            int q1 = p1 - sK1[s];
            q1 += (q1 < 0) ? N : 0;
            const double es = sEps[s];
            const double *qr = sQT + (size_t)q1 * QR;  // [om NM][occ_n NM*nt][u NM*NM complex]
            double om[NM];
#pragma unroll
            for (int nu = 0; nu < NM; nu++) om[nu] = qr[nu];
            bool hit = false;
            int nterm = 0;
            while (mm) {
              const int m = __ffs(mm) - 1;
              mm &= mm - 1;
              const double *pr = sPT + (size_t)(p1 * NW + m) * PR;  // [eps][occ_f nt][V row NW complex]
              const double ep = pr[0];
              unsigned vp = 0, vm = 0;
#pragma unroll
              for (int nu = 0; nu < NM; nu++) {
                const bool okw = om[nu] >= a.wcut;
                vp |= (okw && fabs(es + om[nu] - ep) <= cut) ? (1u << nu) : 0u;
                vm |= (okw && fabs(es - om[nu] - ep) <= cut) ? (1u << nu) : 0u;
              }
              if ((vp | vm) == 0u) continue;
              hit = true;
              if (s >= S) continue;  // shadow state: counted only
              my_nv++;
              // W_mu = sum_p1' e^{i 2pi q1 p1'/N} sum_i conj(V_im(p)) Z_s(p1'; mu, i)
              const double2 *vr = reinterpret_cast<const double2 *>(pr + poff_v(nt));
              double2 vrow[NW];
#pragma unroll
              for (int i2 = 0; i2 < NW; i2++) vrow[i2] = vr[i2];
              double wr[NM], wi[NM];
#pragma unroll
              for (int mu = 0; mu < NM; mu++) wr[mu] = wi[mu] = 0.0;
              int i1 = imod(q1 * lo1, N);
              const double2 *zs = sZ + s * NB * C;
#pragma unroll 1
              for (int pp = 0; pp < NB; pp++) {
                const double2 ph = sTab[i1];
                i1 += q1;
                i1 -= (i1 >= N) ? N : 0;
#pragma unroll
                for (int mu = 0; mu < NM; mu++) {
                  double tr = 0, ti = 0;
#pragma unroll
                  for (int i2 = 0; i2 < NW; i2++) {
                    const double2 z = zs[pp * C + mu * NW + i2];
                    tr += vrow[i2].x * z.x + vrow[i2].y * z.y;
                    ti += vrow[i2].x * z.y - vrow[i2].y * z.x;
                  }
                  wr[mu] += ph.x * tr - ph.y * ti;
                  wi[mu] += ph.x * ti + ph.y * tr;
                }
              }
              const double2 *ur = reinterpret_cast<const double2 *>(qr + qoff_u(NM, nt));
#pragma unroll
              for (int nu = 0; nu < NM; nu++) {
                const bool okp = (vp >> nu) & 1u, okm = (vm >> nu) & 1u;
                if (!(okp || okm)) continue;
                double gr = 0, gi = 0;
#pragma unroll
                for (int mu = 0; mu < NM; mu++) {
                  const double2 u = ur[nu * NM + mu];
                  gr += wr[mu] * u.x - wi[mu] * u.y;
                  gi += wr[mu] * u.y + wi[mu] * u.x;
                }
                const double g2 = gr * gr + gi * gi;
                const double xp = es + om[nu] - ep, xm = es - om[nu] - ep;
                const double dp = okp ? exp(-(xp * inv_eta) * (xp * inv_eta)) * dnorm : 0.0;
                const double dm = okm ? exp(-(xm * inv_eta) * (xm * inv_eta)) * dnorm : 0.0;
                nterm += (int)okp + (int)okm;
#pragma unroll
                for (int t = 0; t < EPH_MAX_TEMPS; t++) {
                  if (t < nt) {
                    const double nq = qr[NM + nu * nt + t], fo = pr[1 + t];
                    contrib[t] += g2 * ((nq + fo) * dp + (1.0 + nq - fo) * dm);
                  }
                }
              }
            }
            if (hit) atomicOr(&sMask[s * MW + (q1 >> 6)], 1ull << (q1 & 63));
            if (nterm) atomicAdd(&sTerms[s], nterm);
          }
#pragma unroll
          for (int t = 0; t < EPH_MAX_TEMPS; t++)
            if (t < nt) sContrib[li * nt + t] = contrib[t];
        }
        __syncthreads();
        // per-state sums of this round, in candidate order
        if (tid < S * nt) {
          const int s = tid / nt, t = tid - (tid / nt) * nt;
          int b = 0;
          for (int s2 = 0; s2 < s; s2++) b += sCnt[s2];
          const int e = b + sCnt[s];
          const int lo = b > r0 ? b : r0, hi = e < r0 + kRound ? e : r0 + kRound;
          double v = 0.0;
          for (int i = lo; i < hi; i++) v += sContrib[(i - r0) * nt + t];
          sAcc[s * nt + t] += v;
        }
        __syncthreads();
      }
      // ---- q-line counts, stage the next line ----
      if (tid < S) {
        unsigned long long c = 0;
        for (int w = 0; w < MW; w++) c += __popcll(sMask[tid * MW + w]);
        my_nq += c;
        my_nt += (unsigned long long)sTerms[tid];
        bool first = !(cont && sK1[tid] == sK1[0]);
        for (int s2 = 0; s2 < tid; s2++) first = first && (sK1[s2] != sK1[tid]);
        if (first) {
          const bool with_shadow = sK1[tid] == sK1[S - 1];
          for (int w = 0; w < MW; w++) {
            unsigned long long o = 0;
            for (int s2 = 0; s2 < S; s2++)
              if (sK1[s2] == sK1[tid]) o |= sMask[s2 * MW + w];
            if (with_shadow)
              for (int s2 = S; s2 < ST; s2++) o |= sMask[s2 * MW + w];
            my_nkq += __popcll(o);
          }
        }
      }
      __syncthreads();
      for (int t = tid; t < SMX * MW; t += kThreads) sMask[t] = 0ull;
      if (tid < SMX) sTerms[tid] = 0;
#pragma unroll
      for (int i = 0; i < LPF; i++) {
        if (i < qsl) {
          const int e = tid + kThreads * i;
          if (e < nq_chunk) sQT[e] = pf[i];
        } else {
          const int e = tid + kThreads * (i - qsl);
          if (e < np_chunk) sPT[e] = pf[i];
        }
      }
      __syncthreads();
    }
  }
  // ---- outputs ----
  if (tid < S * nt) {
    const int s = tid / nt, t = tid - (tid / nt) * nt;
    a.inv_tau[(int64_t)t * a.ns_total + s0 + s] = a.pref * sAcc[s * nt + t];
  }
  if (tid < S) {
    a.st_counts[(s0 + tid) * 2] = (int64_t)my_nq;
    a.st_counts[(s0 + tid) * 2 + 1] = (int64_t)my_nt;
  }
  unsigned long long v1 = my_nkq, v2 = my_nv;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    v1 += __shfl_xor(v1, m, 64);
    v2 += __shfl_xor(v2, m, 64);
  }
  if (lane == 0) {
    atomicAdd(a.n_kq, v1);
    atomicAdd(a.n_vertex, v2);
  }
}

// Packed records: q-side [q][om NM | occ_n NM*nt | u NM*NM complex],
// p-side [p][m][eps | occ_f nt | V row NW complex].
__global__ void pack_tables_kernel(int64_t nq, int nw, int nm, int nt, const double *__restrict__ eps,
                                   const double *__restrict__ om, const double2 *__restrict__ evec,
                                   const double2 *__restrict__ uu, const double *__restrict__ occ_f,
                                   const double *__restrict__ occ_n, double *__restrict__ qt,
                                   double *__restrict__ pt) {
  const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (q >= nq) return;
  const int QR = qrec(nm, nt), PR = prec(nw, nt);
  double *r = qt + q * QR;
  for (int nu = 0; nu < nm; nu++) r[nu] = om[q * nm + nu];
  for (int x = 0; x < nm * nt; x++) r[nm + x] = occ_n[(q * nm + x / nt) * EPH_MAX_TEMPS + x % nt];
  const int ou = qoff_u(nm, nt), ov = poff_v(nt);
  for (int x = nm + nm * nt; x < ou; x++) r[x] = 0.0;
  for (int x = 0; x < nm * nm; x++) {
    r[ou + 2 * x] = uu[q * nm * nm + x].x;
    r[ou + 2 * x + 1] = uu[q * nm * nm + x].y;
  }
  for (int m = 0; m < nw; m++) {
    double *p = pt + (q * nw + m) * PR;
    p[0] = eps[q * nw + m];
    for (int t = 0; t < nt; t++) p[1 + t] = occ_f[(q * nw + m) * EPH_MAX_TEMPS + t];
    for (int x = 1 + nt; x < ov; x++) p[x] = 0.0;
    for (int i = 0; i < nw; i++) {
      p[ov + 2 * i] = evec[(q * nw + m) * nw + i].x;
      p[ov + 2 * i + 1] = evec[(q * nw + m) * nw + i].y;
    }
  }
}

template <int NW, int NM, int NB, int SG, int NSLOT, int LPF>
hipError_t launch_stage_l(const RatesArgs &a, const double *qt, const double *pt, hipStream_t st) {
  const StageLayout<NW, NM, NB, SG> L(a.N, a.nt);
  if (L.total > 160 * 1024) return hipErrorInvalidValue;
  auto kern = rates_stage_kernel<NW, NM, NB, SG, NSLOT, LPF>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
  if (e != hipSuccess) return e;
  const int64_t grid = ((a.ng + 7) / 8) * 8;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(kThreads), L.total, st, a, qt, pt);
  return hipGetLastError();
}

}  // namespace

// Served shapes: 4 orbitals or fewer, 3 modes, cubic Rp box of edge 4 or 6,
// staged tables (both chunks) within the LDS budget.  Returns the states per
// group (0 = not served).
int rates_stage_group(int nw, int nm, RpBox box, int N, int nt) {
  const bool cube = box.n[0] == box.n[1] && box.n[1] == box.n[2] && (box.n[0] == 4 || box.n[0] == 6);
  if (!cube || nm != 3 || !(nw == 1 || nw == 2 || nw == 4)) return 0;
  const int slots = (N * qrec(nm, nt) + kThreads - 1) / kThreads + (N * nw * prec(nw, nt) + kThreads - 1) / kThreads;
  if (slots > 24) return 0;
  if (nw == 4 && box.n[0] == 6) {
    StageLayout<4, 3, 6, kStageSG> L(N, nt);
    return L.total <= 160 * 1024 ? kStageSG : 0;
  }
  return 0;
}

hipError_t launch_pack_tables(int64_t nq, int nw, int nm, int nt, const double *eps, const double *om,
                              const double2 *evec, const double2 *uu, const double *occ_f, const double *occ_n,
                              double *qt, double *pt, hipStream_t st) {
  hipLaunchKernelGGL(pack_tables_kernel, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, nq, nw, nm, nt, eps,
                     om, evec, uu, occ_f, occ_n, qt, pt);
  return hipGetLastError();
}

size_t stage_table_words(int64_t nq, int nw, int nm, int nt) {
  return (size_t)nq * (qrec(nm, nt) + (size_t)nw * prec(nw, nt));
}

hipError_t launch_rates_stage(const RatesArgs &a, const double *qt, const double *pt, hipStream_t st) {
  if (a.ng <= 0) return hipSuccess;
  const int lpf = (a.N * qrec(a.nm, a.nt) + kThreads - 1) / kThreads +
                  (a.N * a.nw * prec(a.nw, a.nt) + kThreads - 1) / kThreads;
  constexpr int NS = (kStageSG * 6 * 12 + kThreads - 1) / kThreads;
  if (a.nw == 4 && a.nm == 3 && a.box.n[0] == 6) {
    if (lpf <= 8) return launch_stage_l<4, 3, 6, kStageSG, NS, 8>(a, qt, pt, st);
    if (lpf <= 16) return launch_stage_l<4, 3, 6, kStageSG, NS, 16>(a, qt, pt, st);
    if (lpf <= 24) return launch_stage_l<4, 3, 6, kStageSG, NS, 24>(a, qt, pt, st);
  }
  return hipErrorNotSupported;
}

}  // namespace eph
