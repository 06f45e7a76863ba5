// The k-batch order of the vertex (Sec. III.D, the comparison of the
// q-batch and k-batch algorithms), kept beside the q-batch rate kernel to
// measure the paper's argument on this hardware.  Same rates, the other
// association of the same sum:
//   step 1, per q:       G_q(Re; nu, i, j) = sum_{Rp, mu} e^{iq.Rp} g_ij^mu(Re, Rp) u_{mu nu}(q)
//   step 2, per (k, q):  g_mn^nu = sum_{ij} conj(V_im(k+q)) [sum_Re e^{ik.Re} G_q(Re; nu, i, j)] V_jn(k)
// then the sieve, |g|^2, the Gaussians and the occupations as in the
// q-batch kernel.  The inner product of step 2 runs over Re for every
// valid (k, q): its volume is N_w^2 N_Re N_nu per pair against
// N_w N_nu N_Rp per (n, k, q) of the q-batch order (the ratio of Sec. III.D).
// Step 1 is one thread per output element; step 2 is one wave per state
// and q batch: lanes over the (nu, i, j) channels for the Re sum (LDS), then
// over the kept (m, nu) terms.  FP64, fixed summation order.
#include "dev_util.h"
#include "internal.h"

namespace eph {
namespace {

// Gq[b][r][nu][i][j] for q = q0 + b, b < nb
__global__ void kb_step1_kernel(int64_t q0, int nb, int N, RpBox box, int nre, int nm, int nw, int ncol,
                                const double2 *__restrict__ wt, const double2 *__restrict__ uu,
                                const double2 *__restrict__ tab, double2 *__restrict__ Gq) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t per_q = (int64_t)nre * nm * nw * nw;
  if (e >= per_q * nb) return;
  const int b = (int)(e / per_q);
  int64_t rem = e - (int64_t)b * per_q;
  const int r = (int)(rem / (nm * nw * nw));
  rem -= (int64_t)r * nm * nw * nw;
  const int nu = (int)(rem / (nw * nw));
  const int i = (int)((rem / nw) % nw), j = (int)(rem % nw);
  const int64_t q = q0 + b;
  const int q1 = (int)(q % N), q2 = (int)((q / N) % N), q3 = (int)(q / ((int64_t)N * N));
  double sr = 0.0, si = 0.0;
  for (int p1 = 0; p1 < box.n[0]; p1++)
    for (int p2 = 0; p2 < box.n[1]; p2++)
      for (int p3 = 0; p3 < box.n[2]; p3++) {
        const int p = (p1 * box.n[1] + p2) * box.n[2] + p3;
        int ph = (q1 * (box.lo[0] + p1) % N + q2 * (box.lo[1] + p2) % N + q3 * (box.lo[2] + p3) % N) % N;
        ph += ph < 0 ? N : 0;
        const double2 f = tab[ph];
        for (int mu = 0; mu < nm; mu++) {
          const double2 u = uu[(q * nm + nu) * nm + mu];
          const double2 g = wt[((size_t)r * nw + j) * ncol + ((size_t)p * nm + mu) * nw + i];
          const double fr = f.x * u.x - f.y * u.y, fi = f.x * u.y + f.y * u.x;  // e^{iq.Rp} u_{mu nu}
          sr = fma(fr, g.x, sr);
          sr = fma(-fi, g.y, sr);
          si = fma(fr, g.y, si);
          si = fma(fi, g.x, si);
        }
      }
  Gq[e] = make_double2(sr, si);
}

// one wave per state for the q batch [q0, q0 + nb)
template <int NW, int NM>
__global__ __launch_bounds__(64) void kb_step2_kernel(KBatchArgs a) {
  constexpr int C = NM * NW * NW;
  __shared__ double2 sG[C];  // sum_Re e^{ik.Re} G_q(Re; nu, i, j)
  const int lane = threadIdx.x;
  const int64_t s = blockIdx.x;
  if (s >= a.ns) return;
  const int N = a.N;
  const int64_t k = a.sk[s];
  const int n = a.sn[s];
  const int k1 = (int)(k % N), k2 = (int)((k / N) % N), k3 = (int)(k / ((int64_t)N * N));
  const double es = a.eps[k * NW + n];
  const double cut = a.sw * a.eta, inv_eta = 1.0 / a.eta, dnorm = 1.0 / (1.7724538509055160273 * a.eta);
  double acc[EPH_MAX_TEMPS] = {0.0, 0.0, 0.0, 0.0};
  int64_t nq_valid = 0, nterms = 0;
  for (int b = 0; b < a.nb; b++) {
    const int64_t q = a.q0 + b;
    const int q1 = (int)(q % N), q2 = (int)((q / N) % N), q3 = (int)(q / ((int64_t)N * N));
    const int64_t pidx = (k1 + q1) % N + (int64_t)N * ((k2 + q2) % N + (int64_t)N * ((k3 + q3) % N));
    // sieve: one lane per (m, nu), both signs; FP64 as the oracle writes it
    unsigned okp = 0u, okm = 0u;
    if (lane < NW * NM) {
      const int m = lane / NM, nu = lane % NM;
      const double w = a.om[q * NM + nu], ep = a.eps[pidx * NW + m];
      const bool live = w >= a.wcut;
      okp = (live && fabs(es + w - ep) <= cut) ? 1u : 0u;
      okm = (live && fabs(es - w - ep) <= cut) ? 1u : 0u;
    }
    const unsigned long long anyk = __ballot(okp | okm);
    if (!anyk) continue;
    nq_valid++;
    nterms += __popcll(__ballot(okp)) + __popcll(__ballot(okm));
    // Re sum of the channels
    const double2 *G = a.Gq + (int64_t)b * a.nre * C;
    for (int c = lane; c < C; c += 64) {
      double gr = 0.0, gi = 0.0;
      for (int r = 0; r < a.nre; r++) {
        int ph = (k1 * a.re[3 * r] % N + k2 * a.re[3 * r + 1] % N + k3 * a.re[3 * r + 2] % N) % N;
        ph += ph < 0 ? N : 0;
        const double2 f = a.tab[ph], g = G[(int64_t)r * C + c];
        gr = fma(f.x, g.x, gr);
        gr = fma(-f.y, g.y, gr);
        gi = fma(f.x, g.y, gi);
        gi = fma(f.y, g.x, gi);
      }
      sG[c] = make_double2(gr, gi);
    }
    __syncthreads();
    // band and mode rotation of the kept (m, nu) terms
    if (okp | okm) {
      const int m = lane / NM, nu = lane % NM;
      double tr = 0.0, ti = 0.0;
      for (int i = 0; i < NW; i++) {
        double ur = 0.0, ui = 0.0;  // sum_j G(nu, i, j) V_jn(k)
        for (int j = 0; j < NW; j++) {
          const double2 g = sG[(nu * NW + i) * NW + j], v = a.evec[(k * NW + n) * NW + j];
          ur = fma(g.x, v.x, ur);
          ur = fma(-g.y, v.y, ur);
          ui = fma(g.x, v.y, ui);
          ui = fma(g.y, v.x, ui);
        }
        const double2 vp = a.evec[(pidx * NW + m) * NW + i];  // conj(V_im(k+q))
        tr = fma(vp.x, ur, tr);
        tr = fma(vp.y, ui, tr);
        ti = fma(vp.x, ui, ti);
        ti = fma(-vp.y, ur, ti);
      }
      const double g2 = tr * tr + ti * ti;
      const double w = a.om[q * NM + nu], ep = a.eps[pidx * NW + m];
      const double xp = es + w - ep, xm = es - w - ep;
      const double dp = okp ? exp(-(xp * inv_eta) * (xp * inv_eta)) * dnorm : 0.0;
      const double dm = okm ? exp(-(xm * inv_eta) * (xm * inv_eta)) * dnorm : 0.0;
      for (int t = 0; t < EPH_MAX_TEMPS; t++) {
        const double nq = a.occ_n[(q * NM + nu) * EPH_MAX_TEMPS + t];
        const double fo = a.occ_f[(pidx * NW + m) * EPH_MAX_TEMPS + t];
        acc[t] = fma(g2, fma(nq + fo, dp, (1.0 + nq - fo) * dm), acc[t]);
      }
    }
    __syncthreads();
  }
  for (int t = 0; t < EPH_MAX_TEMPS; t++) {
    double v = acc[t];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane == 0 && t < a.nt) {
      double *dst = a.inv_tau + (int64_t)t * a.ns + s;
      *dst = (a.q0 == 0 ? 0.0 : *dst) + a.pref * v;
    }
  }
  if (lane == 0) {
    int64_t *dst = a.st_counts + s * 2;
    dst[0] = (a.q0 == 0 ? 0 : dst[0]) + nq_valid;
    dst[1] = (a.q0 == 0 ? 0 : dst[1]) + nterms;
  }
}

}  // namespace

hipError_t launch_kbatch_step1(int64_t q0, int nb, int N, RpBox box, int nre, int nm, int nw, int ncol,
                               const double2 *wt, const double2 *uu, const double2 *tab, double2 *Gq, hipStream_t st) {
  const int64_t n = (int64_t)nb * nre * nm * nw * nw;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(kb_step1_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, q0, nb, N, box, nre, nm,
                     nw, ncol, wt, uu, tab, Gq);
  return hipGetLastError();
}

hipError_t launch_kbatch_step2(const KBatchArgs &a, hipStream_t st) {
  if (a.ns <= 0) return hipSuccess;
#define EPH_KB(NW_, NM_) \
  if (a.nw == NW_ && a.nm == NM_) { \
    hipLaunchKernelGGL((kb_step2_kernel<NW_, NM_>), dim3((unsigned)a.ns), dim3(64), 0, st, a); \
    return hipGetLastError(); \
  }
  EPH_KB(1, 3)
  EPH_KB(2, 3)
  EPH_KB(4, 3)
  EPH_KB(8, 3)
  EPH_KB(1, 6)
  EPH_KB(2, 6)
  EPH_KB(4, 6)
  EPH_KB(8, 6)
#undef EPH_KB
  return hipErrorNotSupported;
}

}  // namespace eph
