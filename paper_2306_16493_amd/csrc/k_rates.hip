// SERTA scattering rates on gfx950: the Rp -> q transform, the i -> m and
// mu -> nu rotations, the energy-conservation sieve, |g|^2, occupations and
// the Gaussian delta, fused in one kernel (Sec. II.B interpolation of g in
// the q-batch bracket order of Sec. III.C; SERTA rate of Sec. II.C; sieve of
// Sec. III.A).
//
// Work decomposition.  A workgroup owns a group of <= SMAX initial states
// that share the k-line (k2, k3) and sweeps every q-line (q2, q3) of the
// grid.  The Rp box is separable, so for a state s
//   Y_s(p1,p2; q3) = sum_p3 e^{i 2pi q3 p3/N} X_s(p1,p2,p3)      (per q3)
//   Z_s(p1; q2,q3) = sum_p2 e^{i 2pi q2 p2/N} Y_s(p1,p2; q3)     (per q-line)
//   G_s(q)         = sum_p1 e^{i 2pi q1 p1/N} Z_s(p1; q2,q3)     (per q)
// which is the same sum as the direct Rp sum, associated differently.
// Along a q-line all states of the group see the same final-state line
// p = k + q (shifted by k1), whose (energy, band) entries are pre-sorted by
// energy: a binary search per state yields exactly the candidate final
// states (p1, m) with |eps_s - eps_m(p)| <= max(hbar w) + sw*eta, and only
// those are expanded.  For a candidate, the vertex is contracted onto the
// single final band m first (W_mu = sum_i conj(V_im(p)) G_s(i, mu)) and then
// onto the modes (g_nu = sum_mu W_mu u_{mu nu}(q)), so work scales with the
// energy-conserving (q, m) pairs rather than with all bands.
// Accumulation of 1/tau is per thread in registers and reduced in a fixed
// order at the end (no floating-point atomics).
#include "dev_util.h"
#include "internal.h"

namespace eph {
namespace {

__device__ __forceinline__ int pmod(int64_t a, int N) {
  int64_t r = a % N;
  return (int)(r < 0 ? r + N : r);
}

__device__ __forceinline__ int lower_bound_lds(const double *a, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}
__device__ __forceinline__ int upper_bound_lds(const double *a, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] <= x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

struct Smem {
  size_t tab, y, z, le, lk, mask, misc, total;
};

template <class T>
__host__ __device__ inline Smem smem_layout(int N, int nw, int C, int smax, RpBox box) {
  using C2 = typename V2<T>::t;
  Smem s;
  size_t o = 0;
  s.tab = o; o = align16(o + sizeof(C2) * N);
  s.y = o; o = align16(o + sizeof(C2) * (size_t)smax * box.n[0] * box.n[1] * C);
  s.z = o; o = align16(o + sizeof(C2) * (size_t)smax * box.n[0] * C);
  s.le = o; o = align16(o + sizeof(double) * (size_t)N * nw);
  s.lk = o; o = align16(o + sizeof(uint16_t) * (size_t)N * nw);
  int mw = (N + 63) / 64;
  s.mask = o; o = align16(o + sizeof(unsigned long long) * 2 * (smax + nw) * mw);
  s.misc = o; o = align16(o + 2048 + sizeof(double) * 4 * smax * EPH_MAX_TEMPS + 32 * (smax + nw));
  s.total = o;
  return s;
}

// T: transform/rotation arithmetic (double or float).  Energies, the sieve,
// occupations and the 1/tau accumulation are FP64 in every form.
template <class T, int NW, int NM, int SMAX>
__global__ __launch_bounds__(256) void rates_kernel(RatesArgs a) {
  using C2 = typename V2<T>::t;
  constexpr int C = NW * NM;
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = a.N;
  const int n1 = a.box.n[0], n2 = a.box.n[1], n3 = a.box.n[2];
  const int lo1 = a.box.lo[0], lo2 = a.box.lo[1], lo3 = a.box.lo[2];
  const int nbox = n1 * n2 * n3;
  const int LN = N * NW;
  const int MW = (N + 63) / 64;
  const Smem L = smem_layout<T>(N, NW, C, SMAX, a.box);
  C2 *sTab = reinterpret_cast<C2 *>(smem + L.tab);
  C2 *sY = reinterpret_cast<C2 *>(smem + L.y);
  C2 *sZ = reinterpret_cast<C2 *>(smem + L.z);
  double *sLE = reinterpret_cast<double *>(smem + L.le);
  uint16_t *sLK = reinterpret_cast<uint16_t *>(smem + L.lk);
  unsigned long long *sMask = reinterpret_cast<unsigned long long *>(smem + L.mask);
  // per-state arrays cover the SMAX member states and up to NW-1 "shadow"
  // states: the remaining states of the group's last k point when that
  // k point continues into the next group.  Shadows only take part in the
  // (k,q) pair count, so every k point is counted by exactly one group.
  constexpr int STM = SMAX + NW;
  int *sLo = reinterpret_cast<int *>(smem + L.misc);
  int *sCnt = sLo + STM;
  int *sK1 = sCnt + STM;
  int *sTerms = sK1 + STM;  // kept terms of the current q-line
  unsigned long long *sNq = reinterpret_cast<unsigned long long *>(sTerms + STM + (STM & 1));
  unsigned long long *sNt = sNq + SMAX;
  unsigned long long *sNkq = sNt + SMAX;  // [0] (k,q) pairs, [1] vertex contractions
  double *sEps = reinterpret_cast<double *>(sNkq + 2);  // sNkq holds 2 counters
  double *sPart = sEps + STM;  // [4 waves][SMAX*EPH_MAX_TEMPS]

  const int tid = threadIdx.x;
  // XCD-aware: the 8 XCDs receive blocks round-robin; give each XCD a
  // contiguous range of groups so neighbouring k-lines share L2.
  const int64_t per_xcd = (a.ng + 7) / 8;
  const int64_t g = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (g >= a.ng) return;
  const int64_t s0 = a.gstart[g];
  const int S = (int)(a.gstart[g + 1] - s0);
  const int64_t kfirst = a.sk[s0];
  int SH = 0;
  {
    const int64_t klast = a.sk[s0 + S - 1];
    while (SH < NW - 1 && s0 + S + SH < a.ns_total && a.sk[s0 + S + SH] == klast) SH++;
  }
  const int ST = S + SH;
  const bool cont = (s0 > 0) && (a.sk[s0 - 1] == kfirst);  // first k point owned by an earlier group
  const int k2 = (int)((kfirst / N) % N), k3 = (int)(kfirst / ((int64_t)N * N));
  const double W = a.wmax + a.sw * a.eta;
  const double cut = a.sw * a.eta;
  const double inv_eta = 1.0 / a.eta;
  const double dnorm = 1.0 / (1.7724538509055160273 * a.eta);  // 1/(sqrt(pi) eta)

  for (int t = tid; t < N; t += 256) sTab[t] = mk<T>((T)a.tab[t].x, (T)a.tab[t].y);
  if (tid < STM) {
    if (tid < ST) {
      int64_t k = a.sk[s0 + tid];
      sK1[tid] = (int)(k % N);
      sEps[tid] = a.eps[k * NW + a.sn[s0 + tid]];
    }
    if (tid < SMAX) {
      sNq[tid] = 0;
      sNt[tid] = 0;
    }
    sTerms[tid] = 0;
  }
  if (tid == 0) sNkq[0] = sNkq[1] = 0;  // [1] unused
  for (int t = tid; t < 2 * STM * MW; t += 256) sMask[t] = 0ull;

  double acc[SMAX][EPH_MAX_TEMPS];
#pragma unroll
  for (int s = 0; s < SMAX; s++)
#pragma unroll
    for (int t = 0; t < EPH_MAX_TEMPS; t++) acc[s][t] = 0.0;

  const C2 *Xg = reinterpret_cast<const C2 *>(a.X);
  int buf = 0;
  unsigned nvx = 0;  // vertex contractions done by this thread
  for (int q3 = 0; q3 < N; q3++) {
    __syncthreads();
    // ---- Y_s(p1,p2; q3) ----
    for (int idx = tid; idx < S * n1 * n2 * C; idx += 256) {
      int s = idx / (n1 * n2 * C), rem = idx % (n1 * n2 * C);
      int p12 = rem / C, c = rem % C;
      const C2 *xs = Xg + ((s0 + s - a.s_base) * nbox + (int64_t)p12 * n3) * C + c;
      T yr = 0, yi = 0;
      for (int p3 = 0; p3 < n3; p3++) {
        C2 ph = sTab[pmod((int64_t)q3 * (lo3 + p3), N)];
        C2 x = xs[p3 * C];
        yr += ph.x * x.x - ph.y * x.y;
        yi += ph.x * x.y + ph.y * x.x;
      }
      sY[(s * n1 * n2 + p12) * C + c] = mk<T>(yr, yi);
    }
    __syncthreads();
    for (int q2 = 0; q2 < N; q2++) {
      // ---- Z_s(p1; q2, q3) and the energy-sorted final-state line ----
      for (int idx = tid; idx < S * n1 * C; idx += 256) {
        int s = idx / (n1 * C), rem = idx % (n1 * C);
        int p1 = rem / C, c = rem % C;
        const C2 *ys = sY + (s * n1 * n2 + p1 * n2) * C + c;
        T zr = 0, zi = 0;
        for (int p2 = 0; p2 < n2; p2++) {
          C2 ph = sTab[pmod((int64_t)q2 * (lo2 + p2), N)];
          C2 y = ys[p2 * C];
          zr += ph.x * y.x - ph.y * y.y;
          zi += ph.x * y.y + ph.y * y.x;
        }
        sZ[(s * n1 + p1) * C + c] = mk<T>(zr, zi);
      }
      const int64_t line = (int64_t)((k2 + q2) % N) + (int64_t)N * ((k3 + q3) % N);
      for (int t = tid; t < LN; t += 256) {
        sLE[t] = a.line_e[line * LN + t];
        sLK[t] = a.line_key[line * LN + t];
      }
      __syncthreads();
      if (tid < ST) {
        double e = sEps[tid];
        int lo = lower_bound_lds(sLE, LN, e - W);
        int hi = upper_bound_lds(sLE, LN, e + W);
        sLo[tid] = lo;
        sCnt[tid] = hi - lo;
      }
      __syncthreads();
      int pre[STM + 1];
      pre[0] = 0;
#pragma unroll
      for (int s = 0; s < STM; s++) pre[s + 1] = pre[s] + (s < ST ? sCnt[s] : 0);
      const int total = pre[STM];
      unsigned long long *mask = sMask + buf * STM * MW;
      for (int t = tid; t < total; t += 256) {
        int s = 0;
#pragma unroll
        for (int ss = 1; ss < STM; ss++) s += (t >= pre[ss]) ? 1 : 0;
        const int jj = sLo[s] + (t - pre[s]);
        const int key = sLK[jj];
        const int p1 = key / NW, m = key % NW;
        const int q1 = pmod(p1 - sK1[s], N);
        const int64_t qidx = q1 + (int64_t)N * (q2 + (int64_t)N * q3);
        const int64_t pidx = p1 + (int64_t)N * line;
        const double es = sEps[s], ep = sLE[jj];
        double om[NM];
        unsigned vp = 0, vm = 0;
#pragma unroll
        for (int nu = 0; nu < NM; nu++) {
          om[nu] = a.om[qidx * NM + nu];
          bool ok = om[nu] >= a.wcut;
          vp |= (ok && fabs(es + om[nu] - ep) <= cut) ? (1u << nu) : 0u;
          vm |= (ok && fabs(es - om[nu] - ep) <= cut) ? (1u << nu) : 0u;
        }
        if ((vp | vm) == 0u) continue;
        if (s >= S) {  // shadow state: count the (k,q) pair only
          atomicOr(&mask[s * MW + (q1 >> 6)], 1ull << (q1 & 63));
          continue;
        }
        // W_mu = sum_p1' e^{i 2pi q1 p1'/N} sum_i conj(V_im(p)) Z_s(p1'; mu, i)
        C2 vrow[NW];
#pragma unroll
        for (int i = 0; i < NW; i++) {
          if constexpr (sizeof(T) == 8) {
            vrow[i] = a.evec[(pidx * NW + m) * NW + i];
          } else {
            vrow[i] = a.evec32[(pidx * NW + m) * NW + i];
          }
        }
        T wr[NM], wi[NM];
#pragma unroll
        for (int mu = 0; mu < NM; mu++) wr[mu] = wi[mu] = 0;
        for (int pp = 0; pp < n1; pp++) {
          C2 ph = sTab[pmod((int64_t)q1 * (lo1 + pp), N)];
          const C2 *zs = sZ + (s * n1 + pp) * C;
#pragma unroll
          for (int mu = 0; mu < NM; mu++) {
            T tr = 0, ti = 0;
#pragma unroll
            for (int i = 0; i < NW; i++) {
              C2 z = zs[mu * NW + i];
              // conj(v) * z
              tr += vrow[i].x * z.x + vrow[i].y * z.y;
              ti += vrow[i].x * z.y - vrow[i].y * z.x;
            }
            wr[mu] += ph.x * tr - ph.y * ti;
            wi[mu] += ph.x * ti + ph.y * tr;
          }
        }
        double contrib[EPH_MAX_TEMPS];
#pragma unroll
        for (int t2 = 0; t2 < EPH_MAX_TEMPS; t2++) contrib[t2] = 0.0;
        int nterm = 0;
#pragma unroll
        for (int nu = 0; nu < NM; nu++) {
          const bool okp = (vp >> nu) & 1u, okm = (vm >> nu) & 1u;
          if (!(okp || okm)) continue;
          T gr = 0, gi = 0;
#pragma unroll
          for (int mu = 0; mu < NM; mu++) {
            C2 u;
            if constexpr (sizeof(T) == 8) {
              u = a.uu[(qidx * NM + nu) * NM + mu];
            } else {
              u = a.uu32[(qidx * NM + nu) * NM + mu];
            }
            gr += wr[mu] * u.x - wi[mu] * u.y;
            gi += wr[mu] * u.y + wi[mu] * u.x;
          }
          const double g2 = (double)gr * (double)gr + (double)gi * (double)gi;
          const double xp = es + om[nu] - ep, xm = es - om[nu] - ep;
          const double dp = okp ? exp(-(xp * inv_eta) * (xp * inv_eta)) * dnorm : 0.0;
          const double dm = okm ? exp(-(xm * inv_eta) * (xm * inv_eta)) * dnorm : 0.0;
          nterm += (int)okp + (int)okm;
#pragma unroll
          for (int t2 = 0; t2 < EPH_MAX_TEMPS; t2++) {
            if (t2 < a.nt) {
              const double kt = a.temps_kt[t2];
              const double nq = 1.0 / expm1(om[nu] / kt);
              const double f = 1.0 / (exp((ep - a.mu) / kt) + 1.0);
              contrib[t2] += g2 * ((nq + f) * dp + (1.0 + nq - f) * dm);
            }
          }
        }
#pragma unroll
        for (int ss = 0; ss < SMAX; ss++)
          if (ss == s)
#pragma unroll
            for (int t2 = 0; t2 < EPH_MAX_TEMPS; t2++) acc[ss][t2] += contrib[t2];
        atomicOr(&mask[s * MW + (q1 >> 6)], 1ull << (q1 & 63));
        atomicAdd(&sTerms[s], nterm);
        nvx++;
      }
      __syncthreads();
      // ---- per-q-line counts; clear the other mask buffer ----
      if (tid < S) {
        unsigned long long c = 0;
        for (int w = 0; w < MW; w++) c += __popcll(mask[tid * MW + w]);
        sNq[tid] += c;
        sNt[tid] += sTerms[tid];
        sTerms[tid] = 0;
        bool first = !(cont && sK1[tid] == sK1[0]);
        for (int s2 = 0; s2 < tid; s2++) first = first && (sK1[s2] != sK1[tid]);
        if (first) {
          const bool with_shadow = sK1[tid] == sK1[S - 1];
          unsigned long long ck = 0;
          for (int w = 0; w < MW; w++) {
            unsigned long long o = 0;
            for (int s2 = 0; s2 < S; s2++)
              if (sK1[s2] == sK1[tid]) o |= mask[s2 * MW + w];
            if (with_shadow)
              for (int s2 = S; s2 < ST; s2++) o |= mask[s2 * MW + w];
            ck += __popcll(o);
          }
          atomicAdd(&sNkq[0], ck);
        }
      }
      unsigned long long *other = sMask + (buf ^ 1) * STM * MW;
      for (int t = tid; t < STM * MW; t += 256) other[t] = 0ull;
      buf ^= 1;
    }
  }
  // ---- fixed-order reduction of the per-thread rates ----
  __syncthreads();
  const int wave = tid / 64, lane = tid % 64;
#pragma unroll
  for (int s = 0; s < SMAX; s++)
#pragma unroll
    for (int t2 = 0; t2 < EPH_MAX_TEMPS; t2++) {
      double v = acc[s][t2];
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
      if (lane == 0) sPart[wave * SMAX * EPH_MAX_TEMPS + s * EPH_MAX_TEMPS + t2] = v;
    }
  __syncthreads();
  if (tid < S * EPH_MAX_TEMPS) {
    int s = tid / EPH_MAX_TEMPS, t2 = tid % EPH_MAX_TEMPS;
    if (t2 < a.nt) {
      double v = 0.0;
      for (int w = 0; w < 4; w++) v += sPart[w * SMAX * EPH_MAX_TEMPS + tid];
      a.inv_tau[(int64_t)t2 * a.ns_total + s0 + s] = a.pref * v;
    }
  }
  if (tid < S) {
    a.st_counts[(s0 + tid) * 2] = (int64_t)sNq[tid];
    a.st_counts[(s0 + tid) * 2 + 1] = (int64_t)sNt[tid];
  }
  {
    unsigned long long v = nvx;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    if (lane == 0) atomicAdd(a.n_vertex, v);
  }
  if (tid == 0) atomicAdd(a.n_kq, sNkq[0]);
}

template <class T, int NW, int NM, int SMAX>
hipError_t launch_one(const RatesArgs &a, hipStream_t st) {
  Smem L = smem_layout<T>(a.N, NW, NW * NM, SMAX, a.box);
  if (L.total > 160 * 1024) return hipErrorInvalidValue;
  auto kern = rates_kernel<T, NW, NM, SMAX>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.total);
  if (e != hipSuccess) return e;
  int64_t nblk = ((a.ng + 7) / 8) * 8;
  hipLaunchKernelGGL(kern, dim3((unsigned)nblk), dim3(256), L.total, st, a);
  return hipGetLastError();
}

template <class T>
hipError_t dispatch(const RatesArgs &a, hipStream_t st) {
  const int nw = a.nw, nm = a.nm;
#define EPH_R(NW_, NM_, SM_) \
  if (nw == NW_ && nm == NM_) return launch_one<T, NW_, NM_, SM_>(a, st)
  EPH_R(1, 3, 8);
  EPH_R(2, 3, 8);
  EPH_R(4, 3, 8);
  EPH_R(8, 3, 4);
  EPH_R(1, 6, 8);
  EPH_R(2, 6, 8);
  EPH_R(4, 6, 4);
  EPH_R(8, 6, 2);
#undef EPH_R
  return hipErrorNotSupported;
}

}  // namespace

int rates_group_max(int nw, int nm) {
  if (nm == 3) return nw >= 8 ? 4 : 8;
  return nw >= 8 ? 2 : nw >= 4 ? 4 : 8;
}

hipError_t launch_rates(int precision, const RatesArgs &a, hipStream_t st) {
  if (a.ng <= 0) return hipSuccess;
  if (precision == EPH_FP64) return dispatch<double>(a, st);
  return dispatch<float>(a, st);
}

size_t rates_smem_bytes(int precision, int N, int nw, int nm, RpBox box) {
  int smax = rates_group_max(nw, nm);
  if (precision == EPH_FP64) return smem_layout<double>(N, nw, nw * nm, smax, box).total;
  return smem_layout<float>(N, nw, nw * nm, smax, box).total;
}

}  // namespace eph
