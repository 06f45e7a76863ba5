#pragma once
// SERTA scattering rates, wave-autonomous form (gfx950): the kernel template.
// Instantiated per (precision, phonon modes) in k_rates_wave_<p><nm>.hip and
// dispatched by k_rates_wave.hip.
//
// Same arithmetic as the workgroup form (separable Rp box: Y per q3, Z per
// q-line, G per q; vertex contracted onto the final band m first, then onto
// the modes; sieve, occupations, Gaussian delta; Sec. II.B/II.C/III.A/III.C),
// organised so that no workgroup barrier sits inside the q loops:
//   * each wave64 owns a group of <= GW initial states on one k-line and
//     sweeps all q-lines on its own; the four waves of a workgroup take
//     consecutive groups of the same k-line, so their table reads share L1;
//   * Y_s(p1,p2; q3) lives in registers, one (state, p1, channel) pair per
//     lane slot, so Z_s(p1; q2,q3) is a lane-local 1-D transform whose
//     result goes to a ring of Z slots in the wave's LDS slice;
//   * the final-state line p = k + q (contiguous in the energy table) is
//     prefiltered 64 entries at a time against the group's state energies
//     (window max(hbar w) + sw*eta); passing (k-slot, p1) candidates are
//     compacted with ballots into a candidate queue;
//   * full passes of candidates are sieved exactly (FP64, every state and
//     final band) and the (state, m, p1) pairs with a kept term go to a
//     vertex queue; full passes of that queue evaluate one vertex per lane,
//     so no lane idles through state, band or mode loops;
//   * Fermi and Bose factors come from per-call grid tables, so a vertex
//     pays one exp per kept term (the delta) and no other transcendental;
//   * phases use 32-bit indices and, in the vertex, a recurrence.
// Per-state rates are accumulated per lane and reduced with a fixed
// butterfly at the end, so results are bit-reproducible.
#include <type_traits>

#include "dev_util.h"
#include "internal.h"

namespace eph {
namespace wave {

// Waves per workgroup: 4 (they share the phase table and, working on
// consecutive groups of one k-line, their L1), 2 for the FP64 form of 48
// channels, whose per-wave LDS would otherwise let only one workgroup of 4
// onto a CU.
template <class T, int NW, int NM>
__host__ __device__ constexpr int waves_per_block() {
  return (NW * NM >= 48 && sizeof(T) == 8) ? 2 : 4;
}

template <class T, int NW, int NM, int GW, int NB, class LT = double>
struct WaveLayout {
  static constexpr int C = NW * NM;
  static constexpr int SMX = GW + NW;  // member states + shadow states
  // Z ring slots (q-lines in flight): 4, or 2 for 48 channels (LDS)
  static constexpr int NZ = C >= 48 ? 2 : 4;
  static constexpr int WPB = waves_per_block<T, NW, NM>();
  static constexpr int VCAP = 64 + 64 * GW * NW;  // vertex queue: one pass of candidates + a partial pass
  // one Z block per (slot, state), padded by 16 bytes so that the blocks a
  // vertex pass reads at the same offset fall in different LDS banks
  static constexpr int ZB = NB * C + (int)(16 / sizeof(typename V2<T>::t));
  __host__ __device__ static size_t z_bytes() { return align16(sizeof(typename V2<T>::t) * NZ * GW * ZB); }
  __host__ __device__ static int qcap(int) { return 128; }  // drained in whole passes during the scan
  __host__ __device__ static size_t q_bytes(int N) { return align16(4 * (size_t)qcap(N)); }
  __host__ __device__ static size_t misc_bytes() { return align16(SMX * 8 + SMX * 4 * 4 + NZ * 8 + 64); }
  __host__ __device__ static size_t line_bytes(int N) { return align16(sizeof(LT) * (size_t)N * NW); }
  __host__ __device__ static size_t v_bytes() { return align16(8 * (size_t)VCAP); }
  __host__ __device__ static size_t per_wave(int N) {
    return z_bytes() + q_bytes(N) + misc_bytes() + line_bytes(N) + v_bytes();
  }
  __host__ __device__ static size_t tab_bytes(int N) { return align16(sizeof(typename V2<T>::t) * N); }
  __host__ __device__ static size_t total(int N) { return tab_bytes(N) + WPB * per_wave(N); }
};

// Waves per SIMD the register allocation targets: 3 for the FP32 form of up
// to 24 channels (whose LDS then also admits three workgroups per CU), 2
// otherwise.
template <class T, int NW, int NM>
__host__ __device__ constexpr int waves_per_eu() {
  return (sizeof(T) == 4 && NW * NM <= 24) ? 3 : 2;
}
// MODE: kRates computes 1/tau; kCount only counts, per state, the transition
// rates to final states in the state list (no transforms, no vertices);
// kEmit computes 1/tau and also writes those transition rates (the summed
// terms of each (state, q, m) vertex) at the state's running cursor.
template <class T, int NW, int NM, int GW, int NB, int LPL, int MODE>
__global__ __launch_bounds__((waves_per_block<T, NW, NM>() * 64))
__attribute__((amdgpu_waves_per_eu(waves_per_eu<T, NW, NM>())))
void rates_wave_kernel(RatesArgs a) {
  using C2 = typename V2<T>::t;
  // the prefilter reads a float copy of the final-state energies (half the
  // LDS and prefetch registers of an FP64 copy); its window is widened to
  // cover the rounding, and the exact sieve that follows is FP64
  using LT = float;
  using LY = WaveLayout<T, NW, NM, GW, NB, LT>;
  constexpr int C = NW * NM;
  constexpr int SMX = LY::SMX;
  constexpr int NZ = LY::NZ;
  constexpr int NPAIR = (GW * NB * C + 63) / 64;
  constexpr int WPB = LY::WPB;
  // lanes per vertex: with 8 orbitals and 6 modes a vertex is split over two
  // lanes (each contracts half of the orbitals, the halves are added, and
  // each rotates onto half of the modes), which keeps the kernel within its
  // registers next to Y
  constexpr int VL = (NW == 8 && NM == 6) ? 2 : 1;
  constexpr int NWL = NW / VL;  // orbitals per lane in the W contraction
  constexpr int NML = NM / VL;  // modes per lane in the rotation
  extern __shared__ __align__(16) unsigned char smem[];
  const int N = a.N;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int LN = N * NW;

  C2 *sTab = reinterpret_cast<C2 *>(smem);
  unsigned char *wb = smem + LY::tab_bytes(N) + (size_t)wave * LY::per_wave(N);
  C2 *sZ = reinterpret_cast<C2 *>(wb);  // [NZ][GW][ZB]: [NB][C] + pad
  uint32_t *sQ = reinterpret_cast<uint32_t *>(wb + LY::z_bytes());
  unsigned char *misc = wb + LY::z_bytes() + LY::q_bytes(N);
  double *sEps = reinterpret_cast<double *>(misc);  // [SMX] state energies
  int *sKs = reinterpret_cast<int *>(sEps + SMX);     // [SMX] k-slot of each state
  int *sKfirst = sKs + SMX;                           // [SMX] first state of each k-slot
  int *sKcnt = sKfirst + SMX;                         // [SMX] states of each k-slot
  int *sK1 = sKcnt + SMX;                             // [SMX] k1 of each k-slot
  int *sSlot = sK1 + SMX;                             // [NZ][2] (q2, line) of each Z slot
  LT *sLine = reinterpret_cast<LT *>(misc + LY::misc_bytes());  // [N][NW] current line energies
  uint2 *sV = reinterpret_cast<uint2 *>(misc + LY::misc_bytes() + LY::line_bytes(N));  // vertex queue

  for (int t = threadIdx.x; t < N; t += WPB * 64) sTab[t] = mk<T>((T)a.tab[t].x, (T)a.tab[t].y);
  __syncthreads();  // the only workgroup barrier

  // XCD-aware block order: consecutive block indices go round-robin to the
  // 8 XCDs, so give each XCD a contiguous range of groups.
  const int64_t nblk = (a.ng + WPB - 1) / WPB;
  const int64_t per_xcd = (nblk + 7) / 8;
  const int64_t blk = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  const int64_t g = blk * WPB + wave;
  if (blk >= nblk || g >= a.ng) return;  // wave-uniform

  const int64_t s0 = a.gstart[g];
  const int S = (int)(a.gstart[g + 1] - s0);
  const int64_t kfirst = a.sk[s0];
  int SH = 0;
  {
    const int64_t klast = a.sk[s0 + S - 1];
    while (SH < NW - 1 && s0 + S + SH < a.ns_total && a.sk[s0 + S + SH] == klast) SH++;
  }
  const int ST = S + SH;
  const bool cont = (s0 > 0) && (a.sk[s0 - 1] == kfirst);  // first k point counted by an earlier group
  const int k2 = (int)((kfirst / N) % N), k3 = (int)(kfirst / ((int64_t)N * N));
  // prefilter window (a float line copy is within 1e-4 eV of the FP64
  // values for |eps| < 1000 eV; the exact sieve that follows uses FP64)
  // (a float copy is within 1e-4 eV of the FP64 values for |eps| < 1000 eV)
  const double W = a.wmax + a.sw * a.eta + 1e-4;
  const double cut = a.sw * a.eta;
  const double inv_eta = 1.0 / a.eta;
  const double dnorm = 1.0 / (1.7724538509055160273 * a.eta);
  const int nt = a.nt;
  const int lo1 = a.box.lo[0], lo2 = a.box.lo[1], lo3 = a.box.lo[2];

  // states and k-slots (distinct k points, states of one k are contiguous)
  int NK = 0;
  if (lane == 0) {
    int64_t prev = -1;
    for (int s = 0; s < ST; s++) {
      const int64_t k = a.sk[s0 + s];
      if (k != prev) {
        sKfirst[NK] = s;
        sKcnt[NK] = 0;
        sK1[NK] = (int)(k % N);
        NK++;
        prev = k;
      }
      sKs[s] = NK - 1;
      sKcnt[NK - 1]++;
      sEps[s] = a.eps[k * NW + a.sn[s0 + s]];
    }
  }
  NK = __shfl(NK, 0, 64);
  __syncwarp();
  int KMX = 0;  // most states at one k point of the group (wave-uniform)
  for (int ks = 0; ks < NK; ks++) KMX = max(KMX, sKcnt[ks]);
  double esm[GW];  // energies of the member states (wave-uniform)
#pragma unroll
  for (int ss = 0; ss < GW; ss++) esm[ss] = sEps[min(ss, S - 1)];

  double acc[GW][EPH_MAX_TEMPS];
  unsigned nq_s[GW], nt_s[GW];
#pragma unroll
  for (int s = 0; s < GW; s++) {
    nq_s[s] = nt_s[s] = 0u;
#pragma unroll
    for (int t = 0; t < EPH_MAX_TEMPS; t++) acc[s][t] = 0.0;
  }
  unsigned long long my_nkq = 0, my_nv = 0;
  // transition rates: per-state counts (kCount, per lane) or running write
  // positions (kEmit, wave-uniform)
  int64_t gcur[GW];
#pragma unroll
  for (int ss = 0; ss < GW; ss++) gcur[ss] = (MODE == kEmit && ss < S) ? a.g_cursor[s0 + ss] : 0;

  // pair slots of this lane: P = lane + 64 j -> (s, p1, c) = (P / (NB C), (P / C) % NB, P % C)
  T yr[NPAIR][NB], yi[NPAIR][NB];
  const C2 *Xg = reinterpret_cast<const C2 *>(a.X);
  const int64_t xrow = (int64_t)NB * NB * NB * C;

  // final-state line energies: the next q-line's are loaded into registers
  // while the current one (in LDS, [m][p1]) is scanned
  // in FP64, lines of up to 512 energies are prefetched into registers while
  // a line is worked on; longer lines, and every line in FP32, are copied at
  // the staging point instead (measured faster: the FP32 instances spill
  // with the prefetch registers, and at three waves per SIMD hide the
  // staging loads)
  constexpr bool PF = sizeof(T) == 8 && LPL <= 8;
  constexpr int LPR = PF ? LPL : 1;
  LT nxt[LPR];
  const LT *eline = a.eps32;  // float copy of the band energies, the prefilter's input
  // a line is kept in LDS as in the table, [p1][m], and copied with 16-byte
  // accesses when a row is a whole number of float4
  auto copy_line = [&](const LT *src) __attribute__((always_inline)) {
    if constexpr (NW % 4 == 0) {
      const float4 *s4 = reinterpret_cast<const float4 *>(src);
      float4 *d4 = reinterpret_cast<float4 *>(sLine);
      for (int e = lane; e < LN / 4; e += 64) d4[e] = s4[e];
    } else {
      for (int e = lane; e < LN; e += 64) sLine[e] = src[e];
    }
  };
  {
    const int l3 = (k3 + a.q3_lo >= N) ? k3 + a.q3_lo - N : k3 + a.q3_lo;
    copy_line(eline + (size_t)(k2 + N * l3) * LN);
  }

  // One candidate = (k-slot, p1, Z slot): every state of that k point against
  // every final band m at p = k + q.  Queue item (32 bits): p1 | ks << 10 |
  // zslot << 15 | (mask of the bands inside the prefilter window) << 17.
  static_assert(NZ <= 4 && NW <= 8 && SMX <= 32, "candidate item fields");
  int qn = 0;
  // Two-level form: stage1(n) sieves the first n queued candidates against
  // every (state, final band) pair and appends the pairs with a kept term to
  // the vertex queue (drained in whole passes after each candidate pass, so
  // it holds < 64 + 64*GW*NW entries); vdrain(n) evaluates the first n
  // vertices, one per lane.
  // Vertex item (64 bits): x = p1 | q1 << 10 | i1 << 20 | zslot << 30 with
  // i1 = q1*lo1 mod N the first phase index; y = s | m << 3 | vp << 6 |
  // vm << 12 | q2 << 18.
  int vn = 0;
  auto vdrain = [&](int count) __attribute__((always_inline)) {
    if constexpr (MODE == kCount) {
      // only which final states the kept vertices reach
      for (int base = 0; base < count; base += 64) {
        const int i = base + lane;
        if (i < count) {
          const uint2 it = sV[i];
          const int p1 = (int)(it.x & 1023u), s = (int)(it.y & 7u), m = (int)((it.y >> 3) & 7u);
          const int q2 = (int)((it.y >> 18) & 1023u);
          const int p2l = (k2 + q2 >= N) ? k2 + q2 - N : k2 + q2;
          const int p3l = (k3 + a.q3_cur >= N) ? k3 + a.q3_cur - N : k3 + a.q3_cur;
          const int64_t pidx = p1 + (int64_t)N * (p2l + (int64_t)N * p3l);
          const bool in_list = a.stidx[pidx * NW + m] >= 0;
#pragma unroll
          for (int ss = 0; ss < GW; ss++) gcur[ss] += (in_list && ss == s) ? 1 : 0;
        }
      }
      return;
    }
    const int h = (VL == 1) ? 0 : (lane & (VL - 1));  // this lane's half of a vertex
    for (int base = 0; base < count; base += 64 / VL) {
      const int i = base + lane / VL;
      int e_state = -1, e_col = -1;  // transition rate of this lane's vertex (kEmit)
      double e_val[EPH_MAX_TEMPS];
      if (i < count) {
      // everything the vertex needs is in its queue item (no table lookups)
      const uint2 it = sV[i];
      const int p1 = (int)(it.x & 1023u), q1 = (int)((it.x >> 10) & 1023u), i1 = (int)((it.x >> 20) & 1023u);
      const int zs_slot = (int)(it.x >> 30);
      const int s = (int)(it.y & 7u), m = (int)((it.y >> 3) & 7u);
      const unsigned vp = (it.y >> 6) & 63u, vm = (it.y >> 12) & 63u;
      const int q2 = (int)((it.y >> 18) & 1023u);
      const int p2l = (k2 + q2 >= N) ? k2 + q2 - N : k2 + q2;
      const int p3l = (k3 + a.q3_cur >= N) ? k3 + a.q3_cur - N : k3 + a.q3_cur;
      const int64_t qidx = q1 + (int64_t)N * (q2 + (int64_t)N * a.q3_cur);
      const int64_t pidx = p1 + (int64_t)N * (p2l + (int64_t)N * p3l);
      double es = esm[0];
#pragma unroll
      for (int ss = 1; ss < GW; ss++) es = (s == ss) ? esm[ss] : es;
      const double epm = a.eps[pidx * NW + m];
      double omq[NML];  // phonon energies of this lane's modes
#pragma unroll
      for (int nl = 0; nl < NML; nl++) omq[nl] = a.om[qidx * NM + h * NML + nl];
      my_nv += (h == 0) ? 1 : 0;
      C2 vrow[NWL];
#pragma unroll
      for (int j = 0; j < NWL; j++) {
        if constexpr (sizeof(T) == 8) vrow[j] = a.evec[(pidx * NW + m) * NW + h * NWL + j];
        else vrow[j] = a.evec32[(pidx * NW + m) * NW + h * NWL + j];
      }
      T wr[NM], wi[NM];
#pragma unroll
      for (int mu = 0; mu < NM; mu++) wr[mu] = wi[mu] = 0;
      // phases e^{i 2pi q1 p1'/N}, p1' = lo1 .. lo1 + NB - 1, by recurrence from
      // two table entries (per-lane table lookups would conflict in LDS banks)
      C2 ph = sTab[i1];
      const C2 rq = sTab[q1];
      const C2 *zs = sZ + ((size_t)zs_slot * GW + s) * LY::ZB + h * NWL;
#pragma unroll 1
      for (int pp = 0; pp < NB; pp++) {
#pragma unroll
        for (int mu = 0; mu < NM; mu++) {
          T tr = 0, ti = 0;
#pragma unroll
          for (int j = 0; j < NWL; j++) {
            const C2 z = zs[pp * C + mu * NW + j];
            cmac_conj<T>(tr, ti, vrow[j].x, vrow[j].y, z.x, z.y);
          }
          cmac<T>(wr[mu], wi[mu], ph.x, ph.y, tr, ti);
        }
        ph = mk<T>(fma(ph.x, rq.x, -ph.y * rq.y), fma(ph.x, rq.y, ph.y * rq.x));
      }
      if constexpr (VL == 2) {  // the two halves of the orbital sum (both lanes share i)
#pragma unroll
        for (int mu = 0; mu < NM; mu++) {
          wr[mu] += __shfl_xor(wr[mu], 1, 64);
          wi[mu] += __shfl_xor(wi[mu], 1, 64);
        }
      }
      double contrib[EPH_MAX_TEMPS];
      if constexpr (sizeof(T) == 8) {
        // FP64: the q-side data is loaded mode by mode (a single batch does not
        // fit the registers next to Y); occupation rows are padded to
        // EPH_MAX_TEMPS and padding is never accumulated into a written rate
        double fo[EPH_MAX_TEMPS];
#pragma unroll
        for (int t = 0; t < EPH_MAX_TEMPS; t++) fo[t] = a.occ_f[(pidx * NW + m) * EPH_MAX_TEMPS + t];
#pragma unroll
        for (int t = 0; t < EPH_MAX_TEMPS; t++) contrib[t] = 0.0;
#pragma unroll
        for (int nl = 0; nl < NML; nl++) {
          const int nu = h * NML + nl;
          const bool okp = (vp >> nu) & 1u, okm = (vm >> nu) & 1u;
          if (!(okp || okm)) continue;
          T gr = 0, gi = 0;
#pragma unroll
          for (int mu = 0; mu < NM; mu++) {
            const C2 u = a.uu[(qidx * NM + nu) * NM + mu];
            cmac<T>(gr, gi, wr[mu], wi[mu], u.x, u.y);
          }
          const double g2 = fma((double)gr, (double)gr, (double)gi * (double)gi);
          const double xp = es + omq[nl] - epm, xm = es - omq[nl] - epm;
          const double dp = okp ? exp(-(xp * inv_eta) * (xp * inv_eta)) * dnorm : 0.0;
          const double dm = okm ? exp(-(xm * inv_eta) * (xm * inv_eta)) * dnorm : 0.0;
#pragma unroll
          for (int t = 0; t < EPH_MAX_TEMPS; t++) {
            const double nq = a.occ_n[(qidx * NM + nu) * EPH_MAX_TEMPS + t];
            contrib[t] = fma(g2, fma(nq + fo[t], dp, (1.0 + nq - fo[t]) * dm), contrib[t]);
          }
        }
      } else {
        // FP32 form: the q-side data of this lane's modes and the Fermi
        // factors in one batch of loads from FP32 copies of the tables, and
        // |g|^2, the Gaussians and the occupation weights in FP32 (the
        // arguments x are formed in FP64 from the FP64 energies); the
        // vertex's contribution is then accumulated in FP64 (occupation rows
        // are padded to EPH_MAX_TEMPS; padding is never accumulated into a
        // written rate)
        static_assert(EPH_MAX_TEMPS == 4, "occupation rows are read as one float4");
        C2 uq[NML][NM];
        float4 nqv[NML];
#pragma unroll
        for (int nl = 0; nl < NML; nl++)
#pragma unroll
          for (int mu = 0; mu < NM; mu++) uq[nl][mu] = a.uu32[(qidx * NM + h * NML + nl) * NM + mu];
#pragma unroll
        for (int nl = 0; nl < NML; nl++)
          nqv[nl] = reinterpret_cast<const float4 *>(a.occ32_n)[qidx * NM + h * NML + nl];
        const float4 fo = reinterpret_cast<const float4 *>(a.occ32_f)[pidx * NW + m];
        const float ie = (float)inv_eta, dn = (float)dnorm;
        float cf[EPH_MAX_TEMPS] = {0.f, 0.f, 0.f, 0.f};
        // every mode is evaluated and masked (about 5 of the 6 (nu, +-) terms
        // of a vertex are kept, so branching would not save work)
#pragma unroll
        for (int nl = 0; nl < NML; nl++) {
          const int nu = h * NML + nl;
          const bool okp = (vp >> nu) & 1u, okm = (vm >> nu) & 1u;
          T gr = 0, gi = 0;
#pragma unroll
          for (int mu = 0; mu < NM; mu++) cmac<T>(gr, gi, wr[mu], wi[mu], uq[nl][mu].x, uq[nl][mu].y);
          const float g2 = fmaf(gr, gr, gi * gi);
          const float xp = (float)(es + omq[nl] - epm) * ie, xm = (float)(es - omq[nl] - epm) * ie;
          const float dp = okp ? __expf(-xp * xp) * dn : 0.f, dm = okm ? __expf(-xm * xm) * dn : 0.f;
          const float nq[EPH_MAX_TEMPS] = {nqv[nl].x, nqv[nl].y, nqv[nl].z, nqv[nl].w};
          const float ff[EPH_MAX_TEMPS] = {fo.x, fo.y, fo.z, fo.w};
#pragma unroll
          for (int t = 0; t < EPH_MAX_TEMPS; t++)
            cf[t] = fmaf(g2, fmaf(nq[t] + ff[t], dp, (1.f + nq[t] - ff[t]) * dm), cf[t]);
        }
#pragma unroll
        for (int t = 0; t < EPH_MAX_TEMPS; t++) contrib[t] = (double)cf[t];
      }
#pragma unroll
      for (int ss = 0; ss < GW; ss++) {
        const bool me = ss == s;
#pragma unroll
        for (int t = 0; t < EPH_MAX_TEMPS; t++) acc[ss][t] += me ? contrib[t] : 0.0;
      }
      if constexpr (MODE == kEmit) {
        // the vertex's transition rate: both halves' modes, emitted by lane half 0
#pragma unroll
        for (int t = 0; t < EPH_MAX_TEMPS; t++) {
          double v = contrib[t];
          if constexpr (VL == 2) v += __shfl_xor(v, 1, 64);
          e_val[t] = a.pref * v;
        }
        e_col = (h == 0) ? a.stidx[pidx * NW + m] : -1;
        e_state = s;
      }
      }
      if constexpr (MODE == kEmit) {
        // entries of one state go to consecutive positions in lane order
        // (all lanes take part in the ballots)
        const bool keep = e_col >= 0;
#pragma unroll
        for (int ss = 0; ss < GW; ss++) {
          const unsigned long long bits = __ballot(keep && e_state == ss);
          if (keep && e_state == ss) {
            const int64_t e = gcur[ss] + __popcll(bits & ((1ull << lane) - 1ull)) - a.g_base;
            a.g_col[e] = e_col;
            for (int t = 0; t < EPH_MAX_TEMPS; t++)
              if (t < nt) a.g_val[(int64_t)t * a.g_stride + e] = e_val[t];
          }
          gcur[ss] += __popcll(bits);
        }
      }
    }
  };
  auto vpop = [&](int n) __attribute__((always_inline)) {
    const int rem = vn - n;
    for (int b = 0; b < rem; b += 64) {
      const uint2 v = (b + lane < rem) ? sV[n + b + lane] : make_uint2(0u, 0u);
      __syncwarp();
      if (b + lane < rem) sV[b + lane] = v;
      __syncwarp();
    }
    vn = rem;
  };
  auto stage1 = [&](int count) __attribute__((always_inline)) {
    for (int base = 0; base < count; base += 64) {
      const int i = base + lane;
      const bool act = i < count;
      const uint32_t it = act ? sQ[i] : 0u;
      const int p1 = (int)(it & 1023u), ks = (int)((it >> 10) & 31u), zs_slot = (int)((it >> 15) & 3u);
      const unsigned bmask = it >> 17;  // final bands that passed the prefilter (0 for idle lanes)
      const int line = sSlot[2 * zs_slot + 1], q2 = sSlot[2 * zs_slot];
      int q1 = p1 - sK1[ks];
      q1 += (q1 < 0) ? N : 0;
      const int i1 = imod(q1 * lo1, N);
      const int64_t qidx = q1 + (int64_t)N * (q2 + (int64_t)N * a.q3_cur);
      const int64_t pidx = p1 + (int64_t)N * line;
      double om[NM], ep[NW];
#pragma unroll
      for (int nu = 0; nu < NM; nu++) om[nu] = act ? a.om[qidx * NM + nu] : 0.0;
#pragma unroll
      for (int m = 0; m < NW; m++) ep[m] = act ? a.eps[pidx * NW + m] : 0.0;
      // modes above the frequency cut (branch-free bit mask)
      unsigned okw = 0u;
#pragma unroll
      for (int nu = 0; nu < NM; nu++) okw |= (om[nu] >= a.wcut) ? (1u << nu) : 0u;
      // bands some lane needs: a band outside the prefilter window of every
      // lane's k-slot keeps no term, so it is skipped by the whole wave
      unsigned long long band_any[NW];
#pragma unroll
      for (int m = 0; m < NW; m++) band_any[m] = __ballot((bmask >> m) & 1u);
      const int sf = sKfirst[ks], sc = act ? sKcnt[ks] : 0;
      double esr[NW];
#pragma unroll
      for (int j = 0; j < NW; j++) esr[j] = (j < sc) ? sEps[sf + j] : 0.0;
      bool hit = false;
#pragma unroll
      for (int j = 0; j < NW; j++) {
        if (j >= KMX) break;  // wave-uniform
        const int s = sf + j;
        const bool sv = j < sc;
        const unsigned okj = sv ? okw : 0u;
        const double es = esr[j];
        // (es + w) and (es - w) once per state, in the oracle's order
        double wp[NM], wm[NM];
#pragma unroll
        for (int nu = 0; nu < NM; nu++) {
          wp[nu] = es + om[nu];
          wm[nu] = es - om[nu];
        }
        bool hit_s = false;
        unsigned nterm = 0;
#pragma unroll
        for (int m = 0; m < NW; m++) {
          if (!band_any[m]) continue;  // wave-uniform
          unsigned vp = 0u, vm = 0u;
#pragma unroll
          for (int nu = 0; nu < NM; nu++) {
            vp |= (fabs(wp[nu] - ep[m]) <= cut) ? (1u << nu) : 0u;
            vm |= (fabs(wm[nu] - ep[m]) <= cut) ? (1u << nu) : 0u;
          }
          vp &= okj;
          vm &= okj;
          const bool any = (vp | vm) != 0u;
          hit_s |= any;
          nterm += (unsigned)(__popc(vp) + __popc(vm));
          const bool push = any && s < S;
          const unsigned long long bits = __ballot(push);
          if (push)
            sV[vn + __popcll(bits & ((1ull << lane) - 1ull))] =
                make_uint2((uint32_t)p1 | ((uint32_t)q1 << 10) | ((uint32_t)i1 << 20) | ((uint32_t)zs_slot << 30),
                           (uint32_t)s | ((uint32_t)m << 3) | (vp << 6) | (vm << 12) | ((uint32_t)q2 << 18));
          vn += __popcll(bits);
        }
        hit = hit || hit_s;
        // branch-free per-slot updates (a select on s would become a
        // dynamically indexed private array)
#pragma unroll
        for (int ss = 0; ss < GW; ss++) {
          const bool me = (ss == s) && sv;
          nq_s[ss] += (me && hit_s) ? 1u : 0u;
          nt_s[ss] += me ? nterm : 0u;
        }
      }
      if (act && hit && !(cont && ks == 0)) my_nkq++;
      __syncwarp();
      if (vn >= 64) {  // keep the vertex queue below one pass before the next candidates
        const int vf = vn & ~63;
        vdrain(vf);
        __syncwarp();
        vpop(vf);
      }
    }
  };
  // drop the first n entries of the queue (after they were evaluated)
  auto pop = [&](int n) __attribute__((always_inline)) {
    const int rem = qn - n;
    for (int b = 0; b < rem; b += 64) {
      const uint32_t v = (b + lane < rem) ? sQ[n + b + lane] : 0u;
      __syncwarp();
      if (b + lane < rem) sQ[b + lane] = v;
      __syncwarp();
    }
    qn = rem;
  };

  int ql = 0;  // q-lines started in this launch
  const LT *nline = eline;  // energies of the next q-line
  for (int q3 = a.q3_lo; q3 < a.q3_hi; q3++) {
    // ---- Y_s(p1, p2; q3) into registers (p3 loop rolled) ----
#pragma unroll
    for (int j = 0; j < NPAIR; j++)
#pragma unroll
      for (int p2 = 0; p2 < NB; p2++) yr[j][p2] = yi[j][p2] = 0;
    if constexpr (MODE != kCount) {
      // one pair slot at a time, p3 rolled: at most NB loads of X in flight,
      // so the loads do not compete with Y for registers
#pragma unroll
      for (int j = 0; j < NPAIR; j++) {
        const int P = lane + 64 * j;
        const int s = P / (NB * C), p1 = (P / C) % NB, c = P % C;
        if (s < S) {
          const C2 *xs = Xg + (s0 + s - a.s_base) * xrow + (int64_t)p1 * NB * NB * C + c;
          int i3 = imod(q3 * lo3, N);
#pragma unroll 1
          for (int p3 = 0; p3 < NB; p3++) {
            const C2 ph = sTab[i3];
            i3 += q3;
            i3 -= (i3 >= N) ? N : 0;
#pragma unroll
            for (int p2 = 0; p2 < NB; p2++) {
              const C2 x = xs[p2 * NB * C + p3 * C];
              cmac<T>(yr[j][p2], yi[j][p2], ph.x, ph.y, x.x, x.y);
            }
          }
        }
      }
    }
    const int p3line = (k3 + q3 >= N) ? k3 + q3 - N : k3 + q3;
    for (int q2 = 0; q2 < N; q2++, ql++) {
      const int zslot = ql & (NZ - 1);
      {  // the Z slot is reused: evaluate queued work that still points at it
        bool stale = false;
        for (int b = 0; b < qn; b += 64)
          stale |= (b + lane < qn) && (int)((sQ[b + lane] >> 15) & 3u) == zslot;
        for (int b = 0; b < vn; b += 64)
          stale |= (b + lane < vn) && (int)(sV[b + lane].x >> 30) == zslot;
        if (__any(stale)) {
          stage1(qn);
          __syncwarp();
          qn = 0;
          vdrain(vn);
          __syncwarp();
          vn = 0;
        }
      }
      {  // issue the loads of the next q-line's energies
        int nq2 = q2 + 1, nq3 = q3;
        if (nq2 == N) {
          nq2 = 0;
          nq3 = (q3 + 1 == N) ? 0 : q3 + 1;
        }
        const int n2l = (k2 + nq2 >= N) ? k2 + nq2 - N : k2 + nq2;
        const int n3l = (k3 + nq3 >= N) ? k3 + nq3 - N : k3 + nq3;
        nline = eline + (size_t)(n2l + N * n3l) * LN;
        if constexpr (PF) {
#pragma unroll
          for (int i = 0; i < LPL; i++) {
            const int e = lane + 64 * i;
            nxt[i] = (e < LN) ? nline[e] : (LT)0;
          }
        }
      }
      // ---- Z_s(p1; q2, q3) -> LDS slot ----
      C2 ph2[NB];
      {
        int i2 = imod(q2 * lo2, N);
#pragma unroll
        for (int p = 0; p < NB; p++) {
          ph2[p] = sTab[i2];
          i2 += q2;
          i2 -= (i2 >= N) ? N : 0;
        }
      }
      C2 *zslot_base = sZ + (size_t)zslot * GW * LY::ZB;
#pragma unroll
      for (int j = 0; j < NPAIR; j++) {
        const int P = lane + 64 * j;
        if (MODE != kCount && P < GW * NB * C) {
          T r = 0, i = 0;
#pragma unroll
          for (int p2 = 0; p2 < NB; p2++) cmac<T>(r, i, ph2[p2].x, ph2[p2].y, yr[j][p2], yi[j][p2]);
          zslot_base[(P / (NB * C)) * LY::ZB + P % (NB * C)] = mk<T>(r, i);
        }
      }
      const int p2line = (k2 + q2 >= N) ? k2 + q2 - N : k2 + q2;
      const int line = p2line + N * p3line;
      if (lane == 0) {
        sSlot[2 * zslot] = q2;
        sSlot[2 * zslot + 1] = line;
      }
      __syncwarp();
      // ---- candidates of this q-line: (k-slot, p1) with some band in the window ----
      // The states of one k point come in band order, so their energies
      // ascend; a final band within W of any of them lies in [e_first - W,
      // e_last + W], which is tested in float (a superset of the exact
      // test, which the FP64 sieve then makes).
      for (int ks = 0; ks < NK; ks++) {
        const int sf = sKfirst[ks], sc = sKcnt[ks];
        const float lo_w = (float)(sEps[sf] - W), hi_w = (float)(sEps[sf + sc - 1] + W);
        for (int c0 = 0; c0 < N; c0 += 64) {
          const int p1 = c0 + lane;
          unsigned bm = 0u;  // bands of this p1 inside the window
          if (p1 < N) {
            float ev[NW];
            if constexpr (NW % 4 == 0) {
#pragma unroll
              for (int v = 0; v < NW / 4; v++) {
                const float4 f = reinterpret_cast<const float4 *>(sLine + (size_t)p1 * NW)[v];
                ev[4 * v] = f.x;
                ev[4 * v + 1] = f.y;
                ev[4 * v + 2] = f.z;
                ev[4 * v + 3] = f.w;
              }
            } else {
#pragma unroll
              for (int m = 0; m < NW; m++) ev[m] = sLine[p1 * NW + m];
            }
#pragma unroll
            for (int m = 0; m < NW; m++) bm |= ((ev[m] >= lo_w) & (ev[m] <= hi_w)) ? (1u << m) : 0u;
          }
          const bool any = bm != 0u;
          const unsigned long long bits = __ballot(any);
          if (any) sQ[qn + __popcll(bits & ((1ull << lane) - 1ull))] =
              (uint32_t)p1 | ((uint32_t)ks << 10) | ((uint32_t)zslot << 15) | (bm << 17);
          qn += __popcll(bits);
          __syncwarp();
          if (qn >= 64) {  // whole passes only, so the queue stays below 128
            const int full = qn & ~63;
            stage1(full);
            __syncwarp();
            pop(full);
          }
        }
      }
      __syncwarp();
      // stage the next line's energies; the scan of this line is done, and
      // the drains read energies from global memory
      if constexpr (PF) {
#pragma unroll
        for (int i = 0; i < LPL; i++) {
          const int e = lane + 64 * i;
          if (e < LN) sLine[e] = nxt[i];
        }
      } else {
        copy_line(nline);
      }
      __syncwarp();
    }
  }
  stage1(qn);
  __syncwarp();
  vdrain(vn);

  if constexpr (MODE == kCount) {
    // per-state counts of transition rates, added up over the plane launches
#pragma unroll
    for (int s = 0; s < GW; s++) {
      int64_t c = gcur[s];
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m, 64);
      if (lane == 0 && s < S) a.g_cursor[s0 + s] += c;
    }
    return;
  }
  if constexpr (MODE == kEmit) {
#pragma unroll
    for (int s = 0; s < GW; s++)
      if (lane == 0 && s < S) a.g_cursor[s0 + s] = gcur[s];
  }

  // ---- fixed-order reductions; q3 slabs add up in launch order ----
#pragma unroll
  for (int s = 0; s < GW; s++) {
#pragma unroll
    for (int t = 0; t < EPH_MAX_TEMPS; t++) {
      double v = acc[s][t];
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
      if (lane == 0 && s < S && t < nt) {
        double *dst = a.inv_tau + (int64_t)t * a.ns_total + s0 + s;
        *dst = (a.q3_lo == 0 ? 0.0 : *dst) + a.pref * v;
      }
    }
    unsigned long long c1 = nq_s[s], c2 = nt_s[s];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      c1 += __shfl_xor(c1, m, 64);
      c2 += __shfl_xor(c2, m, 64);
    }
    if (lane == 0 && s < S) {
      int64_t *dst = a.st_counts + (s0 + s) * 2;
      dst[0] = (a.q3_lo == 0 ? 0 : dst[0]) + (int64_t)c1;
      dst[1] = (a.q3_lo == 0 ? 0 : dst[1]) + (int64_t)c2;
    }
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

template <class T, int NW, int NM, int GW, int NB, int LPL, int MODE>
hipError_t launch_wave_l(const RatesArgs &a, hipStream_t st) {
  using LY = WaveLayout<T, NW, NM, GW, NB, float>;
  const size_t sh = LY::total(a.N);
  if (sh > 160 * 1024) return hipErrorInvalidValue;
  auto kern = rates_wave_kernel<T, NW, NM, GW, NB, LPL, MODE>;
  hipError_t e = hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sh);
  if (e != hipSuccess) return e;
  const int64_t nblk = (a.ng + LY::WPB - 1) / LY::WPB;
  const int64_t grid = ((nblk + 7) / 8) * 8;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(LY::WPB * 64), sh, st, a);
  return hipGetLastError();
}

template <class T, int NW, int NM, int GW, int NB, int MODE>
hipError_t launch_wave(const RatesArgs &a, hipStream_t st) {
  const int ln = a.N * NW;
  if (ln <= 512) return launch_wave_l<T, NW, NM, GW, NB, 8, MODE>(a, st);
  if (ln <= 1024) return launch_wave_l<T, NW, NM, GW, NB, 16, MODE>(a, st);
  if (ln <= 2048) return launch_wave_l<T, NW, NM, GW, NB, 32, MODE>(a, st);
  return hipErrorNotSupported;
}


// Launch for one (precision, modes, mode) triple: dispatch on the orbital
// count and the Rp box edge.  GW (states per group) must match
// rates_wave_group.
template <class T, int NM, int MODE>
hipError_t dispatch_nm(const RatesArgs &a, hipStream_t st) {
  const int nb = a.box.n[0];
#define EPH_W(NW_, GW_)                                               \
  if (a.nw == NW_) {                                                  \
    if (nb == 4) return launch_wave<T, NW_, NM, GW_, 4, MODE>(a, st); \
    if (nb == 6) return launch_wave<T, NW_, NM, GW_, 6, MODE>(a, st); \
    return hipErrorNotSupported;                                      \
  }
  if constexpr (NM == 3) {
    EPH_W(1, 2)
    EPH_W(2, 2)
    EPH_W(4, 2)
    EPH_W(8, 1)
  } else {
    EPH_W(1, 2)
    EPH_W(2, 2)
    EPH_W(4, 1)
    EPH_W(8, 1)
  }
#undef EPH_W
  return hipErrorNotSupported;
}

}  // namespace wave
}  // namespace eph
