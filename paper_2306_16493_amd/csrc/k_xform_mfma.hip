// Re transform fused with the j -> n rotation on bf16 MFMA with a split
// (x = hi + lo) and three products hi*hi + hi*lo + lo*hi accumulated in FP32
// (the reduced-precision form of the Re -> k step, the first bracket of the
// q-batch order of Sec. III.C; gfx950).
//
// Real formulation of the complex GEMM X[s][c] = sum_kk B[s][kk] W[kk][c]:
//   A[s][kk']  = Re B (kk' < K) | Im B (K <= kk' < 2K) | 0 (padding)
//   W'[2c  ][kk'] = Re W[kk][c] (kk' < K) | -Im W[kk][c]
//   W'[2c+1][kk'] = Im W[kk][c] (kk' < K) |  Re W[kk][c]
// so that X'[s][2c] = Re X and X'[s][2c+1] = Im X, i.e. X' is X as
// interleaved (re, im) floats.  Both operands are stored K-contiguous with
// the K extent padded to a multiple of 32 (KP), split into bf16 hi/lo: W'
// once per context, A once per batch of states (phase e^{ik.Re} times the
// eigenvector component, formed in FP64, rounded to FP32, then split).
//
// GEMM tiling: a 256-thread workgroup computes 128 (states) x 128 (real
// columns); each wave64 a 64 x 64 quarter as 4 x 4 tiles of
// v_mfma_f32_16x16x32_bf16 (three products each), K advancing 32 per step.
// The next K step's tiles are loaded from global memory into registers while
// the current one is multiplied, then written to the other half of a
// double-buffered LDS (rows padded against bank conflicts).  Workgroups are
// ordered so that each XCD takes a contiguous range of state tiles.
#include "dev_util.h"
#include "internal.h"

namespace eph {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int TM = 128, TN = 128, TK = 32;
constexpr int LDR = TK + 8;  // LDS row of one tile (bf16), padded by 16 bytes

__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

__host__ __device__ inline int padk(int k2) { return (k2 + TK - 1) / TK * TK; }

// A hi/lo [ns][KP] of the states: one thread per (state, kk).
__global__ void state_operand_kernel(int64_t ns, const int32_t *__restrict__ sk, const int32_t *__restrict__ sn,
                                     int N, int nw, int K, int KP, const int *__restrict__ re,
                                     const double2 *__restrict__ evec, const double2 *__restrict__ tab,
                                     __bf16 *__restrict__ ahi, __bf16 *__restrict__ alo) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t s = i / KP;
  const int kk = (int)(i - s * KP);
  if (s >= ns || kk >= KP) return;
  __bf16 *rh = ahi + s * KP, *rl = alo + s * KP;
  if (kk >= 2 * K) {  // padding of the K extent
    rh[kk] = (__bf16)0.f;
    rl[kk] = (__bf16)0.f;
    return;
  }
  if (kk >= K) return;  // the imaginary half is written with the real half
  const int k = sk[s], n = sn[s];
  const int k1 = k % N, k2 = (k / N) % N, k3 = k / (N * N);
  const int ir = kk / nw, j = kk - ir * nw;
  // phase index (k.Re mod N) in 32-bit integers: |k_i re_i| < 2^31
  int ph = (k1 * re[3 * ir] % N + k2 * re[3 * ir + 1] % N + k3 * re[3 * ir + 2] % N) % N;
  ph += ph < 0 ? N : 0;
  const double2 p = tab[ph], e = evec[((int64_t)k * nw + n) * nw + j];
  __bf16 h, l;
  split_bf16((float)(p.x * e.x - p.y * e.y), h, l);
  rh[kk] = h;
  rl[kk] = l;
  split_bf16((float)(p.x * e.y + p.y * e.x), h, l);
  rh[K + kk] = h;
  rl[K + kk] = l;
}

// 16-byte chunks of one operand tile (rows x TK bf16, hi and lo): 2 * rows * 4
__device__ __forceinline__ uint4 load_chunk(const __bf16 *__restrict__ base, int64_t rows_total, int64_t r0, int KP,
                                            int k0, int q) {
  // q = row * 4 + part, part = 8-element chunk of the 32-wide K step
  const int64_t r = r0 + (q >> 2);
  if (r >= rows_total) return make_uint4(0u, 0u, 0u, 0u);
  return *reinterpret_cast<const uint4 *>(base + r * KP + k0 + (q & 3) * 8);
}

__global__ __launch_bounds__(256) void xform_bf16x3_kernel(int64_t ns, int ncol2, int KP,
                                                           const __bf16 *__restrict__ ahi,
                                                           const __bf16 *__restrict__ alo,
                                                           const __bf16 *__restrict__ whi,
                                                           const __bf16 *__restrict__ wlo, float *__restrict__ X,
                                                           int tiles_m, int tiles_n) {
  // LDS (dynamic, 80 KB): [stage][hi/lo][rows][LDR] for A (states), then W (columns)
  extern __shared__ __align__(16) unsigned char smem[];
  auto sA = reinterpret_cast<__bf16(*)[2][TM][LDR]>(smem);
  auto sW = reinterpret_cast<__bf16(*)[2][TN][LDR]>(smem + sizeof(__bf16) * 2 * 2 * TM * LDR);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // XCD-aware order: consecutive workgroup ids go round-robin to the 8 XCDs;
  // give each XCD a contiguous range of tiles (the W tiles it streams stay
  // in its L2 while the state tiles advance)
  const int64_t ntile = (int64_t)tiles_m * tiles_n;
  const int64_t per_xcd = (ntile + 7) / 8;
  const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (t >= ntile) return;
  const int tn = (int)(t % tiles_n);
  const int64_t tm = t / tiles_n;
  const int64_t m0 = tm * TM;
  const int n0 = tn * TN;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;

  floatx4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  // each thread moves 2 chunks of A hi, 2 of A lo, 2 of W hi, 2 of W lo per K step
  uint4 ra[2][2], rw[2][2];
  auto fetch = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < 2; c++) {
      const int q = tid + 256 * c;  // 0 .. 511 = 128 rows x 4 chunks
      ra[0][c] = load_chunk(ahi, ns, m0, KP, k0, q);
      ra[1][c] = load_chunk(alo, ns, m0, KP, k0, q);
      rw[0][c] = load_chunk(whi, ncol2, n0, KP, k0, q);
      rw[1][c] = load_chunk(wlo, ncol2, n0, KP, k0, q);
    }
  };
  auto stash = [&](int st) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < 2; c++) {
      const int q = tid + 256 * c, r = q >> 2, kc = (q & 3) * 8;
#pragma unroll
      for (int hl = 0; hl < 2; hl++) {
        *reinterpret_cast<uint4 *>(&sA[st][hl][r][kc]) = ra[hl][c];
        *reinterpret_cast<uint4 *>(&sW[st][hl][r][kc]) = rw[hl][c];
      }
    }
  };

  fetch(0);
  stash(0);
  __syncthreads();
  const int fr = lane & 15, fk = (lane >> 4) * 8;
  int st = 0;
  for (int k0 = 0; k0 < KP; k0 += TK) {
    const bool more = k0 + TK < KP;
    if (more) fetch(k0 + TK);  // in flight while this step multiplies
    // fragments: A[row = l%16][k = 8*(l/16) + 0..7], B[k = 8*(l/16) + 0..7][col = l%16]
    bf16x8 bh[4], bl[4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
      bh[j] = *reinterpret_cast<const bf16x8 *>(&sW[st][0][wn + 16 * j + fr][fk]);
      bl[j] = *reinterpret_cast<const bf16x8 *>(&sW[st][1][wn + 16 * j + fr][fk]);
    }
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const bf16x8 ah = *reinterpret_cast<const bf16x8 *>(&sA[st][0][wm + 16 * i + fr][fk]);
      const bf16x8 al = *reinterpret_cast<const bf16x8 *>(&sA[st][1][wm + 16 * i + fr][fk]);
#pragma unroll
      for (int j = 0; j < 4; j++) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[j], acc[i][j], 0, 0, 0);
      }
    }
    if (more) {
      stash(st ^ 1);  // the other buffer: last read before the previous barrier
      __syncthreads();
      st ^= 1;
    }
  }
  // D[row = 4*(l/16) + r][col = l%16]
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int col = n0 + wn + 16 * j + (lane & 15);
      if (col >= ncol2) continue;
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int64_t s = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        if (s < ns) X[s * ncol2 + col] = acc[i][j][r];
      }
    }
}

// W'[2c + part][kk'] from Wt[kk][c] (complex), split into bf16 hi/lo, K
// extent padded with zeros to KP.
__global__ void split_w_kernel(int K, int KP, int ncol, const double2 *__restrict__ wt, __bf16 *__restrict__ whi,
                               __bf16 *__restrict__ wlo) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)KP * 2 * ncol;
  if (i >= total) return;
  const int64_t col2 = i / KP, kk2 = i - col2 * KP;
  __bf16 h = (__bf16)0.f, l = (__bf16)0.f;
  if (kk2 < 2 * K) {
    const int c = (int)(col2 / 2), part = (int)(col2 & 1);
    const int kk = (int)(kk2 < K ? kk2 : kk2 - K);
    const double2 w = wt[(size_t)kk * ncol + c];
    double v;
    if (part == 0) v = kk2 < K ? w.x : -w.y;
    else v = kk2 < K ? w.y : w.x;
    split_bf16((float)v, h, l);
  }
  whi[i] = h;
  wlo[i] = l;
}

}  // namespace

size_t bf16_w_elems(int nre, int nw, int ncol) { return (size_t)padk(2 * nre * nw) * 2 * ncol; }

size_t bf16_a_elems(int nre, int nw) { return (size_t)padk(2 * nre * nw); }

hipError_t launch_split_bf16(int nre, int nw, int ncol, const double2 *wt, void *out, hipStream_t st) {
  const int K = nre * nw, KP = padk(2 * K);
  const size_t n = bf16_w_elems(nre, nw, ncol);
  __bf16 *whi = static_cast<__bf16 *>(out), *wlo = whi + n;
  hipLaunchKernelGGL(split_w_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, K, KP, ncol, wt, whi, wlo);
  return hipGetLastError();
}

hipError_t launch_xform_bf16x3(int64_t ns, const int32_t *sk, const int32_t *sn, int N, int nw, int nre,
                               const int *re, int ncol, const void *wbf, void *abf, const double2 *evec,
                               const double2 *tab, float2 *X, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  const int K = nre * nw, KP = padk(2 * K), ncol2 = 2 * ncol;
  const size_t nw_el = bf16_w_elems(nre, nw, ncol);
  const __bf16 *whi = static_cast<const __bf16 *>(wbf), *wlo = whi + nw_el;
  __bf16 *ahi = static_cast<__bf16 *>(abf), *alo = ahi + (size_t)ns * KP;
  const int64_t na = ns * KP;
  hipLaunchKernelGGL(state_operand_kernel, dim3((unsigned)((na + 255) / 256)), dim3(256), 0, st, ns, sk, sn, N, nw,
                     K, KP, re, evec, tab, ahi, alo);
  const int tiles_m = (int)((ns + TM - 1) / TM), tiles_n = (ncol2 + TN - 1) / TN;
  const int64_t ntile = (int64_t)tiles_m * tiles_n;
  const int64_t grid = (ntile + 7) / 8 * 8;
  const int sh = (int)(sizeof(__bf16) * 2 * 2 * (TM + TN) * LDR);
  hipError_t e = hipFuncSetAttribute((const void *)xform_bf16x3_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, sh);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(xform_bf16x3_kernel, dim3((unsigned)grid), dim3(256), sh, st, ns, ncol2, KP, ahi, alo, whi, wlo,
                     reinterpret_cast<float *>(X), tiles_m, tiles_n);
  return hipGetLastError();
}

}  // namespace eph
