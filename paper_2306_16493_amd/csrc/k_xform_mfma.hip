// Re transform fused with the j -> n rotation on bf16 MFMA with a split
// (x = hi + lo) and three products hi*hi + hi*lo + lo*hi accumulated in FP32
// (the reduced-precision form of the Re -> k step; gfx950).
//
// Real formulation of the complex GEMM X[s][c] = sum_kk B[s][kk] W[kk][c]:
//   A[s][kk']  = Re B (kk' < K) | Im B (kk' >= K)                 (M x 2K)
//   W'[2c  ][kk'] = Re W[kk][c] (kk' < K) | -Im W[kk][c]          (stored
//   W'[2c+1][kk'] = Im W[kk][c] (kk' < K) |  Re W[kk][c]           column-major)
// so that X'[s][2c] = Re X and X'[s][2c+1] = Im X, i.e. X' is X as
// interleaved (re, im) floats.  W' is split into bf16 hi/lo once per
// context; A is generated in FP64 (phase times eigenvector), rounded to FP32
// and split on the fly.
//
// Tiling: a 256-thread workgroup computes a 64 (states) x 64 (real columns)
// tile; each wave64 a 32 x 32 quarter as 2 x 2 tiles of
// v_mfma_f32_16x16x32_bf16, K advancing 32 per step through LDS.
#include "dev_util.h"
#include "internal.h"

namespace eph {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int TM = 64, TN = 64, TK = 32;

__device__ __forceinline__ void split_bf16(float x, __bf16 &hi, __bf16 &lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

__global__ __launch_bounds__(256) void xform_bf16x3_kernel(int64_t ns, const int32_t *__restrict__ sk,
                                                           const int32_t *__restrict__ sn, int N, int nw, int nre,
                                                           const int *__restrict__ re, int ncol2, int K2,
                                                           const __bf16 *__restrict__ whi,
                                                           const __bf16 *__restrict__ wlo,
                                                           const double2 *__restrict__ evec,
                                                           const double2 *__restrict__ tab, float *__restrict__ X) {
  // LDS: A hi/lo [TM][TK], W hi/lo [TN][TK] (k contiguous, 16-byte rows of 8)
  __shared__ __align__(16) __bf16 sAh[TM][TK];
  __shared__ __align__(16) __bf16 sAl[TM][TK];
  __shared__ __align__(16) __bf16 sWh[TN][TK];
  __shared__ __align__(16) __bf16 sWl[TN][TK];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t m0 = (int64_t)blockIdx.y * TM;
  const int n0 = blockIdx.x * TN;
  const int K = K2 / 2;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  floatx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < K2; k0 += TK) {
    // A tile: 64 x 32 elements, 8 per thread
    for (int t = tid; t < TM * TK; t += 256) {
      const int r = t / TK, kk2 = k0 + t % TK;
      const int64_t s = m0 + r;
      float v = 0.f;
      if (s < ns && kk2 < K2) {
        const int kk = kk2 < K ? kk2 : kk2 - K;
        const int64_t k = sk[s];
        const int n = sn[s];
        const int ir = kk / nw, j = kk - (kk / nw) * nw;
        const int64_t k1 = k % N, kb = (k / N) % N, k3 = k / ((int64_t)N * N);
        int64_t ph = (k1 * re[3 * ir] + kb * re[3 * ir + 1] + k3 * re[3 * ir + 2]) % N;
        if (ph < 0) ph += N;
        const double2 p = tab[ph], e = evec[(k * nw + n) * nw + j];
        v = (float)(kk2 < K ? p.x * e.x - p.y * e.y : p.x * e.y + p.y * e.x);
      }
      __bf16 h, l;
      split_bf16(v, h, l);
      sAh[r][t % TK] = h;
      sAl[r][t % TK] = l;
    }
    // W tile: rows n0..n0+63 of W' (column-major), k0..k0+31
    for (int t = tid; t < TN * TK; t += 256) {
      const int c = t / TK, kk2 = k0 + t % TK;
      const int col = n0 + c;
      __bf16 h = (__bf16)0.f, l = (__bf16)0.f;
      if (col < ncol2 && kk2 < K2) {
        h = whi[(size_t)col * K2 + kk2];
        l = wlo[(size_t)col * K2 + kk2];
      }
      sWh[c][t % TK] = h;
      sWl[c][t % TK] = l;
    }
    __syncthreads();
    // fragments: A[row = l%16][k = 8*(l/16) + 0..7], B[k = 8*(l/16) + 0..7][col = l%16]
    const int fr = lane & 15, fk = (lane >> 4) * 8;
    bf16x8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; i++) {
      ah[i] = *reinterpret_cast<const bf16x8 *>(&sAh[wm + 16 * i + fr][fk]);
      al[i] = *reinterpret_cast<const bf16x8 *>(&sAl[wm + 16 * i + fr][fk]);
      bh[i] = *reinterpret_cast<const bf16x8 *>(&sWh[wn + 16 * i + fr][fk]);
      bl[i] = *reinterpret_cast<const bf16x8 *>(&sWl[wn + 16 * i + fr][fk]);
    }
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
      for (int j = 0; j < 2; j++) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
      }
    __syncthreads();
  }
  // D[row = 4*(l/16) + r][col = l%16]
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int64_t s = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int col = n0 + wn + 16 * j + (lane & 15);
        if (s < ns && col < ncol2) X[s * ncol2 + col] = acc[i][j][r];
      }
}

// W'[2c + part][kk'] from Wt[kk][c] (complex), split into bf16 hi/lo.
__global__ void split_w_kernel(int K, int ncol, const double2 *__restrict__ wt, __bf16 *__restrict__ whi,
                               __bf16 *__restrict__ wlo) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t K2 = 2 * (int64_t)K, total = K2 * 2 * ncol;
  if (i >= total) return;
  const int64_t col2 = i / K2, kk2 = i - col2 * K2;
  const int c = (int)(col2 / 2), part = (int)(col2 & 1);
  const int kk = (int)(kk2 < K ? kk2 : kk2 - K);
  const double2 w = wt[(size_t)kk * ncol + c];
  double v;
  if (part == 0) v = kk2 < K ? w.x : -w.y;
  else v = kk2 < K ? w.y : w.x;
  const float f = (float)v;
  __bf16 h, l;
  split_bf16(f, h, l);
  whi[i] = h;
  wlo[i] = l;
}

}  // namespace

size_t bf16_w_elems(int nre, int nw, int ncol) { return (size_t)2 * nre * nw * 2 * ncol; }

hipError_t launch_split_bf16(int nre, int nw, int ncol, const double2 *wt, void *out, hipStream_t st) {
  const int K = nre * nw;
  const size_t n = bf16_w_elems(nre, nw, ncol);
  __bf16 *whi = static_cast<__bf16 *>(out), *wlo = whi + n;
  hipLaunchKernelGGL(split_w_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, K, ncol, wt, whi, wlo);
  return hipGetLastError();
}

hipError_t launch_xform_bf16x3(int64_t ns, const int32_t *sk, const int32_t *sn, int N, int nw, int nre,
                               const int *re, int ncol, const void *wbf, const double2 *evec, const double2 *tab,
                               float2 *X, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  const int K2 = 2 * nre * nw, ncol2 = 2 * ncol;
  const size_t n = bf16_w_elems(nre, nw, ncol);
  const __bf16 *whi = static_cast<const __bf16 *>(wbf), *wlo = whi + n;
  dim3 grid((ncol2 + TN - 1) / TN, (unsigned)((ns + TM - 1) / TM));
  hipLaunchKernelGGL(xform_bf16x3_kernel, grid, dim3(256), 0, st, ns, sk, sn, N, nw, nre, re, ncol2, K2, whi, wlo,
                     evec, tab, reinterpret_cast<float *>(X));
  return hipGetLastError();
}

}  // namespace eph
