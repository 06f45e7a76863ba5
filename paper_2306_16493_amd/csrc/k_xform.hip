// Re transform fused with the j -> n band rotation (gfx950):
//   X_s(Rp, mu, i) = sum_{Re, j} g_ij^mu(Re, Rp) e^{i k_s.Re} V_{j n_s}(k_s)
// i.e. the innermost bracket (g P^el(k) U^+(k)) of the q-batch order of
// Sec. III.C, evaluated per initial state s = (n, k).  It is a complex GEMM
// X[s][col] = sum_kk B[s][kk] W[kk][col] with kk = (Re, j) and
// col = (Rp, mu, i); the state-side operand B (a phase times one
// eigenvector component) is generated on the fly into LDS.
#include "dev_util.h"
#include "internal.h"

namespace eph {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// T = accumulation/operand type (double for the FP64 form, float for FP32).
template <class T>
__global__ __launch_bounds__(256) void xform_kernel(int64_t ns, const int32_t *__restrict__ sk,
                                                    const int32_t *__restrict__ sn, int N, int nw, int nre,
                                                    const int *__restrict__ re, int ncol,
                                                    const typename V2<T>::t *__restrict__ wt,
                                                    const double2 *__restrict__ evec,
                                                    const double2 *__restrict__ tab,
                                                    typename V2<T>::t *__restrict__ X) {
  using C2 = typename V2<T>::t;
  __shared__ C2 sB[BM][BK + 1];
  __shared__ C2 sW[BK][BN];
  const int tid = threadIdx.x;
  const int tx = tid % 16, ty = tid / 16;
  const int64_t s0 = (int64_t)blockIdx.y * BM;
  const int c0 = blockIdx.x * BN;
  const int K = nre * nw;
  C2 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; r++)
#pragma unroll
    for (int c = 0; c < 4; c++) acc[r][c] = mk<T>(0, 0);

  for (int kk0 = 0; kk0 < K; kk0 += BK) {
    // state-side operand: phase(k_s, Re) * V_{j n_s}(k_s)
    for (int t = tid; t < BM * BK; t += 256) {
      int sl = t / BK, kl = t % BK;
      int64_t s = s0 + sl;
      int kk = kk0 + kl;
      double2 v = make_double2(0.0, 0.0);  // phase and eigenvector product in FP64, then T
      if (s < ns && kk < K) {
        int64_t k = sk[s];
        int n = sn[s];
        int r = kk / nw, j = kk % nw;
        int64_t k1 = k % N, k2 = (k / N) % N, k3 = k / ((int64_t)N * N);
        int64_t ph = (k1 * re[3 * r] + k2 * re[3 * r + 1] + k3 * re[3 * r + 2]) % N;
        if (ph < 0) ph += N;
        v = cmul(tab[ph], evec[(k * nw + n) * nw + j]);
      }
      sB[sl][kl] = mk<T>((T)v.x, (T)v.y);
    }
    for (int t = tid; t < BK * BN; t += 256) {
      int kl = t / BN, cl = t % BN;
      int kk = kk0 + kl, c = c0 + cl;
      sW[kl][cl] = (kk < K && c < ncol) ? wt[(size_t)kk * ncol + c] : mk<T>(0, 0);
    }
    __syncthreads();
#pragma unroll 4
    for (int kl = 0; kl < BK; kl++) {
      C2 a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; r++) a[r] = sB[ty * 4 + r][kl];
#pragma unroll
      for (int c = 0; c < 4; c++) b[c] = sW[kl][tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; r++)
#pragma unroll
        for (int c = 0; c < 4; c++) {
          acc[r][c].x = fma(a[r].x, b[c].x, acc[r][c].x);
          acc[r][c].x = fma(-a[r].y, b[c].y, acc[r][c].x);
          acc[r][c].y = fma(a[r].x, b[c].y, acc[r][c].y);
          acc[r][c].y = fma(a[r].y, b[c].x, acc[r][c].y);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; r++) {
    int64_t s = s0 + ty * 4 + r;
    if (s >= ns) continue;
#pragma unroll
    for (int c = 0; c < 4; c++) {
      int col = c0 + tx + 16 * c;
      if (col < ncol) X[s * ncol + col] = acc[r][c];
    }
  }
}

}  // namespace

hipError_t launch_xform64(int64_t ns, const int32_t *sk, const int32_t *sn, int N, int nw, int nre, const int *re,
                          int ncol, const double2 *wt, const double2 *evec, const double2 *tab, double2 *X,
                          hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  dim3 grid((ncol + BN - 1) / BN, (unsigned)((ns + BM - 1) / BM));
  hipLaunchKernelGGL(xform_kernel<double>, grid, dim3(256), 0, st, ns, sk, sn, N, nw, nre, re, ncol, wt, evec,
                     tab, X);
  return hipGetLastError();
}

hipError_t launch_xform32(int64_t ns, const int32_t *sk, const int32_t *sn, int N, int nw, int nre, const int *re,
                          int ncol, const float2 *wt, const double2 *evec, const double2 *tab, float2 *X,
                          hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  dim3 grid((ncol + BN - 1) / BN, (unsigned)((ns + BM - 1) / BM));
  hipLaunchKernelGGL(xform_kernel<float>, grid, dim3(256), 0, st, ns, sk, sn, N, nw, nre, re, ncol, wt, evec,
                     tab, X);
  return hipGetLastError();
}

}  // namespace eph
