// Iterative solution of the linearised BTE (Sec. II.C, iteration equation;
// Sec. III.E, the transition rates stored row by row) on gfx950:
//   * the state-index table (k, m) -> position in the state list, which the
//     rate kernel uses to keep only transition rates to listed final states;
//   * F0 = v tau;
//   * one iteration step F_new = F0 + tau sum_e Gamma_e F_old[col_e] per
//     row (state), one wave per row with a fixed-order reduction, so
//     results are bit-identical from run to run; rows can be processed in
//     batches whose entries sit in a staging buffer (Gamma spilled to host).
// The step is bound by HBM: per entry it reads a 4-byte column index and
// an 8-byte value and gathers 24 bytes of F (from L2 for most entries).
#include "internal.h"

namespace eph {
namespace {

__global__ void fill_i32_kernel(int64_t n, int32_t v, int32_t *__restrict__ p) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void state_index_kernel(int64_t ns, int nw, const int32_t *__restrict__ sk, const int32_t *__restrict__ sn,
                                   int32_t *__restrict__ stidx) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s < ns) stidx[(int64_t)sk[s] * nw + sn[s]] = (int32_t)s;
}

// F0[t][s][a] = v[s][a] / inv_tau[t][s] (0 where inv_tau = 0)
__global__ void f0_kernel(int64_t ns, int nt, const double *__restrict__ vel, const double *__restrict__ inv_tau,
                          double *__restrict__ F0) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= ns * nt) return;
  const int64_t t = i / ns, s = i % ns;
  const double it = inv_tau[t * ns + s];
  for (int a = 0; a < 3; a++) F0[(t * ns + s) * 3 + a] = it == 0.0 ? 0.0 : vel[s * 3 + a] / it;
}

// rows r0..r1-1; entry e of row s sits at e - base of col / val
__global__ __launch_bounds__(256) void bte_step_kernel(int64_t r0, int64_t r1, const int64_t *__restrict__ row_start,
                                                       int64_t base, const int32_t *__restrict__ col,
                                                       const double *__restrict__ val,
                                                       const double *__restrict__ inv_tau,
                                                       const double *__restrict__ F0, const double *__restrict__ Fin,
                                                       double *__restrict__ Fout) {
  const int lane = threadIdx.x & 63;
  const int64_t s = r0 + (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (s >= r1) return;  // wave-uniform
  const int64_t e0 = row_start[s] - base, e1 = row_start[s + 1] - base;
  double ax = 0.0, ay = 0.0, az = 0.0;
  for (int64_t e = e0 + lane; e < e1; e += 64) {
    const double g = val[e];
    const double *f = Fin + (int64_t)col[e] * 3;
    ax = fma(g, f[0], ax);
    ay = fma(g, f[1], ay);
    az = fma(g, f[2], az);
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    ax += __shfl_xor(ax, m, 64);
    ay += __shfl_xor(ay, m, 64);
    az += __shfl_xor(az, m, 64);
  }
  if (lane == 0) {
    const double it = inv_tau[s];
    double *o = Fout + s * 3;
    const double *f0 = F0 + s * 3;
    o[0] = it == 0.0 ? 0.0 : f0[0] + ax / it;
    o[1] = it == 0.0 ? 0.0 : f0[1] + ay / it;
    o[2] = it == 0.0 ? 0.0 : f0[2] + az / it;
  }
}

// number of states whose emitted entries do not end at the next row's start
__global__ void check_rows_kernel(int64_t ns, const int64_t *__restrict__ cursor, const int64_t *__restrict__ row_start,
                                  unsigned long long *__restrict__ bad) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s < ns && cursor[s] != row_start[s + 1]) atomicAdd(bad, 1ull);
}

}  // namespace

hipError_t launch_state_index(int64_t nq, int nw, int64_t ns, const int32_t *sk, const int32_t *sn, int32_t *stidx,
                              hipStream_t st) {
  const int64_t n = nq * nw;
  if (n > 0) hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, -1, stidx);
  if (ns > 0)
    hipLaunchKernelGGL(state_index_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, ns, nw, sk, sn, stidx);
  return hipGetLastError();
}

hipError_t launch_f0(int64_t ns, int nt, const double *vel, const double *inv_tau, double *F0, hipStream_t st) {
  if (ns * nt <= 0) return hipSuccess;
  hipLaunchKernelGGL(f0_kernel, dim3((unsigned)((ns * nt + 255) / 256)), dim3(256), 0, st, ns, nt, vel, inv_tau, F0);
  return hipGetLastError();
}

hipError_t launch_bte_step(int64_t r0, int64_t r1, const int64_t *row_start, int64_t base, const int32_t *col,
                           const double *val, const double *inv_tau, const double *F0, const double *Fin, double *Fout,
                           hipStream_t st) {
  if (r1 <= r0) return hipSuccess;
  const int64_t nb = (r1 - r0 + 3) / 4;
  hipLaunchKernelGGL(bte_step_kernel, dim3((unsigned)nb), dim3(256), 0, st, r0, r1, row_start, base, col, val, inv_tau,
                     F0, Fin, Fout);
  return hipGetLastError();
}

hipError_t launch_check_rows(int64_t ns, const int64_t *cursor, const int64_t *row_start, unsigned long long *bad,
                             hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(check_rows_kernel, dim3((unsigned)((ns + 255) / 256)), dim3(256), 0, st, ns, cursor, row_start,
                     bad);
  return hipGetLastError();
}

}  // namespace eph
