// Conductivity reduction and its energy moments (Sec. II.C), the carrier
// density, and small element-wise helpers (gfx950).
//
// M_n,ab(T) = 2 e^2/(N_k V) sum_s v_a v_b tau_s f(1-f)/(k_B T) (eps_s - mu)^n
// (n = 0 is sigma; eps in eV), or with v_b tau_s replaced by the mean free
// path F_b of the iterative solution: each block reduces a contiguous chunk of
// states with Neumaier-compensated per-thread sums and a fixed butterfly,
// writing [block][T][9] partials; a one-block kernel then adds the partials
// in block order and applies the prefactor.  The carrier density sums f over
// the bands of the full grid the same way.  Results are bit-identical from
// run to run.
#include "internal.h"

namespace eph {
namespace {

constexpr int kSigThreads = 256;

__device__ __forceinline__ void neumaier(double &s, double &c, double x) {
  double t = s + x;
  if (fabs(s) >= fabs(x)) c += (s - t) + x;
  else c += (x - t) + s;
  s = t;
}

__global__ __launch_bounds__(kSigThreads) void sigma_kernel(int64_t ns, const double *__restrict__ e,
                                                             const double *__restrict__ v,
                                                             const double *__restrict__ inv_tau, double mu, int nt,
                                                             const double *__restrict__ kts,
                                                             double *__restrict__ partials, int64_t chunk,
                                                             int order, const double *__restrict__ F) {
  __shared__ double red[kSigThreads / 64][EPH_MAX_TEMPS * 9];
  const int64_t b0 = blockIdx.x * chunk, b1 = min(ns, b0 + chunk);
  double s[EPH_MAX_TEMPS][9], c[EPH_MAX_TEMPS][9];
  for (int t = 0; t < EPH_MAX_TEMPS; t++)
    for (int q = 0; q < 9; q++) s[t][q] = c[t][q] = 0.0;
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kSigThreads) {
    const double vx = v[3 * i], vy = v[3 * i + 1], vz = v[3 * i + 2];
    const double vv[9] = {vx * vx, vx * vy, vx * vz, vy * vx, vy * vy, vy * vz, vz * vx, vz * vy, vz * vz};
    for (int t = 0; t < EPH_MAX_TEMPS; t++) {
      if (t >= nt) break;
      const double it = inv_tau[t * ns + i];
      if (it == 0.0) continue;
      const double kt = kts[t];
      const double f = 1.0 / (exp((e[i] - mu) / kt) + 1.0);
      const double de = e[i] - mu;
      if (F) {  // mean free paths of the iterative solution: v_a F_b in place of v_a v_b tau
        const double *fb = F + ((int64_t)t * ns + i) * 3;
        const double w = f * (1.0 - f) / kt * (order == 0 ? 1.0 : order == 1 ? de : de * de);
        const double vf[9] = {vx * fb[0], vx * fb[1], vx * fb[2], vy * fb[0], vy * fb[1],
                              vy * fb[2], vz * fb[0], vz * fb[1], vz * fb[2]};
        for (int q = 0; q < 9; q++) neumaier(s[t][q], c[t][q], vf[q] * w);
        continue;
      }
      const double w = f * (1.0 - f) / kt / it * (order == 0 ? 1.0 : order == 1 ? de : de * de);
      for (int q = 0; q < 9; q++) neumaier(s[t][q], c[t][q], vv[q] * w);
    }
  }
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  for (int t = 0; t < EPH_MAX_TEMPS; t++)
    for (int q = 0; q < 9; q++) {
      double x = s[t][q] + c[t][q];
      for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
      if (lane == 0) red[wave][t * 9 + q] = x;
    }
  __syncthreads();
  if (threadIdx.x < EPH_MAX_TEMPS * 9) {
    double x = 0.0;
    for (int w = 0; w < kSigThreads / 64; w++) x += red[w][threadIdx.x];
    partials[blockIdx.x * EPH_MAX_TEMPS * 9 + threadIdx.x] = x;
  }
}

__global__ void sigma_final_kernel(int nblk, const double *__restrict__ partials, double pref,
                                   double *__restrict__ out) {
  const int q = threadIdx.x;
  if (q >= EPH_MAX_TEMPS * 9) return;
  double s = 0.0, c = 0.0;
  for (int b = 0; b < nblk; b++) neumaier(s, c, partials[b * EPH_MAX_TEMPS * 9 + q]);
  out[q] = pref * (s + c);
}

// sum over k of f(eps_nk) for band_lo <= n <= band_hi, per temperature
__global__ __launch_bounds__(kSigThreads) void density_kernel(int64_t nk, int nw, const double *__restrict__ eps,
                                                               int blo, int bhi, double mu, int nt,
                                                               const double *__restrict__ kts,
                                                               double *__restrict__ partials, int64_t chunk) {
  __shared__ double red[kSigThreads / 64][EPH_MAX_TEMPS];
  const int64_t b0 = blockIdx.x * chunk, b1 = min(nk, b0 + chunk);
  double s[EPH_MAX_TEMPS], c[EPH_MAX_TEMPS];
  for (int t = 0; t < EPH_MAX_TEMPS; t++) s[t] = c[t] = 0.0;
  for (int64_t k = b0 + threadIdx.x; k < b1; k += kSigThreads)
    for (int n = blo; n <= bhi; n++) {
      const double e = eps[k * nw + n];
      for (int t = 0; t < EPH_MAX_TEMPS; t++) {
        if (t >= nt) break;
        neumaier(s[t], c[t], 1.0 / (exp((e - mu) / kts[t]) + 1.0));
      }
    }
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  for (int t = 0; t < EPH_MAX_TEMPS; t++) {
    double x = s[t] + c[t];
    for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
    if (lane == 0) red[wave][t] = x;
  }
  __syncthreads();
  if (threadIdx.x < EPH_MAX_TEMPS) {
    double x = 0.0;
    for (int w = 0; w < kSigThreads / 64; w++) x += red[w][threadIdx.x];
    partials[blockIdx.x * EPH_MAX_TEMPS + threadIdx.x] = x;
  }
}

__global__ void density_final_kernel(int nblk, const double *__restrict__ partials, double pref,
                                     double *__restrict__ out) {
  const int t = threadIdx.x;
  if (t >= EPH_MAX_TEMPS) return;
  double s = 0.0, c = 0.0;
  for (int b = 0; b < nblk; b++) neumaier(s, c, partials[b * EPH_MAX_TEMPS + t]);
  out[t] = pref * (s + c);
}

__global__ void real_to_f32_kernel(int64_t n, const double *__restrict__ in, float *__restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = (float)in[i];
}

__global__ void to_f32_kernel(int64_t n, const double2 *__restrict__ in, float2 *__restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = make_float2((float)in[i].x, (float)in[i].y);
}

}  // namespace

hipError_t launch_sigma(int64_t ns, const double *e, const double *v, const double *inv_tau, double mu, int nt,
                        const double *kts, double pref, double *partials, int nblk, double *out,
                        hipStream_t st, int order, const double *F) {
  int64_t chunk = (ns + nblk - 1) / nblk;
  if (chunk < 1) chunk = 1;
  hipLaunchKernelGGL(sigma_kernel, dim3(nblk), dim3(kSigThreads), 0, st, ns, e, v, inv_tau, mu, nt, kts, partials,
                     chunk, order, F);
  hipLaunchKernelGGL(sigma_final_kernel, dim3(1), dim3(64), 0, st, nblk, partials, pref, out);
  return hipGetLastError();
}

hipError_t launch_density(int64_t nk, int nw, const double *eps, int blo, int bhi, double mu, int nt,
                          const double *kts, double pref, double *partials, int nblk, double *out, hipStream_t st) {
  int64_t chunk = (nk + nblk - 1) / nblk;
  if (chunk < 1) chunk = 1;
  hipLaunchKernelGGL(density_kernel, dim3(nblk), dim3(kSigThreads), 0, st, nk, nw, eps, blo, bhi, mu, nt, kts,
                     partials, chunk);
  hipLaunchKernelGGL(density_final_kernel, dim3(1), dim3(64), 0, st, nblk, partials, pref, out);
  return hipGetLastError();
}

hipError_t launch_real_to_f32(int64_t n, const double *in, float *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(real_to_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, in, out);
  return hipGetLastError();
}

hipError_t launch_to_f32(int64_t n, const double2 *in, float2 *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(to_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, in, out);
  return hipGetLastError();
}

}  // namespace eph
