// Small device helpers: fills, a max reduction and the per-call count
// summary (gfx950).  Fills use a kernel rather than hipMemsetAsync so the
// library never records memset nodes if a caller captures its stream.
#include "internal.h"

namespace eph {
namespace {

__global__ void zero_kernel(int64_t n64, unsigned long long *__restrict__ p) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n64) p[i] = 0ull;
}

// max of non-negative doubles through their (monotone) bit patterns
__global__ void max_nonneg_kernel(int64_t n, const double *__restrict__ x, unsigned long long *__restrict__ out) {
  __shared__ unsigned long long red[256];
  unsigned long long m = 0ull;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v = x[i];
    if (v > 0.0) {
      unsigned long long b = (unsigned long long)__double_as_longlong(v);
      m = b > m ? b : m;
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + s] ? red[threadIdx.x] : red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(out, red[0]);
}

// out[0] += sum n_q_valid, out[1] += sum n_terms, out[2] += #(inv_tau[0][s] == 0)
__global__ void summarize_kernel(int64_t ns, const int64_t *__restrict__ st_counts,
                                 const double *__restrict__ inv_tau0, unsigned long long *__restrict__ out) {
  __shared__ unsigned long long red[3][256];
  unsigned long long a = 0, b = 0, c = 0;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < ns; s += (int64_t)gridDim.x * blockDim.x) {
    a += (unsigned long long)st_counts[2 * s];
    b += (unsigned long long)st_counts[2 * s + 1];
    c += inv_tau0[s] == 0.0 ? 1ull : 0ull;
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int q = 0; q < 3; q++) red[q][threadIdx.x] += red[q][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x < 3) atomicAdd(out + threadIdx.x, red[threadIdx.x][0]);
}

struct Kts {
  double v[EPH_MAX_TEMPS];
};

__global__ void occupation_kernel(int64_t nq, int nw, int nm, const double *__restrict__ eps,
                                  const double *__restrict__ om, double mu, int nt, Kts kts, double wcut,
                                  double *__restrict__ occ_f, double *__restrict__ occ_n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  // rows padded to EPH_MAX_TEMPS entries (zeros past nt) for vector loads
  if (i < nq * nw) {
    const double e = eps[i];
    for (int t = 0; t < EPH_MAX_TEMPS; t++)
      occ_f[i * EPH_MAX_TEMPS + t] = t < nt ? 1.0 / (exp((e - mu) / kts.v[t]) + 1.0) : 0.0;
  }
  if (i < nq * nm) {
    const double w = om[i];
    for (int t = 0; t < EPH_MAX_TEMPS; t++)
      occ_n[i * EPH_MAX_TEMPS + t] = (t < nt && w >= wcut && w > 0.0) ? 1.0 / expm1(w / kts.v[t]) : 0.0;
  }
}

}  // namespace

hipError_t launch_occupations(int64_t nq, int nw, int nm, const double *eps, const double *om, double mu, int nt,
                              const double *kts_host, double wcut, double *occ_f, double *occ_n, hipStream_t st) {
  Kts k;
  for (int t = 0; t < EPH_MAX_TEMPS; t++) k.v[t] = t < nt ? kts_host[t] : 1.0;
  const int64_t n = nq * (nw > nm ? nw : nm);
  hipLaunchKernelGGL(occupation_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, nq, nw, nm, eps, om,
                     mu, nt, k, wcut, occ_f, occ_n);
  return hipGetLastError();
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t st) {
  int64_t n64 = (int64_t)((bytes + 7) / 8);
  if (n64 <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n64 + 255) / 256)), dim3(256), 0, st, n64,
                     static_cast<unsigned long long *>(p));
  return hipGetLastError();
}

hipError_t launch_max_nonneg(int64_t n, const double *x, unsigned long long *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(max_nonneg_kernel, dim3((unsigned)blocks), dim3(256), 0, st, n, x, out);
  return hipGetLastError();
}

hipError_t launch_summarize(int64_t ns, const int64_t *st_counts, const double *inv_tau0, unsigned long long *out,
                            hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  int64_t blocks = (ns + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(summarize_kernel, dim3((unsigned)blocks), dim3(256), 0, st, ns, st_counts, inv_tau0, out);
  return hipGetLastError();
}

}  // namespace eph
