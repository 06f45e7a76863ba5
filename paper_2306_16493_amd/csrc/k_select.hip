// Preprocessing on the grid tables (gfx950): selection of the initial states
// in the energy window (the effective states of Sec. III.A), prefix sums,
// grouping of states by k-line, and energy-sorted p-lines that turn the
// energy-conservation sieve (Sec. III.A) into a range search.
#include "internal.h"

namespace eph {
namespace {

constexpr int kScanBlock = 1024;

__global__ void count_states_kernel(int64_t nklist, const int64_t *__restrict__ klist, int nw,
                                    const double *__restrict__ eps, int blo, int bhi, double wlo, double whi,
                                    int64_t *__restrict__ cnt) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nklist) return;
  int64_t k = klist ? klist[t] : t;
  int c = 0;
  for (int n = blo; n <= bhi; n++) {
    double e = eps[k * nw + n];
    c += (e >= wlo && e <= whi);
  }
  cnt[t] = c;
}

__global__ void write_states_kernel(int64_t nklist, const int64_t *__restrict__ klist, int nw,
                                    const double *__restrict__ eps, const double *__restrict__ vel, int blo,
                                    int bhi, double wlo, double whi, const int64_t *__restrict__ offs,
                                    int32_t *__restrict__ sk, int32_t *__restrict__ sn, double *__restrict__ se,
                                    double *__restrict__ sv) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= nklist) return;
  int64_t k = klist ? klist[t] : t;
  int64_t o = offs[t];
  for (int n = blo; n <= bhi; n++) {
    double e = eps[k * nw + n];
    if (e >= wlo && e <= whi) {
      sk[o] = (int32_t)k;
      sn[o] = n;
      se[o] = e;
      sv[3 * o] = vel[(k * nw + n) * 3];
      sv[3 * o + 1] = vel[(k * nw + n) * 3 + 1];
      sv[3 * o + 2] = vel[(k * nw + n) * 3 + 2];
      o++;
    }
  }
}

// Block-wise exclusive scan of int64 (Hillis-Steele in LDS), block totals to sums.
__global__ __launch_bounds__(kScanBlock) void scan_block_kernel(int64_t n, const int64_t *__restrict__ in,
                                                                 int64_t *__restrict__ out,
                                                                 int64_t *__restrict__ sums) {
  __shared__ int64_t s[kScanBlock];
  int64_t g = blockIdx.x * (int64_t)kScanBlock + threadIdx.x;
  int64_t v = g < n ? in[g] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    int64_t t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (g < n) out[g] = s[threadIdx.x] - v;
  if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void scan_add_kernel(int64_t n, int64_t *__restrict__ out, const int64_t *__restrict__ sums_excl) {
  int64_t g = blockIdx.x * (int64_t)kScanBlock + threadIdx.x;
  if (g < n) out[g] += sums_excl[blockIdx.x];
}

// First state of each k-line (same i2, i3): binary search in the sorted
// state list; a group starts every gmax states of a line.
__global__ void group_heads_kernel(int64_t ns, const int32_t *__restrict__ sk, int N, int gmax,
                                   int64_t *__restrict__ flag) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= ns) return;
  int32_t line = sk[s] / N;
  int64_t lo = 0, hi = s;  // first index with line(sk[idx]) == line
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (sk[mid] / N < line) lo = mid + 1;
    else hi = mid;
  }
  flag[s] = ((s - lo) % gmax) == 0 ? 1 : 0;
}

__global__ void group_starts_kernel(int64_t ns, const int64_t *__restrict__ flag, const int64_t *__restrict__ pos,
                                    int64_t *__restrict__ gstart) {
  int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s < ns && flag[s]) gstart[pos[s]] = s;
  if (s == ns - 1) gstart[pos[s] + flag[s]] = ns;
}

// One workgroup per p-line; bitonic sort of (eps, key) pairs in LDS.
__global__ __launch_bounds__(256) void line_sort_kernel(int N, int nw, const double *__restrict__ eps,
                                                        double *__restrict__ line_e,
                                                        uint16_t *__restrict__ line_key) {
  extern __shared__ unsigned char smem[];
  const int cnt = N * nw;
  int P = 1;
  while (P < cnt) P <<= 1;
  double *se = reinterpret_cast<double *>(smem);
  uint16_t *sk = reinterpret_cast<uint16_t *>(se + P);
  const int64_t line = blockIdx.x;  // i2 + N*i3
  for (int t = threadIdx.x; t < P; t += blockDim.x) {
    if (t < cnt) {
      int i1 = t / nw, m = t % nw;
      se[t] = eps[(line * N + i1) * nw + m];
      sk[t] = (uint16_t)t;
    } else {
      se[t] = __builtin_huge_val();
      sk[t] = 0xffff;
    }
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int t = threadIdx.x; t < P; t += blockDim.x) {
        int ixj = t ^ jj;
        if (ixj > t) {
          bool up = (t & k) == 0;
          double a = se[t], b = se[ixj];
          uint16_t ka = sk[t], kb = sk[ixj];
          bool gt = (a > b) || (a == b && ka > kb);
          if (gt == up) {
            se[t] = b; se[ixj] = a;
            sk[t] = kb; sk[ixj] = ka;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
    line_e[line * cnt + t] = se[t];
    line_key[line * cnt + t] = sk[t];
  }
}

}  // namespace

size_t scan_tmp_elems(int64_t n) {
  size_t total = 0;
  int64_t m = n;
  while (true) {
    int64_t nb = (m + kScanBlock - 1) / kScanBlock;
    total += 2 * nb + 2;
    if (nb <= 1) break;
    m = nb;
  }
  return total;
}

hipError_t launch_scan(int64_t n, const int64_t *in, int64_t *out_excl, int64_t *tmp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  int64_t *sums = tmp, *sums_ex = tmp + nb + 1;
  hipLaunchKernelGGL(scan_block_kernel, dim3(nb), dim3(kScanBlock), 0, st, n, in, out_excl, sums);
  if (nb > 1) {
    hipError_t e = launch_scan(nb, sums, sums_ex, tmp + 2 * nb + 2, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_add_kernel, dim3(nb), dim3(kScanBlock), 0, st, n, out_excl, sums_ex);
  }
  return hipGetLastError();
}

hipError_t launch_count_states(int64_t nklist, const int64_t *klist, int nw, const double *eps, int blo, int bhi,
                               double wlo, double whi, int64_t *cnt, hipStream_t st) {
  if (nklist <= 0) return hipSuccess;
  hipLaunchKernelGGL(count_states_kernel, dim3((nklist + 255) / 256), dim3(256), 0, st, nklist, klist, nw, eps,
                     blo, bhi, wlo, whi, cnt);
  return hipGetLastError();
}

hipError_t launch_write_states(int64_t nklist, const int64_t *klist, int nw, const double *eps, const double *vel,
                               int blo, int bhi, double wlo, double whi, const int64_t *offs, int32_t *sk,
                               int32_t *sn, double *se, double *sv, hipStream_t st) {
  if (nklist <= 0) return hipSuccess;
  hipLaunchKernelGGL(write_states_kernel, dim3((nklist + 255) / 256), dim3(256), 0, st, nklist, klist, nw, eps,
                     vel, blo, bhi, wlo, whi, offs, sk, sn, se, sv);
  return hipGetLastError();
}

hipError_t launch_group_heads(int64_t ns, const int32_t *sk, int N, int gmax, int64_t *flag, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(group_heads_kernel, dim3((ns + 255) / 256), dim3(256), 0, st, ns, sk, N, gmax, flag);
  return hipGetLastError();
}

hipError_t launch_group_starts(int64_t ns, const int64_t *flag, const int64_t *pos, int64_t *gstart,
                               hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(group_starts_kernel, dim3((ns + 255) / 256), dim3(256), 0, st, ns, flag, pos, gstart);
  return hipGetLastError();
}

hipError_t launch_line_sort(int N, int nw, const double *eps, double *line_e, uint16_t *line_key,
                            hipStream_t st) {
  int cnt = N * nw, P = 1;
  while (P < cnt) P <<= 1;
  size_t sh = (size_t)P * (sizeof(double) + sizeof(uint16_t));
  hipLaunchKernelGGL(line_sort_kernel, dim3((int64_t)N * N), dim3(256), sh, st, N, nw, eps, line_e, line_key);
  return hipGetLastError();
}

}  // namespace eph
