// Ensemble MLP surrogate of the scattering rates (gfx950, FP32).
//
// Members are independent multilayer perceptrons
//   x (10) -> 128 -> 128 -> 128 -> n_out,   SiLU between layers,
// trained by Adam on the mean squared error of normalised log(1/tau).
// Parameter layout of one member (row-major W[out][in]):
//   W1 b1 | W2 b2 | W3 b3 | W4 b4.
// Kernels (all hand-written):
//   mlp_fwdbwd_kernel  one workgroup = one member x one tile of 32 samples:
//                      forward through the layers with pre-activations kept
//                      in LDS, backward, and the tile's gradient written to
//                      its own slot (no atomics).  The hidden 128 x 128
//                      weights are staged in LDS (padded rows, the next
//                      layer's loads issued before the current one's
//                      products); every layer product (forward, input and
//                      weight gradients, output layer) runs on 16 x 16 x 4
//                      FP32 MFMA tiles, the first layer's forward on the
//                      vector units;
//   mlp_adam_kernel    per parameter: the tile gradients summed in tile
//                      order, then the Adam update;
//   mlp_forward_kernel inference for all members;
//   helpers for features, normalisation, ensemble blending and merging.
// Minibatch indices are the high half of a counter-based hash (splitmix64 of
// seed, member, step and position) times n, so training is reproducible for
// a given seed.
#include <math.h>

#include "internal.h"

namespace eph {
namespace mlp {

constexpr int NIN = 10;  // features: (sin, cos)(2 pi k_i/N) x 3, eps - mu, v x 3
constexpr int H = 128;
constexpr int TS = 32;       // samples per workgroup tile (inference)
constexpr int THREADS = 256;
constexpr int MAXOUT = EPH_MAX_TEMPS;

__host__ __device__ inline int64_t n_params(int nout) {
  return (int64_t)H * NIN + H + 2 * ((int64_t)H * H + H) + (int64_t)nout * H + nout;
}
struct Offs {
  int64_t w1, b1, w2, b2, w3, b3, w4, b4;
};
__host__ __device__ inline Offs offsets(int nout) {
  Offs o;
  o.w1 = 0;
  o.b1 = o.w1 + (int64_t)H * NIN;
  o.w2 = o.b1 + H;
  o.b2 = o.w2 + (int64_t)H * H;
  o.w3 = o.b2 + H;
  o.b3 = o.w3 + (int64_t)H * H;
  o.w4 = o.b3 + H;
  o.b4 = o.w4 + (int64_t)nout * H;
  return o;
}

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
// logistic function with the hardware exponential and reciprocal (a few ulp;
// the network is fit in FP32 to a target far coarser than that)
__device__ __forceinline__ float sigm(float z) { return __fdividef(1.0f, 1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigm(z);
  return s * (1.0f + z * (1.0f - s));
}

// out[s][o] = b[o] + sum_i W[o][i] in[s][i] for the TS samples; thread t
// owns output column o = t % H for samples (t / H) * TS/2 ... + TS/2 - 1.
__device__ void dense_fwd(const float *__restrict__ W, const float *__restrict__ b, const float *in, int nin,
                          int in_stride, float *out, int nout) {
  constexpr int SG = THREADS / H;  // 2 sample groups
  constexpr int SPT = TS / SG;     // 16 samples per thread
  const int t = threadIdx.x;
  const int o = t % H, g = t / H;
  if (o < nout) {
    float acc[SPT];
    const float bo = b[o];
#pragma unroll
    for (int j = 0; j < SPT; j++) acc[j] = bo;
    for (int i = 0; i < nin; i++) {
      const float w = W[(size_t)o * nin + i];
#pragma unroll
      for (int j = 0; j < SPT; j++) acc[j] = fmaf(w, in[(g * SPT + j) * in_stride + i], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < SPT; j++) out[(g * SPT + j) * H + o] = acc[j];
  }
}

// Training tile: TT samples per workgroup of TN threads (four waves).
constexpr int TT = 32;
constexpr int TN = 256;
// Row pitch (floats) of activations, gradients and staged weights in LDS: a
// column read by the 16 rows of an MFMA operand falls in distinct banks.
constexpr int HP = H + 4;

struct TrainArgs {
  int nout;
  int64_t n;             // training samples
  const float *x;        // [n][NIN] normalised
  const float *y;        // [n][nout] normalised
  const float *params;   // [members][P]
  float *grad_part;      // [members][tiles][P]
  float *loss_part;      // [members][tiles]
  int tiles;             // tiles per member (batch = tiles * TT)
  unsigned long long seed;
  long long step;        // -1: the batch is samples 0..batch-1 in order
};

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ float comp(const float4 &v, int q) { return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w; }

// FP32 matrix product D = A B + C on one 16 x 16 tile, K = 4:
// lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// D[4 (l / 16) + q][l % 16], q < 4.  The hidden-layer sums run over blocks of
// 16 inner indices; in a block, lane group g = l / 16 takes the indices
// 16 kb + 4 g + r (r < 4) in four successive products, for both operands.
__device__ __forceinline__ f4v mfma(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// One H x H weight matrix (row-major, any 4-byte alignment) from global
// memory: coalesced loads into registers, then into LDS rows of pitch HP.
struct WStage {
  float v[H * H / TN];
  __device__ __forceinline__ void load(const float *__restrict__ W) {
#pragma unroll
    for (int k = 0; k < H * H / TN; k++) v[k] = W[threadIdx.x + TN * k];
  }
  __device__ __forceinline__ void store(float *sW) const {
#pragma unroll
    for (int k = 0; k < H * H / TN; k++) {
      const int f = threadIdx.x + TN * k;
      sW[(f / H) * HP + f % H] = v[k];
    }
  }
};

// Tile ownership of the hidden-layer products: wave w, lane l, r16 = l % 16,
// g = l / 16.  Forward and input gradient: the wave holds samples
// 16 st + 4 g + q (st < 2) x columns 16 (2 w + ot) + r16 (ot < 2).
struct Lane {
  int w, r16, g;
  __device__ Lane() : w(threadIdx.x >> 6), r16(threadIdx.x & 15), g((threadIdx.x >> 4) & 3) {}
};

// z[s][o] = b[o] + sum_i W[o][i] a[s][i]  (W staged in sW, a in sA)
__device__ __forceinline__ void hidden_fwd(const Lane &L, const float *sW, const float *__restrict__ b,
                                           const float *sA, f4v acc[2][2]) {
#pragma unroll
  for (int ot = 0; ot < 2; ot++) {
    const float bo = b[16 * (2 * L.w + ot) + L.r16];
#pragma unroll
    for (int st = 0; st < 2; st++) acc[st][ot] = f4v{bo, bo, bo, bo};
  }
  for (int kb = 0; kb < H; kb += 16) {
    float4 av[2], wv[2];
#pragma unroll
    for (int st = 0; st < 2; st++) av[st] = ld4(&sA[(16 * st + L.r16) * HP + kb + 4 * L.g]);
#pragma unroll
    for (int ot = 0; ot < 2; ot++) wv[ot] = ld4(&sW[(16 * (2 * L.w + ot) + L.r16) * HP + kb + 4 * L.g]);
#pragma unroll
    for (int r = 0; r < 4; r++)
#pragma unroll
      for (int st = 0; st < 2; st++)
#pragma unroll
        for (int ot = 0; ot < 2; ot++) acc[st][ot] = mfma(comp(av[st], r), comp(wv[ot], r), acc[st][ot]);
  }
}

// g[s][i] = sum_o dz[s][o] W[o][i]  (W staged in sW, dz in sD)
__device__ __forceinline__ void hidden_bwd_input(const Lane &L, const float *sW, const float *sD, f4v acc[2][2]) {
#pragma unroll
  for (int st = 0; st < 2; st++)
#pragma unroll
    for (int ot = 0; ot < 2; ot++) acc[st][ot] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
  for (int kb = 0; kb < H; kb += 16) {
    float4 dv[2];
    float wv[2][4];
#pragma unroll
    for (int st = 0; st < 2; st++) dv[st] = ld4(&sD[(16 * st + L.r16) * HP + kb + 4 * L.g]);
#pragma unroll
    for (int ot = 0; ot < 2; ot++)
#pragma unroll
      for (int r = 0; r < 4; r++) wv[ot][r] = sW[(kb + 4 * L.g + r) * HP + 16 * (2 * L.w + ot) + L.r16];
#pragma unroll
    for (int r = 0; r < 4; r++)
#pragma unroll
      for (int st = 0; st < 2; st++)
#pragma unroll
        for (int ot = 0; ot < 2; ot++) acc[st][ot] = mfma(comp(dv[st], r), wv[ot][r], acc[st][ot]);
  }
}

// dW[o][i] = sum_s dz[s][o] a[s][i] over the tile's samples (the wave holds
// rows 16 (2 w + ot) + 4 g + q x all columns), stored into the tile's slot;
// db[o] = sum_s dz[s][o] (per lane over its samples, then across the four
// lane groups).
__device__ __forceinline__ void hidden_bwd_weights(const Lane &L, const float *sD, const float *sA,
                                                   float *__restrict__ gW, float *__restrict__ gb) {
  f4v acc[2][8];
  float db[2] = {0.0f, 0.0f};
#pragma unroll
  for (int ot = 0; ot < 2; ot++)
#pragma unroll
    for (int it = 0; it < 8; it++) acc[ot][it] = f4v{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kb = 0; kb < TT; kb += 16) {
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int s = kb + 4 * L.g + r;
      float dv[2], av[8];
#pragma unroll
      for (int ot = 0; ot < 2; ot++) {
        dv[ot] = sD[s * HP + 16 * (2 * L.w + ot) + L.r16];
        db[ot] += dv[ot];
      }
#pragma unroll
      for (int it = 0; it < 8; it++) av[it] = sA[s * HP + 16 * it + L.r16];
#pragma unroll
      for (int ot = 0; ot < 2; ot++)
#pragma unroll
        for (int it = 0; it < 8; it++) acc[ot][it] = mfma(dv[ot], av[it], acc[ot][it]);
    }
  }
#pragma unroll
  for (int ot = 0; ot < 2; ot++)
#pragma unroll
    for (int it = 0; it < 8; it++)
#pragma unroll
      for (int q = 0; q < 4; q++) gW[(size_t)(16 * (2 * L.w + ot) + 4 * L.g + q) * H + 16 * it + L.r16] = acc[ot][it][q];
#pragma unroll
  for (int ot = 0; ot < 2; ot++) {
    db[ot] += __shfl_xor(db[ot], 16);
    db[ot] += __shfl_xor(db[ot], 32);
    if (L.g == 0) gb[16 * (2 * L.w + ot) + L.r16] = db[ot];
  }
}

__global__ __launch_bounds__(TN) void mlp_fwdbwd_kernel(TrainArgs a) {
  __shared__ float sX[TT][NIN + 1];
  __shared__ __align__(16) float sZ[3][TT * HP];  // pre-activations of the hidden layers
  __shared__ __align__(16) float sA[TT * HP];     // input activations of the current layer
  __shared__ __align__(16) float sD[TT * HP];     // gradient w.r.t. the current layer's pre-activation
  __shared__ __align__(16) float sW[H * HP];      // the current hidden layer's weights
  __shared__ __align__(16) float sW4[MAXOUT * H];  // output-layer weights
  __shared__ float sDY[TT][MAXOUT];
  __shared__ float sYT[TT][MAXOUT];               // targets of the tile's samples
  __shared__ float sLoss[TN / 64];
  __shared__ long long sIdx[TT];
  const int member = blockIdx.y, tile = blockIdx.x, t = threadIdx.x;
  const int nout = a.nout;
  const int64_t P = n_params(nout);
  const Offs of = offsets(nout);
  const float *prm = a.params + (size_t)member * P;
  float *gp = a.grad_part + ((size_t)member * a.tiles + tile) * P;
  const float inv_batch = 1.0f / (float)(a.tiles * TT * nout);
  const Lane L;

  // minibatch sample indices
  if (t < TT) {
    long long idx;
    if (a.step < 0) idx = (long long)tile * TT + t;
    else {
      unsigned long long h = splitmix64(a.seed ^ splitmix64((unsigned long long)member * 0x100000001ull +
                                                            (unsigned long long)a.step * 0x9E37ull +
                                                            (unsigned long long)(tile * TT + t)));
      idx = (long long)__umul64hi(h, (unsigned long long)a.n);  // uniform in [0, n)
    }
    sIdx[t] = idx;
  }
  // first layer (NIN inputs) on the vector units: thread (og, sg) owns
  // columns og + 32 j and samples 4 sg + u; its weight rows are loaded now
  const int og = t & 31, sg = t >> 5;
  float w1r[4][NIN + 1];
#pragma unroll
  for (int j = 0; j < 4; j++) {
#pragma unroll
    for (int i = 0; i < NIN; i++) w1r[j][i] = prm[of.w1 + (size_t)(og + 32 * j) * NIN + i];
    w1r[j][NIN] = prm[of.b1 + og + 32 * j];
  }
  WStage ws;
  ws.load(prm + of.w2);
  __syncthreads();
  for (int e = t; e < TT * NIN; e += TN) {
    const int s = e / NIN, i = e % NIN;
    const long long idx = sIdx[s];
    sX[s][i] = idx < a.n ? a.x[idx * NIN + i] : 0.0f;
  }
  for (int e = t; e < nout * H; e += TN) sW4[e] = prm[of.w4 + e];
  for (int e = t; e < TT * nout; e += TN) {
    const long long idx = sIdx[e / nout];
    sYT[e / nout][e % nout] = idx < a.n ? a.y[idx * nout + e % nout] : 0.0f;
  }
  __syncthreads();
  // ---- forward ----
  {
    float z[4][4];
#pragma unroll
    for (int j = 0; j < 4; j++) {
#pragma unroll
      for (int u = 0; u < 4; u++) z[u][j] = w1r[j][NIN];
#pragma unroll
      for (int i = 0; i < NIN; i++)
#pragma unroll
        for (int u = 0; u < 4; u++) z[u][j] = fmaf(w1r[j][i], sX[4 * sg + u][i], z[u][j]);
    }
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
      for (int j = 0; j < 4; j++) {
        sZ[0][(4 * sg + u) * HP + og + 32 * j] = z[u][j];
        sA[(4 * sg + u) * HP + og + 32 * j] = silu(z[u][j]);
      }
  }
  ws.store(sW);
  __syncthreads();
  f4v acc[2][2];
  // hidden activations written back from the product tiles
  auto put = [&](float *z_out, const f4v (&v)[2][2]) {
#pragma unroll
    for (int st = 0; st < 2; st++)
#pragma unroll
      for (int ot = 0; ot < 2; ot++)
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const int e = (16 * st + 4 * L.g + q) * HP + 16 * (2 * L.w + ot) + L.r16;
          z_out[e] = v[st][ot][q];
          sA[e] = silu(v[st][ot][q]);
        }
  };
  ws.load(prm + of.w3);
  hidden_fwd(L, sW, prm + of.b2, sA, acc);
  __syncthreads();
  put(sZ[1], acc);
  ws.store(sW);
  __syncthreads();
  hidden_fwd(L, sW, prm + of.b3, sA, acc);
  __syncthreads();
  put(sZ[2], acc);
  __syncthreads();
  // output layer and dL/dy (mean squared error over batch and outputs):
  // wave w < 2 takes samples 16 w + 4 g + q x outputs n = r16 (< nout) as
  // one 16 x 16 tile over the 128 inputs
  float lsum = 0.0f;
  if (L.w < 2) {
    f4v yv = f4v{0.0f, 0.0f, 0.0f, 0.0f};
    const bool nv = L.r16 < nout;
    for (int kb = 0; kb < H; kb += 16) {
      const float4 av = ld4(&sA[(16 * L.w + L.r16) * HP + kb + 4 * L.g]);
      const float4 w4 = ld4(&sW4[(nv ? L.r16 : 0) * H + kb + 4 * L.g]);
      const float4 wv = nv ? w4 : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
      for (int r = 0; r < 4; r++) yv = mfma(comp(av, r), comp(wv, r), yv);
    }
    if (nv) {
      const float bn = prm[of.b4 + L.r16];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int s = 16 * L.w + 4 * L.g + q;
        const float y = yv[q] + bn;
        const float d = sIdx[s] < a.n ? y - sYT[s][L.r16] : 0.0f;
        sDY[s][L.r16] = 2.0f * d * inv_batch;
        lsum += d * d * inv_batch;
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
  if ((t & 63) == 0) sLoss[t >> 6] = lsum;
  __syncthreads();
  if (t == 0) a.loss_part[(size_t)member * a.tiles + tile] = (sLoss[0] + sLoss[1]) + (sLoss[2] + sLoss[3]);
  // ---- backward ----
  {  // output layer on 16 x 16 tiles over this wave's columns
     // i = 16 (2 w + ot) + r16: dW4[n][i] = sum_s dy[s][n] h3[s][i] (rows
     // n >= nout are zero and not stored); dh3 = dy W4 (inner index n, one
     // product per tile), dz3 = dh3 silu'(z3) into sD; then h2 into sA on the
     // same columns (this wave's reads of h3 there are done)
    f4v g4[2] = {f4v{0.0f, 0.0f, 0.0f, 0.0f}, f4v{0.0f, 0.0f, 0.0f, 0.0f}};
    float b4 = 0.0f;
#pragma unroll
    for (int kb = 0; kb < TT; kb += 16)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int s = kb + 4 * L.g + r;
        const float dv = L.r16 < nout ? sDY[s][L.r16 < nout ? L.r16 : 0] : 0.0f;
        b4 += dv;
#pragma unroll
        for (int ot = 0; ot < 2; ot++) g4[ot] = mfma(dv, sA[s * HP + 16 * (2 * L.w + ot) + L.r16], g4[ot]);
      }
    if (L.g == 0) {
#pragma unroll
      for (int ot = 0; ot < 2; ot++)
#pragma unroll
        for (int q = 0; q < 4; q++)
          if (q < nout) gp[of.w4 + (size_t)q * H + 16 * (2 * L.w + ot) + L.r16] = g4[ot][q];
    }
    b4 += __shfl_xor(b4, 16);
    b4 += __shfl_xor(b4, 32);
    if (L.w == 0 && L.g == 0 && L.r16 < nout) gp[of.b4 + L.r16] = b4;
#pragma unroll
    for (int st = 0; st < 2; st++)
#pragma unroll
      for (int ot = 0; ot < 2; ot++) {
        const int col = 16 * (2 * L.w + ot) + L.r16;
        const f4v d = mfma(L.g < nout ? sDY[16 * st + L.r16][L.g] : 0.0f, L.g < nout ? sW4[L.g * H + col] : 0.0f,
                           f4v{0.0f, 0.0f, 0.0f, 0.0f});
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const int e = (16 * st + 4 * L.g + q) * HP + col;
          sD[e] = d[q] * dsilu(sZ[2][e]);
          sA[e] = silu(sZ[1][e]);
        }
      }
  }
  // third hidden layer: the input gradient with W3 (still staged), then the
  // weight gradients
  ws.load(prm + of.w2);
  __syncthreads();
  hidden_bwd_input(L, sW, sD, acc);
  hidden_bwd_weights(L, sD, sA, gp + of.w3, gp + of.b3);
  __syncthreads();
  // dz2 = g * silu'(z2) into sD, h1 into sA, W2 into sW
#pragma unroll
  for (int st = 0; st < 2; st++)
#pragma unroll
    for (int ot = 0; ot < 2; ot++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int e = (16 * st + 4 * L.g + q) * HP + 16 * (2 * L.w + ot) + L.r16;
        sD[e] = acc[st][ot][q] * dsilu(sZ[1][e]);
        sA[e] = silu(sZ[0][e]);
      }
  ws.store(sW);
  __syncthreads();
  // second hidden layer
  hidden_bwd_input(L, sW, sD, acc);
  hidden_bwd_weights(L, sD, sA, gp + of.w2, gp + of.b2);
  __syncthreads();
#pragma unroll
  for (int st = 0; st < 2; st++)
#pragma unroll
    for (int ot = 0; ot < 2; ot++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int e = (16 * st + 4 * L.g + q) * HP + 16 * (2 * L.w + ot) + L.r16;
        sD[e] = acc[st][ot][q] * dsilu(sZ[0][e]);
      }
  __syncthreads();
  {  // first layer: dW1[o][i] = sum_s dz1[s][o] x[s][i] on 16 x 16 tiles
     // (columns i >= NIN are zero and not stored), db1 as for the hidden layers
    f4v w1[2] = {f4v{0.0f, 0.0f, 0.0f, 0.0f}, f4v{0.0f, 0.0f, 0.0f, 0.0f}};
    float b1[2] = {0.0f, 0.0f};
#pragma unroll
    for (int kb = 0; kb < TT; kb += 16)
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int s = kb + 4 * L.g + r;
        const float xv = L.r16 < NIN ? sX[s][L.r16 < NIN ? L.r16 : 0] : 0.0f;
#pragma unroll
        for (int ot = 0; ot < 2; ot++) {
          const float dv = sD[s * HP + 16 * (2 * L.w + ot) + L.r16];
          w1[ot] = mfma(dv, xv, w1[ot]);
          b1[ot] += dv;
        }
      }
    if (L.r16 < NIN) {
#pragma unroll
      for (int ot = 0; ot < 2; ot++)
#pragma unroll
        for (int q = 0; q < 4; q++) gp[of.w1 + (size_t)(16 * (2 * L.w + ot) + 4 * L.g + q) * NIN + L.r16] = w1[ot][q];
    }
#pragma unroll
    for (int ot = 0; ot < 2; ot++) {
      b1[ot] += __shfl_xor(b1[ot], 16);
      b1[ot] += __shfl_xor(b1[ot], 32);
      if (L.g == 0) gp[of.b1 + 16 * (2 * L.w + ot) + L.r16] = b1[ot];
    }
  }
}

// Sum tile gradients in tile order; optionally the Adam update.
__global__ void mlp_adam_kernel(int members, int tiles, int64_t P, const float *__restrict__ grad_part,
                                float *__restrict__ params, float *__restrict__ m1, float *__restrict__ m2,
                                float *__restrict__ grad_out, float lr, float b1, float b2, float eps,
                                float bc1, float bc2, int update) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)members * P) return;
  const int64_t e = i / P, p = i - (i / P) * P;
  float g = 0.0f;
  for (int t = 0; t < tiles; t++) g += grad_part[((size_t)e * tiles + t) * P + p];
  if (grad_out) grad_out[i] = g;
  if (update) {
    const float a = b1 * m1[i] + (1.0f - b1) * g;
    const float v = b2 * m2[i] + (1.0f - b2) * g * g;
    m1[i] = a;
    m2[i] = v;
    params[i] -= lr * (a / bc1) / (sqrtf(v / bc2) + eps);
  }
}

__global__ void mlp_loss_kernel(int members, int tiles, const float *__restrict__ loss_part,
                                float *__restrict__ loss) {
  const int e = threadIdx.x;
  if (e >= members) return;
  float l = 0.0f;
  for (int t = 0; t < tiles; t++) l += loss_part[e * tiles + t];
  loss[e] = l;
}

// Inference: y_out[member][s][n] = denormalised network output.
__global__ __launch_bounds__(THREADS) void mlp_forward_kernel(int nout, int64_t n, const float *__restrict__ x,
                                                              const float *__restrict__ params,
                                                              const float *__restrict__ norm,
                                                              float *__restrict__ y_out) {
  __shared__ float sX[TS][NIN + 1];
  __shared__ float sA[TS][H];
  __shared__ float sB[TS][H];
  const int member = blockIdx.y, t = threadIdx.x;
  const int64_t s0 = (int64_t)blockIdx.x * TS;
  const int64_t P = n_params(nout);
  const Offs of = offsets(nout);
  const float *prm = params + (size_t)member * P;
  const float *xm = norm, *xs = norm + NIN, *ym = norm + 2 * NIN, *ys = norm + 2 * NIN + MAXOUT;
  for (int e = t; e < TS * NIN; e += THREADS) {
    const int s = e / NIN, i = e % NIN;
    sX[s][i] = (s0 + s < n) ? (x[(s0 + s) * NIN + i] - xm[i]) / xs[i] : 0.0f;
  }
  __syncthreads();
  dense_fwd(prm + of.w1, prm + of.b1, &sX[0][0], NIN, NIN + 1, &sA[0][0], H);
  __syncthreads();
  for (int e = t; e < TS * H; e += THREADS) sA[e / H][e % H] = silu(sA[e / H][e % H]);
  __syncthreads();
  dense_fwd(prm + of.w2, prm + of.b2, &sA[0][0], H, H, &sB[0][0], H);
  __syncthreads();
  for (int e = t; e < TS * H; e += THREADS) sB[e / H][e % H] = silu(sB[e / H][e % H]);
  __syncthreads();
  dense_fwd(prm + of.w3, prm + of.b3, &sB[0][0], H, H, &sA[0][0], H);
  __syncthreads();
  for (int e = t; e < TS * H; e += THREADS) sA[e / H][e % H] = silu(sA[e / H][e % H]);
  __syncthreads();
  for (int e = t; e < TS * nout; e += THREADS) {
    const int s = e / nout, k = e % nout;
    if (s0 + s >= n) continue;
    float yv = prm[of.b4 + k];
    for (int i = 0; i < H; i++) yv = fmaf(prm[of.w4 + (size_t)k * H + i], sA[s][i], yv);
    y_out[((size_t)member * n + s0 + s) * nout + k] = yv * ys[k] + ym[k];
  }
}

// Features (the reduced k coordinates as (sin, cos)(2 pi k_i / N), which are
// periodic over the zone like the rates themselves, eps - mu, v / 1e6 m/s)
// and log-rate targets.
__global__ void mlp_features_kernel(int64_t n, const int32_t *__restrict__ sk, const double *__restrict__ e,
                                    const double *__restrict__ v, int N, double mu,
                                    const double *__restrict__ inv_tau, int nt, float *__restrict__ x,
                                    float *__restrict__ y) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t k = sk[s];
  const int64_t kc[3] = {k % N, (k / N) % N, k / ((int64_t)N * N)};
  for (int a = 0; a < 3; a++) {
    double sn_, cs_;
    sincospi(2.0 * (double)kc[a] / N, &sn_, &cs_);
    x[s * NIN + 2 * a] = (float)sn_;
    x[s * NIN + 2 * a + 1] = (float)cs_;
  }
  x[s * NIN + 6] = (float)(e[s] - mu);
  for (int a = 0; a < 3; a++) x[s * NIN + 7 + a] = (float)(v[3 * s + a] * 1e-6);
  if (inv_tau && y)
    for (int t = 0; t < nt; t++) y[s * nt + t] = (float)log(fmax(inv_tau[(int64_t)t * n + s], 1e-300));
}

// Column means and standard deviations of x [n][NIN] and y [n][nout] (one
// workgroup per column, fixed-order tree), into norm = xm | xs | ym | ys.
__global__ void mlp_norm_kernel(int64_t n, int nout, const float *__restrict__ x, const float *__restrict__ y,
                                float *__restrict__ norm) {
  __shared__ double s1[256], s2[256];
  const int col = blockIdx.x;
  const bool isx = col < NIN;
  const int c = isx ? col : col - NIN;
  const int stride = isx ? NIN : nout;
  const float *d = isx ? x : y;
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double v = d[i * stride + c];
    a += v;
    b += v * v;
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      s1[threadIdx.x] += s1[threadIdx.x + h];
      s2[threadIdx.x] += s2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double mean = s1[0] / (double)n;
    double var = s2[0] / (double)n - mean * mean;
    const double sd = var > 1e-24 ? sqrt(var) : 1.0;
    if (isx) {
      norm[c] = (float)mean;
      norm[NIN + c] = (float)sd;
    } else {
      norm[2 * NIN + c] = (float)mean;
      norm[2 * NIN + MAXOUT + c] = (float)sd;
    }
  }
}

__global__ void mlp_apply_norm_kernel(int64_t n, int nout, const float *__restrict__ x, const float *__restrict__ y,
                                      const float *__restrict__ norm, float *__restrict__ xn,
                                      float *__restrict__ yn) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n * NIN) xn[i] = (x[i] - norm[i % NIN]) / norm[NIN + i % NIN];
  if (i < n * nout) yn[i] = (y[i] - norm[2 * NIN + i % nout]) / norm[2 * NIN + MAXOUT + i % nout];
}

// Ensemble mean of exp(prediction) and relative spread (std/mean, max over
// outputs); flag[s] = spread > thr.
__global__ void mlp_blend_kernel(int members, int nout, int64_t n, const float *__restrict__ y, double thr,
                                 double *__restrict__ inv_tau, int32_t *__restrict__ flag,
                                 unsigned long long *__restrict__ nflag) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  double worst = 0.0;
  for (int k = 0; k < nout; k++) {
    double m = 0.0, q = 0.0;
    for (int e = 0; e < members; e++) {
      const double r = exp((double)y[((size_t)e * n + s) * nout + k]);
      m += r;
      q += r * r;
    }
    m /= members;
    const double var = fmax(q / members - m * m, 0.0);
    const double spread = m > 0.0 ? sqrt(var) / m : 1e300;
    worst = fmax(worst, spread);
    inv_tau[(int64_t)k * n + s] = m;
  }
  const int f = worst > thr ? 1 : 0;
  flag[s] = f;
  if (f) atomicAdd(nflag, 1ull);
}

__global__ void mlp_init_kernel(int members, int nout, unsigned long long seed, float *__restrict__ params) {
  const int64_t P = n_params(nout);
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= members * P) return;
  const int64_t p = i % P;
  const Offs of = offsets(nout);
  float fan_in;
  bool bias;
  if (p < of.b1) { fan_in = NIN; bias = false; }
  else if (p < of.w2) { fan_in = NIN; bias = true; }
  else if (p < of.b2) { fan_in = H; bias = false; }
  else if (p < of.w3) { fan_in = H; bias = true; }
  else if (p < of.b3) { fan_in = H; bias = false; }
  else if (p < of.w4) { fan_in = H; bias = true; }
  else if (p < of.b4) { fan_in = H; bias = false; }
  else { fan_in = H; bias = true; }
  if (bias) {
    params[i] = 0.0f;
    return;
  }
  const unsigned long long h = splitmix64(seed ^ splitmix64((unsigned long long)i));
  const float u = (float)((h >> 11) * (1.0 / 9007199254740992.0));  // [0, 1)
  const float lim = sqrtf(3.0f / fan_in) * 1.4f;
  params[i] = (2.0f * u - 1.0f) * lim;
}

// Merge: full_inv_tau[t][i] = sub_inv_tau[t][j] where (full_k, full_n)[i] ==
// (sub_k, sub_n)[j]; both lists sorted by (k, n).
__global__ void merge_kernel(int64_t nfull, const int32_t *__restrict__ fk, const int32_t *__restrict__ fn,
                             int64_t nsub, const int32_t *__restrict__ sk, const int32_t *__restrict__ sn, int nt,
                             const double *__restrict__ sub_it, double *__restrict__ full_it) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= nsub) return;
  const long long key = (long long)sk[j] * 64 + sn[j];
  int64_t lo = 0, hi = nfull;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    const long long km = (long long)fk[mid] * 64 + fn[mid];
    if (km < key) lo = mid + 1;
    else hi = mid;
  }
  if (lo < nfull && (long long)fk[lo] * 64 + fn[lo] == key)
    for (int t = 0; t < nt; t++) full_it[(int64_t)t * nfull + lo] = sub_it[(int64_t)t * nsub + j];
}

}  // namespace mlp
}  // namespace eph

// ------------------------------------------------------------------------
// C ABI of the surrogate
// ------------------------------------------------------------------------
using namespace eph;
using namespace eph::mlp;

struct eph_mlp {
  eph_ctx *ctx;
  int members, nout;
  int64_t P;
  bool normalised = false;
  DevBuf params, m1, m2, norm, gpart, lpart, loss, xn, yn, grad, nflag;
  long long step = 0;
  unsigned long long seed;
};

namespace {
int mfail(eph_mlp *m, int code, const std::string &msg) {
  m->ctx->err = msg;
  return code;
}
#define MHIP(m, expr)                                                                                         \
  do {                                                                                                        \
    hipError_t _e = (expr);                                                                                   \
    if (_e != hipSuccess) {                                                                                   \
      (void)hipGetLastError();                                                                                \
      return mfail(m, _e == hipErrorOutOfMemory ? EPH_E_NOMEM : EPH_E_DEVICE, std::string(#expr) + ": " +    \
                                                                                   hipGetErrorString(_e));    \
    }                                                                                                         \
  } while (0)

int run_fwdbwd(eph_mlp *m, int64_t n, const float *x, const float *y, int tiles, long long step, hipStream_t st) {
  MHIP(m, m->gpart.ensure(sizeof(float) * (size_t)m->members * tiles * m->P));
  MHIP(m, m->lpart.ensure(sizeof(float) * (size_t)m->members * tiles));
  TrainArgs a;
  a.nout = m->nout;
  a.n = n;
  a.x = x;
  a.y = y;
  a.params = m->params.as<float>();
  a.grad_part = m->gpart.as<float>();
  a.loss_part = m->lpart.as<float>();
  a.tiles = tiles;
  a.seed = m->seed;
  a.step = step;
  hipLaunchKernelGGL(mlp_fwdbwd_kernel, dim3(tiles, m->members), dim3(TN), 0, st, a);
  MHIP(m, hipGetLastError());
  return EPH_OK;
}
}  // namespace

extern "C" {

int32_t eph_mlp_create(eph_ctx *ctx, int32_t n_members, int32_t n_out, uint64_t seed, eph_mlp **out) {
  if (!ctx || !out) return EPH_E_INVALID;
  *out = nullptr;
  if (n_members < 1 || n_members > 64 || n_out < 1 || n_out > MAXOUT) {
    ctx->err = "n_members must be 1..64 and n_out 1..EPH_MAX_TEMPS";
    return EPH_E_INVALID;
  }
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return EPH_E_DEVICE;
  eph_mlp *m = new eph_mlp();
  m->ctx = ctx;
  m->members = n_members;
  m->nout = n_out;
  m->P = n_params(n_out);
  m->seed = seed;
  const size_t np = (size_t)n_members * m->P;
  hipError_t e;
  if ((e = m->params.ensure(4 * np)) != hipSuccess || (e = m->m1.ensure(4 * np)) != hipSuccess ||
      (e = m->m2.ensure(4 * np)) != hipSuccess || (e = m->norm.ensure(4 * (2 * NIN + 2 * MAXOUT))) != hipSuccess ||
      (e = m->loss.ensure(4 * 64)) != hipSuccess || (e = m->nflag.ensure(8)) != hipSuccess) {
    ctx->err = std::string("mlp allocation: ") + hipGetErrorString(e);
    delete m;
    return EPH_E_NOMEM;
  }
  hipLaunchKernelGGL(mlp_init_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, 0, n_members, n_out, seed,
                     m->params.as<float>());
  (void)launch_zero(m->m1.p, 4 * np, 0);
  (void)launch_zero(m->m2.p, 4 * np, 0);
  if ((e = hipDeviceSynchronize()) != hipSuccess) {
    ctx->err = std::string("mlp init: ") + hipGetErrorString(e);
    delete m;
    return EPH_E_DEVICE;
  }
  *out = m;
  return EPH_OK;
}

void eph_mlp_free(eph_mlp *m) {
  if (!m) return;
  DeviceGuard dg(m->ctx->device);
  delete m;
}

int32_t eph_mlp_params(eph_mlp *m, float *host, int64_t *n_params_out, int32_t set) {
  if (!m) return EPH_E_INVALID;
  if (n_params_out) *n_params_out = m->P;
  if (!host) return EPH_OK;
  DeviceGuard dg(m->ctx->device);
  if (!dg.ok) return EPH_E_DEVICE;
  const size_t bytes = 4 * (size_t)m->members * m->P;
  MHIP(m, set ? hipMemcpy(m->params.p, host, bytes, hipMemcpyHostToDevice)
              : hipMemcpy(host, m->params.p, bytes, hipMemcpyDeviceToHost));
  return EPH_OK;
}

int32_t eph_mlp_features(eph_ctx *ctx, int64_t n, const int32_t *state_k, const double *energy, const double *vel,
                         int32_t grid, double mu, const double *inv_tau, int32_t nt, float *x, float *y,
                         void *stream) {
  if (!ctx || n < 0 || grid < 1 || (n > 0 && (!state_k || !energy || !vel || !x))) return EPH_E_INVALID;
  if (inv_tau && (!y || nt < 1 || nt > MAXOUT)) return EPH_E_INVALID;
  if (n == 0) return EPH_OK;
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return EPH_E_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(mlp_features_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, state_k, energy,
                     vel, grid, mu, inv_tau, nt, x, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ctx->err = hipGetErrorString(e);
    return EPH_E_DEVICE;
  }
  return EPH_OK;
}

int32_t eph_mlp_train(eph_mlp *m, int64_t n, const float *x, const float *y, int32_t steps, int32_t batch,
                      float lr, void *stream, float *loss_host) {
  if (!m) return EPH_E_INVALID;
  if (n < 1 || !x || !y || steps < 0 || batch < TT || batch % TT || !(lr > 0.0f))
    return mfail(m, EPH_E_INVALID, "train: n >= 1, batch a positive multiple of 32, lr > 0");
  DeviceGuard dg(m->ctx->device);
  if (!dg.ok) return EPH_E_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!m->normalised) {  // statistics of the first training set define the normalisation
    hipLaunchKernelGGL(mlp_norm_kernel, dim3(NIN + m->nout), dim3(256), 0, st, n, m->nout, x, y, m->norm.as<float>());
    MHIP(m, hipGetLastError());
    m->normalised = true;
  }
  MHIP(m, m->xn.ensure(4 * (size_t)n * NIN));
  MHIP(m, m->yn.ensure(4 * (size_t)n * m->nout));
  hipLaunchKernelGGL(mlp_apply_norm_kernel, dim3((unsigned)((n * NIN + 255) / 256)), dim3(256), 0, st, n, m->nout, x,
                     y, m->norm.as<float>(), m->xn.as<float>(), m->yn.as<float>());
  MHIP(m, hipGetLastError());
  const int tiles = batch / TT;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const int64_t np = (int64_t)m->members * m->P;
  for (int s = 0; s < steps; s++) {
    m->step++;
    int r = run_fwdbwd(m, n, m->xn.as<float>(), m->yn.as<float>(), tiles, m->step, st);
    if (r != EPH_OK) return r;
    const float bc1 = 1.0f - powf(b1, (float)m->step), bc2 = 1.0f - powf(b2, (float)m->step);
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, m->members, tiles,
                       m->P, m->gpart.as<float>(), m->params.as<float>(), m->m1.as<float>(),
                       m->m2.as<float>(), (float *)nullptr, lr, b1, b2, eps, bc1, bc2, 1);
    MHIP(m, hipGetLastError());
  }
  if (loss_host) {
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(64), 0, st, m->members, tiles, m->lpart.as<float>(),
                       m->loss.as<float>());
    MHIP(m, hipMemcpyAsync(loss_host, m->loss.p, 4 * m->members, hipMemcpyDeviceToHost, st));
  }
  MHIP(m, hipStreamSynchronize(st));
  return EPH_OK;
}

int32_t eph_mlp_gradient(eph_mlp *m, int64_t n, const float *x, const float *y, float *grad_host,
                         float *loss_host) {
  if (!m || n < TT || n % TT || !x || !y || !grad_host) return EPH_E_INVALID;
  DeviceGuard dg(m->ctx->device);
  if (!dg.ok) return EPH_E_DEVICE;
  const int tiles = (int)(n / TT);
  int r = run_fwdbwd(m, n, x, y, tiles, -1, 0);
  if (r != EPH_OK) return r;
  const int64_t np = (int64_t)m->members * m->P;
  MHIP(m, m->grad.ensure(4 * (size_t)np));
  hipLaunchKernelGGL(mlp_adam_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, 0, m->members, tiles, m->P,
                     m->gpart.as<float>(), m->params.as<float>(), m->m1.as<float>(), m->m2.as<float>(),
                     m->grad.as<float>(), 0.0f, 0.0f, 0.0f, 0.0f, 1.0f, 1.0f, 0);
  MHIP(m, hipGetLastError());
  MHIP(m, hipMemcpy(grad_host, m->grad.p, 4 * (size_t)np, hipMemcpyDeviceToHost));
  if (loss_host) {
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(64), 0, 0, m->members, tiles, m->lpart.as<float>(),
                       m->loss.as<float>());
    MHIP(m, hipMemcpy(loss_host, m->loss.p, 4 * m->members, hipMemcpyDeviceToHost));
  }
  return EPH_OK;
}

int32_t eph_mlp_predict(eph_mlp *m, int64_t n, const float *x, float *y, void *stream) {
  if (!m || n < 0 || (n > 0 && (!x || !y))) return EPH_E_INVALID;
  if (!m->normalised) return mfail(m, EPH_E_STATE, "predict before train");
  if (n == 0) return EPH_OK;
  DeviceGuard dg(m->ctx->device);
  if (!dg.ok) return EPH_E_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)((n + TS - 1) / TS), m->members), dim3(THREADS), 0, st,
                     m->nout, n, x, m->params.as<float>(), m->norm.as<float>(), y);
  MHIP(m, hipGetLastError());
  return EPH_OK;
}

int32_t eph_mlp_blend(eph_mlp *m, int64_t n, const float *y, double threshold, double *inv_tau, int32_t *flag,
                      int64_t *n_flagged, void *stream) {
  if (!m || n < 0 || (n > 0 && (!y || !inv_tau || !flag))) return EPH_E_INVALID;
  DeviceGuard dg(m->ctx->device);
  if (!dg.ok) return EPH_E_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  MHIP(m, launch_zero(m->nflag.p, 8, st));
  if (n > 0) {
    hipLaunchKernelGGL(mlp_blend_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m->members, m->nout, n,
                       y, threshold, inv_tau, flag, m->nflag.as<unsigned long long>());
    MHIP(m, hipGetLastError());
  }
  unsigned long long c = 0;
  MHIP(m, hipMemcpyAsync(&c, m->nflag.p, 8, hipMemcpyDeviceToHost, st));
  MHIP(m, hipStreamSynchronize(st));
  if (n_flagged) *n_flagged = (int64_t)c;
  return EPH_OK;
}

int32_t eph_merge_rates(eph_ctx *ctx, int64_t n_full, const int32_t *full_k, const int32_t *full_n, int64_t n_sub,
                        const int32_t *sub_k, const int32_t *sub_n, const double *sub_inv_tau, int32_t nt,
                        double *full_inv_tau, void *stream) {
  if (!ctx || n_full < 0 || n_sub < 0 || nt < 1 || nt > MAXOUT) return EPH_E_INVALID;
  if (n_sub == 0) return EPH_OK;
  if (!full_k || !full_n || !sub_k || !sub_n || !sub_inv_tau || !full_inv_tau) return EPH_E_INVALID;
  DeviceGuard dg(ctx->device);
  if (!dg.ok) return EPH_E_DEVICE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(merge_kernel, dim3((unsigned)((n_sub + 255) / 256)), dim3(256), 0, st, n_full, full_k, full_n,
                     n_sub, sub_k, sub_n, nt, sub_inv_tau, full_inv_tau);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ctx->err = hipGetErrorString(e);
    return EPH_E_DEVICE;
  }
  return EPH_OK;
}

}  // extern "C"
