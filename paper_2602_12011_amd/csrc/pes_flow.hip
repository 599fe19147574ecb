// Learned proposal on the device: an affine-coupling normalizing flow on the
// 11 standardized parameters (8 coupling layers, conditioner networks
// n_C -> 256 -> 256 -> 2 n_T), evaluated and trained with BF16 operands and
// FP32 accumulation on the matrix cores (v_mfma_f32_16x16x32_bf16), the
// coupling arithmetic in FP32, and Adam on FP32 master weights.  Its samples
// feed an independence Metropolis-Hastings proposal whose acceptance uses the
// exact FP64 likelihood; Sec. 2.2 leaves the proposal to the sampler.
//
// Conventions (the flow's definition): u = float(L^-1 (theta - mu)) with L
// lower triangular (a whitening map, L L^T a covariance; forward substitution
// in FP64);
// layer 2p conditions on C_p = {i : (i + 3p) mod 11 < 6} and transforms the
// other 5 coordinates, layer 2p + 1 conditions on those 5 and transforms C_p;
// s = 3 tanh(s_hat / 3); normalizing direction y_T = x_T e^s + t, log det +=
// sum s; base N(0, I).  Parameters per layer (y = x W + b): W1 [n_C][256],
// b1, W2 [256][256], b2, W3 [256][2 n_T], b3, flat in that order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <random>

#include "../../include/pes.h"
#include "pes_flow.hpp"

namespace pes {
namespace fl {

constexpr int kD = 11;
constexpr int kHid = 256;
constexpr int kLayers = 8;
constexpr int kPad = 32;            // padded conditioner input and output width
constexpr int kTensors = 6 * kLayers;
constexpr int kLayerW = kPad * kHid + kHid * kHid + kHid * kPad;   // bf16 weights per layer
constexpr int kLayerB = kHid + kHid + kPad;                          // padded biases per layer
constexpr float kSMax = 3.0f;
constexpr int64_t kRowAlign = 64;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct LayerSpec {
  int nc, nt;
  int cond[6], trans[6];
};

struct TensorDesc {
  int64_t off;    // in the flat FP32 parameters
  int rows, cols;
  int64_t woff;   // bf16 copy (weights) or -1
  int64_t boff;   // padded FP32 copy (biases) or -1
  int ldw;
};
struct TensorTable {
  TensorDesc t[kTensors];
};

struct Norm {
  double mu[kD];
  double L[kD][kD];   // lower triangular
};

// ------------------------------------------------------------------ GEMM
// C[m][n] = sum_k A(m, k) B(n, k) with BF16 operands and FP32 accumulation.
// A(m, k) = A[m lda + k] (A_ROW) or A[k lda + m]; B(n, k) = B[n ldb + k]
// (B_ROW) or B[k ldb + n].  M, N, K are multiples of 32.  A TM x TN output
// tile (TM, TN in {32, 64}) per block of four waves in a 2 x 2 arrangement;
// each wave owns a (TM / 2) x (TN / 2) tile of 16 x 16 matrix-core blocks and
// issues one 16x16x32 operation per block per 32-deep slab staged through LDS
// (both operand layouts are loaded coalesced and transposed in LDS as needed).
// Split over K (EPI_F32 only, for the weight gradients, whose K is the batch):
// block z of the grid's third dimension sums its share of the slabs into
// part[z][M][N]; split_reduce_kernel adds the shares in order (deterministic).
enum : int { EPI_F32 = 0, EPI_BIAS_F32 = 1, EPI_BIAS_RELU_BF16 = 2, EPI_MASK = 3 };

constexpr int kMaxSplit = 16;   // shares of K in a split product (part buffer: kMaxSplit x kHid x kHid)

struct GemmArgs {
  const __bf16* A;
  int64_t lda;
  const __bf16* B;
  int64_t ldb;
  int M, N, K;
  const float* bias;     // [N]
  const __bf16* mask;    // EPI_MASK: zero where mask <= 0
  int64_t ldm;
  float* C;              // FP32 out
  int64_t ldc;
  __bf16* Cb;            // BF16 out
  int64_t ldcb;
  int m_valid, n_valid;  // EPI_F32: rows / columns written
  float* part;           // split products: [split][M][N] (M N <= kHid kHid)
  int split;             // shares of K (1: no split)
};

// Stages rows r0.. of a slab: R rows of 32 k-values (ROW: X[(o + r) ld + k0 + c],
// else the transpose X[(k0 + r) ld + o + c]) into S[R][40], one bf16x8 per thread
// for the threads t < 4 R.
template <bool ROW, int R>
__device__ __forceinline__ void stage_slab(__bf16 (*S)[40], const __bf16* X, int64_t ld, int o, int k0, int t) {
  if (t >= 4 * R) return;
  if (ROW) {
    const int r = t >> 2, c = (t & 3) * 8;
    *(bf16x8*)&S[r][c] = *(const bf16x8*)(X + (int64_t)(o + r) * ld + k0 + c);
  } else {   // r indexes k (32 of them), c the R output rows
    constexpr int PER = R / 8;
    const int r = t / PER, c = (t % PER) * 8;
    const bf16x8 v = *(const bf16x8*)(X + (int64_t)(k0 + r) * ld + o + c);
#pragma unroll
    for (int e = 0; e < 8; ++e) S[c + e][r] = v[e];
  }
}

template <bool A_ROW, bool B_ROW, int EPI, int TM, int TN>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g) {
  constexpr int MI = TM / 32, NJ = TN / 32;   // 16 x 16 blocks per wave
  __shared__ __attribute__((aligned(16))) __bf16 As[TM][40];   // [m][k], rows padded to 80 bytes
  __shared__ __attribute__((aligned(16))) __bf16 Bs[TN][40];   // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int wm = (wv >> 1) * (TM / 2), wn = (wv & 1) * (TN / 2);
  // this block's slabs of K
  const int slabs = g.K / 32, z = blockIdx.z;
  const int s0 = (int)((int64_t)slabs * z / g.split), s1 = (int)((int64_t)slabs * (z + 1) / g.split);
  f32x4 acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) acc[i][jj] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int sl = s0; sl < s1; ++sl) {
    const int k0 = sl * 32;
    stage_slab<A_ROW, TM>(As, g.A, g.lda, m0, k0, tid);
    stage_slab<B_ROW, TN>(Bs, g.B, g.ldb, n0, k0, (tid + 4 * TM) & 255);
    __syncthreads();
    // operand lanes: A[i = lane % 16][k = 8 (lane / 16) + e], B likewise by column
    bf16x8 a[MI], b[NJ];
#pragma unroll
    for (int i = 0; i < MI; ++i) a[i] = *(const bf16x8*)&As[wm + 16 * i + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) b[jj] = *(const bf16x8*)&Bs[wn + 16 * jj + (lane & 15)][8 * (lane >> 4)];
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[jj], acc[i][jj], 0, 0, 0);
    __syncthreads();
  }
  // result lanes: element e of lane l is (row 4 (l / 16) + e, column l % 16)
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int jj = 0; jj < NJ; ++jj) {
      const int n = n0 + wn + 16 * jj + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + e;
        float v = acc[i][jj][e];
        if (EPI == EPI_F32) {
          if (g.split > 1)
            g.part[((int64_t)z * g.M + m) * g.N + n] = v;
          else if (m < g.m_valid && n < g.n_valid)
            g.C[(int64_t)m * g.ldc + n] = v;
        } else if (EPI == EPI_BIAS_F32) {
          g.C[(int64_t)m * g.ldc + n] = v + g.bias[n];
        } else if (EPI == EPI_BIAS_RELU_BF16) {
          v = fmaxf(v + g.bias[n], 0.0f);
          g.Cb[(int64_t)m * g.ldcb + n] = (__bf16)v;
        } else {   // EPI_MASK
          if (!((float)g.mask[(int64_t)m * g.ldm + n] > 0.0f)) v = 0.0f;
          g.C[(int64_t)m * g.ldc + n] = v;
          g.Cb[(int64_t)m * g.ldcb + n] = (__bf16)v;
        }
      }
    }
}

// C[m][n] = sum over the shares z = 0, 1, ... of part[z][m][n], m < m_valid, n < n_valid.
__global__ void split_reduce_kernel(GemmArgs g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)g.m_valid * g.n_valid) return;
  const int m = (int)(i / g.n_valid), n = (int)(i % g.n_valid);
  float v = 0.0f;
  for (int z = 0; z < g.split; ++z) v += g.part[((int64_t)z * g.M + m) * g.N + n];
  g.C[(int64_t)m * g.ldc + n] = v;
}

template <bool AR, bool BR, int EPI, int TM, int TN>
static void launch_gemm(const GemmArgs& g, hipStream_t s) {
  hipLaunchKernelGGL((gemm_kernel<AR, BR, EPI, TM, TN>), dim3(g.N / TN, g.M / TM, g.split), dim3(256), 0, s, g);
}

// Tiles of 64 where the shape allows; products with fewer than 256 tiles and a
// long K (the weight gradients) split K into up to kMaxSplit shares of at
// least eight slabs.
template <bool AR, bool BR, int EPI>
hipError_t gemm(GemmArgs g, hipStream_t s) {
  if (g.M % 32 || g.N % 32 || g.K % 32 || g.M <= 0 || g.N <= 0 || g.K <= 0) return hipErrorInvalidValue;
  const int TM = g.M % 64 ? 32 : 64, TN = g.N % 64 ? 32 : 64;
  const int tiles = (g.M / TM) * (g.N / TN);
  g.split = 1;
  if (EPI == EPI_F32 && g.part && tiles < 256 && (int64_t)g.M * g.N <= (int64_t)kHid * kHid)
    g.split = std::max(1, std::min({kMaxSplit, 256 / tiles, g.K / (32 * 8)}));
  if (TM == 64 && TN == 64) launch_gemm<AR, BR, EPI, 64, 64>(g, s);
  else if (TM == 64) launch_gemm<AR, BR, EPI, 64, 32>(g, s);
  else if (TN == 64) launch_gemm<AR, BR, EPI, 32, 64>(g, s);
  else launch_gemm<AR, BR, EPI, 32, 32>(g, s);
  if (g.split > 1) {
    const int64_t n = (int64_t)g.m_valid * g.n_valid;
    hipLaunchKernelGGL(split_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ elementwise
// u = L^-1 (theta - mu) by forward substitution in FP64, rounded to FP32.
__global__ void standardize_kernel(const double* __restrict__ theta, int64_t n, int64_t Mp, Norm nm,
                                   float* __restrict__ x, float* __restrict__ logdet) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Mp) return;
  logdet[j] = 0.0f;
  double u[kD];
#pragma unroll
  for (int k = 0; k < kD; ++k) {
    double acc = j < n ? theta[j * kD + k] - nm.mu[k] : 0.0;
#pragma unroll
    for (int m = 0; m < k; ++m) acc -= nm.L[k][m] * u[m];
    u[k] = acc / nm.L[k][k];
    x[j * kD + k] = (float)u[k];
  }
}

// Latent rows tau z, rounded to FP32 after the product.
__global__ void load_latent_kernel(const double* __restrict__ z, int64_t n, int64_t Mp, double tau,
                                   float* __restrict__ x, float* __restrict__ logdet) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Mp * kD) return;
  const int64_t j = i / kD;
  x[i] = j < n ? (float)(tau * z[i]) : 0.0f;
  if (i - j * kD == 0) logdet[j] = 0.0f;
}

__global__ void gather_kernel(const float* __restrict__ x, __bf16* __restrict__ xc, int64_t Mp, LayerSpec ls) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Mp * kPad) return;
  const int64_t j = i / kPad;
  const int c = (int)(i - j * kPad);
  float v = 0.0f;
  if (c < ls.nc) v = x[j * kD + ls.cond[c]];
  xc[i] = (__bf16)v;
}

// One coupling layer on the rows: forward y_T = x_T e^s + t or inverse
// x_T = (y_T - t) e^-s; logdet += sum s (the normalizing map's).  xin (may be
// null) receives the rows before the update.
__global__ void couple_kernel(float* __restrict__ x, const float* __restrict__ O, float* __restrict__ logdet,
                              float* __restrict__ xin, int64_t Mp, LayerSpec ls, int inverse) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Mp) return;
  float* xr = x + j * kD;
  if (xin)
    for (int k = 0; k < kD; ++k) xin[j * kD + k] = xr[k];
  const float* o = O + j * kPad;
  float ld = 0.0f;
  for (int q = 0; q < ls.nt; ++q) {
    const float s = kSMax * tanhf(o[q] / kSMax);
    const float t = o[ls.nt + q];
    const int idx = ls.trans[q];
    xr[idx] = inverse ? (xr[idx] - t) * expf(-s) : fmaf(xr[idx], expf(s), t);
    ld += s;
  }
  logdet[j] += ld;
}

// log q(theta) = -|z|^2/(2 tau^2) - 11 log tau - (11/2) log 2 pi + log det - sum log L_kk.
__global__ void logq_kernel(const float* __restrict__ z, const float* __restrict__ logdet, int64_t n,
                            double lsig, double tau, double* __restrict__ logq, double* __restrict__ zout) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double q = 0.0;
  for (int k = 0; k < kD; ++k) {
    const double v = (double)z[j * kD + k];
    q = fma(v, v, q);
    if (zout) zout[j * kD + k] = v;
  }
  logq[j] = -0.5 * q / (tau * tau) - kD * log(tau) - 0.5 * kD * 1.8378770664093454836 + (double)logdet[j] - lsig;
}

// theta = mu + L u.
__global__ void unstandardize_kernel(const float* __restrict__ x, const float* __restrict__ logdet, int64_t n,
                                     Norm nm, double* __restrict__ theta, double* __restrict__ ld_out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double u[kD];
#pragma unroll
  for (int k = 0; k < kD; ++k) u[k] = (double)x[j * kD + k];
#pragma unroll
  for (int k = 0; k < kD; ++k) {
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m <= k; ++m) acc = fma(nm.L[k][m], u[m], acc);
    theta[j * kD + k] = nm.mu[k] + acc;
  }
  if (ld_out) ld_out[j] = (double)logdet[j];
}

// Probe hook: the coupling state and running log-determinant of the first n
// rows into slot k of states [kLayers + 1][n][11] and logdet [kLayers + 1][n].
__global__ void copy_state_kernel(const float* __restrict__ x, const float* __restrict__ logdet, int64_t n, int k,
                                  float* __restrict__ states, float* __restrict__ ld_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * kD) return;
  states[(int64_t)k * n * kD + i] = x[i];
  if (i % kD == 0) ld_out[(int64_t)k * n + i / kD] = logdet[i / kD];
}

// Probe: the conditioner stages of every layer (slot l of the stored
// activations) into acts [kLayers][n][kActCols] as FP32: the BF16 input
// (kPad columns), the two BF16 hidden layers (kHid each), the FP32 output
// (kPad columns).
constexpr int kActCols = kPad + kHid + kHid + kPad;

__global__ void copy_acts_kernel(const __bf16* __restrict__ Xc, const __bf16* __restrict__ H1,
                                 const __bf16* __restrict__ H2, const float* __restrict__ O, int64_t Mp, int64_t n,
                                 float* __restrict__ acts) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)kLayers * n * kActCols) return;
  const int c = (int)(i % kActCols);
  const int64_t r = i / kActCols;        // l * n + row
  const int64_t l = r / n, j = r - l * n;
  const int64_t so = l * Mp + j;
  float v;
  if (c < kPad) v = (float)Xc[so * kPad + c];
  else if (c < kPad + kHid) v = (float)H1[so * kHid + (c - kPad)];
  else if (c < kPad + 2 * kHid) v = (float)H2[so * kHid + (c - kPad - kHid)];
  else v = O[so * kPad + (c - kPad - 2 * kHid)];
  acts[i] = v;
}

// ------------------------------------------------------------------ training
// Seeds the backward pass of NLL = (1/n) sum_j (|z_j|^2/2 + 11/2 log 2 pi - logdet_j):
// dNLL/dz = z / n, and the per-row NLL terms.
__global__ void nll_seed_kernel(const float* __restrict__ z, const float* __restrict__ logdet, int64_t n,
                                int64_t Mp, float* __restrict__ gy, double* __restrict__ rowv) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Mp) return;
  const float w = j < n ? 1.0f / (float)n : 0.0f;
  double q = 0.0;
  for (int k = 0; k < kD; ++k) {
    const float v = z[j * kD + k];
    gy[j * kD + k] = w * v;
    q = fma((double)v, (double)v, q);
  }
  rowv[j] = j < n ? (0.5 * q + 0.5 * kD * 1.8378770664093454836 - (double)logdet[j]) / (double)n : 0.0;
}

// Ordered sum of n doubles by one block (fixed order: bitwise repeatable).
__global__ void __launch_bounds__(256) sum_rows_kernel(const double* __restrict__ v, int64_t n,
                                                       double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += v[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Backward of one coupling layer (normalizing direction).  gy: d/dy of the
// layer output; gx receives d/dx of its input except the conditioner path
// through the network (added later); gO: d/d(network output).
__global__ void couple_bwd_kernel(const float* __restrict__ xin, const float* __restrict__ O,
                                  const float* __restrict__ gy, float* __restrict__ gx, float* __restrict__ gOf,
                                  __bf16* __restrict__ gOb, int64_t n, int64_t Mp, LayerSpec ls) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Mp) return;
  const float gld = j < n ? -1.0f / (float)n : 0.0f;
  for (int k = 0; k < kD; ++k) gx[j * kD + k] = gy[j * kD + k];
  const float* o = O + j * kPad;
  float* go = gOf + j * kPad;
  for (int q = 0; q < kPad; ++q) go[q] = 0.0f;
  for (int q = 0; q < ls.nt; ++q) {
    const int idx = ls.trans[q];
    const float th = tanhf(o[q] / kSMax);
    const float es = expf(kSMax * th);
    const float g = gy[j * kD + idx];
    gx[j * kD + idx] = g * es;
    const float gs = fmaf(g * xin[j * kD + idx], es, gld);
    go[q] = gs * (1.0f - th * th);
    go[ls.nt + q] = g;
  }
  for (int q = 0; q < kPad; ++q) gOb[j * kPad + q] = (__bf16)go[q];
}

// out[c] = sum_rows X[r][c] for c < ncols (one block per column, fixed order).
__global__ void __launch_bounds__(256) colsum_kernel(const float* __restrict__ X, int64_t ldx, int64_t M,
                                                     float* __restrict__ out) {
  __shared__ float sh[256];
  const int c = blockIdx.x;
  float s = 0.0f;
  for (int64_t r = threadIdx.x; r < M; r += 256) s += X[r * ldx + c];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = sh[0];
}

__global__ void scatter_cond_kernel(const float* __restrict__ dxc, float* __restrict__ gx, int64_t Mp,
                                    LayerSpec ls) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= Mp) return;
  for (int c = 0; c < ls.nc; ++c) gx[j * kD + ls.cond[c]] += dxc[j * kPad + c];
}

// Adam (update != 0) and the refresh of the BF16 weight and padded bias copies.
__global__ void adam_kernel(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ m1,
                            float* __restrict__ m2, __bf16* __restrict__ wb, float* __restrict__ bp,
                            TensorTable tt, int update, float lr, float b1, float b2, float c1, float c2,
                            float eps) {
  const TensorDesc d = tt.t[blockIdx.y];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)d.rows * d.cols) return;
  const int64_t p = d.off + i;
  float w = P[p];
  if (update) {
    const float g = G[p];
    const float a = fmaf(b1, m1[p], (1.0f - b1) * g);
    const float v = fmaf(b2, m2[p], (1.0f - b2) * g * g);
    m1[p] = a;
    m2[p] = v;
    w -= lr * (a * c1) / (sqrtf(v * c2) + eps);
    P[p] = w;
  }
  if (d.woff >= 0) {
    const int64_t r = i / d.cols, c = i - r * d.cols;
    wb[d.woff + r * d.ldw + c] = (__bf16)w;
  } else {
    bp[d.boff + i] = w;
  }
}

// Minibatch of rows drawn with replacement (SplitMix64 of (seed, step, row),
// Steele, Lea & Flood, OOPSLA 2014), or all rows in order when batch == n.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

__global__ void batch_kernel(const double* __restrict__ samples, int64_t n, int64_t batch, uint64_t seed,
                             uint64_t step, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= batch) return;
  int64_t src = j;
  if (batch != n) {
    const uint64_t h = splitmix64(seed ^ splitmix64((step << 32) ^ (uint64_t)j));
    src = (int64_t)(h % (uint64_t)n);
  }
  for (int k = 0; k < kD; ++k) out[j * kD + k] = samples[src * kD + k];
}

// Mean (blocks 0..10) of n rows, then the covariance entry (a, b), a >= b,
// of block a * 11 + b (second launch); fixed order per block.
__device__ double block_sum(double s) {
  __shared__ double sh[256];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(256) mean_kernel(const double* __restrict__ x, int64_t n,
                                                   double* __restrict__ out) {
  const int k = blockIdx.x;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) s += x[r * kD + k];
  s = block_sum(s);
  if (threadIdx.x == 0) out[k] = s / (double)n;
}

__global__ void __launch_bounds__(256) cov_kernel(const double* __restrict__ x, int64_t n,
                                                  double* __restrict__ mom) {
  const int a = blockIdx.x / kD, b = blockIdx.x % kD;
  if (b > a) return;
  const double ma = mom[a], mb = mom[b];
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += 256) s = fma(x[r * kD + a] - ma, x[r * kD + b] - mb, s);
  s = block_sum(s);
  if (threadIdx.x == 0) mom[kD + a * kD + b] = s / (double)n;
}

inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace fl
}  // namespace pes

using namespace pes::fl;

struct pes_flow {
  LayerSpec L[kLayers];
  TensorTable tt;
  int64_t np = 0;
  float *P = nullptr, *G = nullptr, *m1 = nullptr, *m2 = nullptr;
  __bf16* wb = nullptr;   // [layer][kLayerW]: W1 [32][256], W2 [256][256], W3 [256][32]
  float* bp = nullptr;    // [layer][kLayerB]: b1 [256], b2 [256], b3 [32]
  Norm nm;
  double lsig = 0.0;
  double tau = 1.0;     // temperature of the base density
  int64_t t_adam = 0;
  // workspace (rows padded to a multiple of 64)
  int64_t cap = 0;
  uint64_t gen = 0;     // bumped whenever the workspace is reallocated
  float *x = nullptr, *logdet = nullptr, *xin = nullptr, *O = nullptr;
  __bf16 *Xc = nullptr, *H1 = nullptr, *H2 = nullptr;
  float *gy = nullptr, *gx = nullptr, *gOf = nullptr, *dpf = nullptr, *dXc = nullptr;
  __bf16 *gOb = nullptr, *dpb = nullptr;
  double *rowv = nullptr, *batchbuf = nullptr, *mom = nullptr;
  float* kpart = nullptr;   // shares of the split weight-gradient products [kMaxSplit][kHid][kHid]
  char err[256] = {0};
};

namespace {

#define FL_HIP(f, expr)                                                          \
  do {                                                                           \
    const hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                      \
      snprintf((f)->err, sizeof((f)->err), "%s: %s", #expr, hipGetErrorString(e_)); \
      return PES_EHIP;                                                           \
    }                                                                            \
  } while (0)

int64_t pad_rows(int64_t n) { return std::max<int64_t>(kRowAlign, (n + kRowAlign - 1) / kRowAlign * kRowAlign); }

void free_ws(pes_flow* f) {
  void* ps[] = {f->x, f->logdet, f->xin, f->O, f->Xc, f->H1, f->H2, f->gy, f->gx,
                f->gOf, f->dpf, f->dXc, f->gOb, f->dpb, f->rowv, f->batchbuf};
  for (void* p : ps) (void)hipFree(p);
  f->x = f->logdet = f->xin = f->O = f->gy = f->gx = f->gOf = f->dpf = f->dXc = nullptr;
  f->Xc = f->H1 = f->H2 = f->gOb = f->dpb = nullptr;
  f->rowv = f->batchbuf = nullptr;
  f->cap = 0;
}

int ensure_ws(pes_flow* f, int64_t n) {
  const int64_t Mp = pad_rows(n);
  if (Mp <= f->cap) return PES_OK;
  free_ws(f);
  const int64_t L = kLayers;
  bool ok = hipMalloc(&f->x, sizeof(float) * Mp * kD) == hipSuccess &&
            hipMalloc(&f->logdet, sizeof(float) * Mp) == hipSuccess &&
            hipMalloc(&f->xin, sizeof(float) * L * Mp * kD) == hipSuccess &&
            hipMalloc(&f->O, sizeof(float) * L * Mp * kPad) == hipSuccess &&
            hipMalloc(&f->Xc, sizeof(__bf16) * L * Mp * kPad) == hipSuccess &&
            hipMalloc(&f->H1, sizeof(__bf16) * L * Mp * kHid) == hipSuccess &&
            hipMalloc(&f->H2, sizeof(__bf16) * L * Mp * kHid) == hipSuccess &&
            hipMalloc(&f->gy, sizeof(float) * Mp * kD) == hipSuccess &&
            hipMalloc(&f->gx, sizeof(float) * Mp * kD) == hipSuccess &&
            hipMalloc(&f->gOf, sizeof(float) * Mp * kPad) == hipSuccess &&
            hipMalloc(&f->gOb, sizeof(__bf16) * Mp * kPad) == hipSuccess &&
            hipMalloc(&f->dpf, sizeof(float) * 2 * Mp * kHid) == hipSuccess &&
            hipMalloc(&f->dpb, sizeof(__bf16) * 2 * Mp * kHid) == hipSuccess &&
            hipMalloc(&f->dXc, sizeof(float) * Mp * kPad) == hipSuccess &&
            hipMalloc(&f->rowv, sizeof(double) * Mp) == hipSuccess &&
            hipMalloc(&f->batchbuf, sizeof(double) * Mp * kD) == hipSuccess;
  if (!ok) {
    free_ws(f);
    snprintf(f->err, sizeof(f->err), "flow workspace for %lld rows failed", (long long)Mp);
    return PES_ENOMEM;
  }
  f->cap = Mp;
  ++f->gen;
  return PES_OK;
}

const __bf16* W1b(const pes_flow* f, int l) { return f->wb + (int64_t)l * kLayerW; }
const __bf16* W2b(const pes_flow* f, int l) { return f->wb + (int64_t)l * kLayerW + kPad * kHid; }
const __bf16* W3b(const pes_flow* f, int l) { return f->wb + (int64_t)l * kLayerW + kPad * kHid + kHid * kHid; }
const float* b1p(const pes_flow* f, int l) { return f->bp + (int64_t)l * kLayerB; }
const float* b2p(const pes_flow* f, int l) { return f->bp + (int64_t)l * kLayerB + kHid; }
const float* b3p(const pes_flow* f, int l) { return f->bp + (int64_t)l * kLayerB + 2 * kHid; }

// Conditioner network of layer l on the rows of x: Xc -> H1 -> H2 -> O.
int net_forward(pes_flow* f, int l, int64_t Mp, int slot, hipStream_t s) {
  const int64_t so = (int64_t)slot * Mp;
  __bf16* Xc = f->Xc + so * kPad;
  __bf16* H1 = f->H1 + so * kHid;
  __bf16* H2 = f->H2 + so * kHid;
  float* O = f->O + so * kPad;
  hipLaunchKernelGGL(gather_kernel, dim3(nblk(Mp * kPad, 256)), dim3(256), 0, s, f->x, Xc, Mp, f->L[l]);
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.M = (int)Mp;
  // H1 = relu(Xc W1 + b1): B(n = out, k = in) = W1[in][out]
  g.A = Xc; g.lda = kPad; g.B = W1b(f, l); g.ldb = kHid; g.N = kHid; g.K = kPad;
  g.bias = b1p(f, l); g.Cb = H1; g.ldcb = kHid;
  FL_HIP(f, (gemm<true, false, EPI_BIAS_RELU_BF16>(g, s)));
  g.A = H1; g.lda = kHid; g.B = W2b(f, l); g.ldb = kHid; g.N = kHid; g.K = kHid;
  g.bias = b2p(f, l); g.Cb = H2; g.ldcb = kHid;
  FL_HIP(f, (gemm<true, false, EPI_BIAS_RELU_BF16>(g, s)));
  g.A = H2; g.lda = kHid; g.B = W3b(f, l); g.ldb = kPad; g.N = kPad; g.K = kHid;
  g.bias = b3p(f, l); g.C = O; g.ldc = kPad; g.Cb = nullptr;
  FL_HIP(f, (gemm<true, false, EPI_BIAS_F32>(g, s)));
  return PES_OK;
}

// Normalizing pass over f->x (standardized rows); store: keep every layer's
// input and activations for the backward pass.
// Where a probe call wants the state after every layer (null on every other path).
struct StateProbe {
  int64_t n;
  float* states;
  float* logdet;
  float* acts;    // may be null
};

int probe_state(pes_flow* f, const StateProbe* pr, int k, hipStream_t s) {
  if (!pr) return PES_OK;
  hipLaunchKernelGGL(copy_state_kernel, dim3(nblk(pr->n * kD, 256)), dim3(256), 0, s, f->x, f->logdet, pr->n, k,
                     pr->states, pr->logdet);
  FL_HIP(f, hipGetLastError());
  return PES_OK;
}

int probe_acts(pes_flow* f, const StateProbe* pr, int64_t Mp, hipStream_t s);

int pass_forward(pes_flow* f, int64_t Mp, bool store, hipStream_t s, const StateProbe* pr = nullptr) {
  int rc = probe_state(f, pr, 0, s);
  if (rc != PES_OK) return rc;
  for (int l = 0; l < kLayers; ++l) {
    const int slot = store || pr ? l : 0;    // a probe keeps every layer's activations
    rc = net_forward(f, l, Mp, slot, s);
    if (rc != PES_OK) return rc;
    hipLaunchKernelGGL(couple_kernel, dim3(nblk(Mp, 256)), dim3(256), 0, s, f->x, f->O + (int64_t)slot * Mp * kPad,
                       f->logdet, store ? f->xin + (int64_t)l * Mp * kD : nullptr, Mp, f->L[l], 0);
    FL_HIP(f, hipGetLastError());
    rc = probe_state(f, pr, l + 1, s);
    if (rc != PES_OK) return rc;
  }
  return probe_acts(f, pr, Mp, s);
}

int probe_acts(pes_flow* f, const StateProbe* pr, int64_t Mp, hipStream_t s) {
  if (!pr || !pr->acts) return PES_OK;
  hipLaunchKernelGGL(copy_acts_kernel, dim3(nblk((int64_t)kLayers * pr->n * kActCols, 256)), dim3(256), 0, s, f->Xc,
                     f->H1, f->H2, f->O, Mp, pr->n, pr->acts);
  FL_HIP(f, hipGetLastError());
  return PES_OK;
}

int pass_inverse(pes_flow* f, int64_t Mp, hipStream_t s, const StateProbe* pr = nullptr) {
  int rc = probe_state(f, pr, 0, s);
  if (rc != PES_OK) return rc;
  for (int l = kLayers - 1; l >= 0; --l) {
    const int slot = pr ? l : 0;    // a probe keeps every layer's activations
    rc = net_forward(f, l, Mp, slot, s);
    if (rc != PES_OK) return rc;
    hipLaunchKernelGGL(couple_kernel, dim3(nblk(Mp, 256)), dim3(256), 0, s, f->x, f->O + (int64_t)slot * Mp * kPad,
                       f->logdet, (float*)nullptr, Mp, f->L[l], 1);
    FL_HIP(f, hipGetLastError());
    rc = probe_state(f, pr, kLayers - l, s);
    if (rc != PES_OK) return rc;
  }
  return probe_acts(f, pr, Mp, s);
}

// Backward of the mean NLL over the first n rows after pass_forward(store):
// gradient into f->G, NLL into nll (device, may be null).
int pass_backward(pes_flow* f, int64_t n, int64_t Mp, double* nll, hipStream_t s) {
  hipLaunchKernelGGL(nll_seed_kernel, dim3(nblk(Mp, 256)), dim3(256), 0, s, f->x, f->logdet, n, Mp, f->gy, f->rowv);
  if (nll) hipLaunchKernelGGL(sum_rows_kernel, dim3(1), dim3(256), 0, s, f->rowv, Mp, nll);
  FL_HIP(f, hipGetLastError());
  float* dpf2 = f->dpf;
  float* dpf1 = f->dpf + Mp * kHid;
  __bf16* dpb2 = f->dpb;
  __bf16* dpb1 = f->dpb + Mp * kHid;
  for (int l = kLayers - 1; l >= 0; --l) {
    const LayerSpec& ls = f->L[l];
    const int64_t so = (int64_t)l * Mp;
    const __bf16* Xc = f->Xc + so * kPad;
    const __bf16* H1 = f->H1 + so * kHid;
    const __bf16* H2 = f->H2 + so * kHid;
    const TensorDesc* td = &f->tt.t[6 * l];   // W1, b1, W2, b2, W3, b3
    hipLaunchKernelGGL(couple_bwd_kernel, dim3(nblk(Mp, 256)), dim3(256), 0, s, f->xin + so * kD, f->O + so * kPad,
                       f->gy, f->gx, f->gOf, f->gOb, n, Mp, ls);
    FL_HIP(f, hipGetLastError());
    GemmArgs g;
    // dW3[i][o] = sum_m H2[m][i] gO[m][o]
    memset(&g, 0, sizeof(g));
    g.A = H2; g.lda = kHid; g.B = f->gOb; g.ldb = kPad; g.M = kHid; g.N = kPad; g.K = (int)Mp;
    g.C = f->G + td[4].off; g.ldc = 2 * ls.nt; g.m_valid = kHid; g.n_valid = 2 * ls.nt; g.part = f->kpart;
    FL_HIP(f, (gemm<false, false, EPI_F32>(g, s)));
    hipLaunchKernelGGL(colsum_kernel, dim3(2 * ls.nt), dim3(256), 0, s, f->gOf, (int64_t)kPad, Mp, f->G + td[5].off);
    // dpre2 = (gO W3^T) * [H2 > 0]: B(n = i, k = o) = W3[i][o]
    memset(&g, 0, sizeof(g));
    g.A = f->gOb; g.lda = kPad; g.B = W3b(f, l); g.ldb = kPad; g.M = (int)Mp; g.N = kHid; g.K = kPad;
    g.mask = H2; g.ldm = kHid; g.C = dpf2; g.ldc = kHid; g.Cb = dpb2; g.ldcb = kHid;
    FL_HIP(f, (gemm<true, true, EPI_MASK>(g, s)));
    // dW2 = H1^T dpre2, db2
    memset(&g, 0, sizeof(g));
    g.A = H1; g.lda = kHid; g.B = dpb2; g.ldb = kHid; g.M = kHid; g.N = kHid; g.K = (int)Mp;
    g.C = f->G + td[2].off; g.ldc = kHid; g.m_valid = kHid; g.n_valid = kHid; g.part = f->kpart;
    FL_HIP(f, (gemm<false, false, EPI_F32>(g, s)));
    hipLaunchKernelGGL(colsum_kernel, dim3(kHid), dim3(256), 0, s, dpf2, (int64_t)kHid, Mp, f->G + td[3].off);
    // dpre1 = (dpre2 W2^T) * [H1 > 0]
    memset(&g, 0, sizeof(g));
    g.A = dpb2; g.lda = kHid; g.B = W2b(f, l); g.ldb = kHid; g.M = (int)Mp; g.N = kHid; g.K = kHid;
    g.mask = H1; g.ldm = kHid; g.C = dpf1; g.ldc = kHid; g.Cb = dpb1; g.ldcb = kHid;
    FL_HIP(f, (gemm<true, true, EPI_MASK>(g, s)));
    // dW1 = Xc^T dpre1 (rows i < n_C), db1
    memset(&g, 0, sizeof(g));
    g.A = Xc; g.lda = kPad; g.B = dpb1; g.ldb = kHid; g.M = kPad; g.N = kHid; g.K = (int)Mp;
    g.C = f->G + td[0].off; g.ldc = kHid; g.m_valid = ls.nc; g.n_valid = kHid; g.part = f->kpart;
    FL_HIP(f, (gemm<false, false, EPI_F32>(g, s)));
    hipLaunchKernelGGL(colsum_kernel, dim3(kHid), dim3(256), 0, s, dpf1, (int64_t)kHid, Mp, f->G + td[1].off);
    FL_HIP(f, hipGetLastError());
    if (l > 0) {
      // dXc = dpre1 W1^T: B(n = i, k = o) = W1[i][o]
      memset(&g, 0, sizeof(g));
      g.A = dpb1; g.lda = kHid; g.B = W1b(f, l); g.ldb = kHid; g.M = (int)Mp; g.N = kPad; g.K = kHid;
      g.C = f->dXc; g.ldc = kPad; g.m_valid = (int)Mp; g.n_valid = kPad;
      FL_HIP(f, (gemm<true, true, EPI_F32>(g, s)));
      hipLaunchKernelGGL(scatter_cond_kernel, dim3(nblk(Mp, 256)), dim3(256), 0, s, f->dXc, f->gx, Mp, ls);
      FL_HIP(f, hipGetLastError());
      std::swap(f->gy, f->gx);
    }
  }
  return PES_OK;
}

int refresh(pes_flow* f, bool update, float lr, hipStream_t s) {
  float c1 = 1.0f, c2 = 1.0f;
  const float b1 = 0.9f, b2 = 0.999f;
  if (update) {
    ++f->t_adam;
    c1 = (float)(1.0 / (1.0 - pow((double)b1, (double)f->t_adam)));
    c2 = (float)(1.0 / (1.0 - pow((double)b2, (double)f->t_adam)));
  }
  hipLaunchKernelGGL(adam_kernel, dim3(nblk(kHid * kHid, 256), kTensors), dim3(256), 0, s, f->P, f->G, f->m1, f->m2,
                     f->wb, f->bp, f->tt, update ? 1 : 0, lr, b1, b2, c1, c2, 1e-8f);
  FL_HIP(f, hipGetLastError());
  return PES_OK;
}

void build_spec(pes_flow* f) {
  int64_t off = 0;
  for (int l = 0; l < kLayers; ++l) {
    const int p = l / 2;
    int in_c[kD], nc = 0, nt = 0;
    for (int i = 0; i < kD; ++i) in_c[i] = ((i + 3 * p) % kD) < 6;
    if (l % 2)
      for (int i = 0; i < kD; ++i) in_c[i] = !in_c[i];
    LayerSpec& ls = f->L[l];
    for (int i = 0; i < kD; ++i) {
      if (in_c[i]) ls.cond[nc++] = i;
      else ls.trans[nt++] = i;
    }
    ls.nc = nc;
    ls.nt = nt;
    const int rows[6] = {nc, 1, kHid, 1, kHid, 1};
    const int cols[6] = {kHid, kHid, kHid, kHid, 2 * nt, 2 * nt};
    const int64_t wo[6] = {0, -1, kPad * kHid, -1, kPad * kHid + kHid * kHid, -1};
    const int64_t bo[6] = {-1, 0, -1, kHid, -1, 2 * kHid};
    const int ldw[6] = {kHid, 0, kHid, 0, kPad, 0};
    for (int q = 0; q < 6; ++q) {
      TensorDesc& d = f->tt.t[6 * l + q];
      d.off = off;
      d.rows = rows[q];
      d.cols = cols[q];
      d.woff = wo[q] >= 0 ? (int64_t)l * kLayerW + wo[q] : -1;
      d.boff = bo[q] >= 0 ? (int64_t)l * kLayerB + bo[q] : -1;
      d.ldw = ldw[q];
      off += (int64_t)rows[q] * cols[q];
    }
  }
  f->np = off;
}

void destroy(pes_flow* f) {
  free_ws(f);
  (void)hipFree(f->P);
  (void)hipFree(f->G);
  (void)hipFree(f->m1);
  (void)hipFree(f->m2);
  (void)hipFree(f->wb);
  (void)hipFree(f->bp);
  (void)hipFree(f->mom);
  (void)hipFree(f->kpart);
  delete f;
}

// mu [11], L [11][11] row-major (entries above the diagonal ignored).
int set_affine(pes_flow* f, const double* mu, const double* L) {
  double ls = 0.0;
  for (int k = 0; k < kD; ++k) {
    if (!std::isfinite(mu[k]) || !(L[k * kD + k] > 0.0)) return PES_EINVAL;
    for (int m = 0; m <= k; ++m)
      if (!std::isfinite(L[k * kD + m])) return PES_EINVAL;
    ls += log(L[k * kD + k]);
  }
  for (int k = 0; k < kD; ++k) {
    f->nm.mu[k] = mu[k];
    for (int m = 0; m < kD; ++m) f->nm.L[k][m] = m <= k ? L[k * kD + m] : 0.0;
  }
  f->lsig = ls;
  return PES_OK;
}

int set_norm(pes_flow* f, const double* mu, const double* sigma) {
  double L[kD * kD] = {0.0};
  for (int k = 0; k < kD; ++k) {
    if (!(sigma[k] > 0.0)) return PES_EINVAL;
    L[k * kD + k] = sigma[k];
  }
  return set_affine(f, mu, L);
}

// Lower Cholesky factor of the symmetric matrix C (lower triangle used); false
// if C is not positive definite.
bool cholesky(const double* C, double* L) {
  for (int i = 0; i < kD * kD; ++i) L[i] = 0.0;
  for (int k = 0; k < kD; ++k) {
    double d = C[k * kD + k];
    for (int m = 0; m < k; ++m) d -= L[k * kD + m] * L[k * kD + m];
    if (!(d > 0.0)) return false;
    L[k * kD + k] = sqrt(d);
    for (int i = k + 1; i < kD; ++i) {
      double v = C[i * kD + k];
      for (int m = 0; m < k; ++m) v -= L[i * kD + m] * L[k * kD + m];
      L[i * kD + k] = v / L[k * kD + k];
    }
  }
  return true;
}

}  // namespace

namespace pes {

int flow_reserve(pes_flow* f, int64_t n) { return ensure_ws(f, n); }

uint64_t flow_generation(const pes_flow* f) { return f->gen; }

int flow_forward(pes_flow* f, const double* theta, int64_t n, double* z, double* logq, hipStream_t s,
                 const StateProbe* pr) {
  if (n <= 0) return PES_OK;
  const int64_t Mp = pad_rows(n);
  if (Mp > f->cap) return PES_ESTATE;
  hipLaunchKernelGGL(standardize_kernel, dim3(nblk(Mp, 256)), dim3(256), 0, s, theta, n, Mp, f->nm, f->x,
                     f->logdet);
  FL_HIP(f, hipGetLastError());
  int rc = pass_forward(f, Mp, false, s, pr);
  if (rc != PES_OK) return rc;
  hipLaunchKernelGGL(logq_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, f->x, f->logdet, n, f->lsig, f->tau, logq,
                     z);
  FL_HIP(f, hipGetLastError());
  return PES_OK;
}

int flow_inverse(pes_flow* f, const double* z, int64_t n, double* theta, double* logdet, hipStream_t s,
                 const StateProbe* pr) {
  if (n <= 0) return PES_OK;
  const int64_t Mp = pad_rows(n);
  if (Mp > f->cap) return PES_ESTATE;
  hipLaunchKernelGGL(load_latent_kernel, dim3(nblk(Mp * kD, 256)), dim3(256), 0, s, z, n, Mp, f->tau, f->x,
                     f->logdet);
  FL_HIP(f, hipGetLastError());
  int rc = pass_inverse(f, Mp, s, pr);
  if (rc != PES_OK) return rc;
  hipLaunchKernelGGL(unstandardize_kernel, dim3(nblk(n, 256)), dim3(256), 0, s, f->x, f->logdet, n, f->nm,
                     theta, logdet);
  FL_HIP(f, hipGetLastError());
  return PES_OK;
}

int flow_forward(pes_flow* f, const double* theta, int64_t n, double* z, double* logq, hipStream_t s) {
  return flow_forward(f, theta, n, z, logq, s, nullptr);
}

int flow_inverse(pes_flow* f, const double* z, int64_t n, double* theta, double* logdet, hipStream_t s) {
  return flow_inverse(f, z, n, theta, logdet, s, nullptr);
}

}  // namespace pes

extern "C" {

int pes_flow_create(uint64_t seed, pes_flow** out) {
  if (!out) return PES_EINVAL;
  *out = nullptr;
  pes_flow* f = new (std::nothrow) pes_flow();
  if (!f) return PES_ENOMEM;
  build_spec(f);
  const int64_t np = f->np;
  if (hipMalloc(&f->P, sizeof(float) * np) != hipSuccess || hipMalloc(&f->G, sizeof(float) * np) != hipSuccess ||
      hipMalloc(&f->m1, sizeof(float) * np) != hipSuccess || hipMalloc(&f->m2, sizeof(float) * np) != hipSuccess ||
      hipMalloc(&f->wb, sizeof(__bf16) * kLayers * kLayerW) != hipSuccess ||
      hipMalloc(&f->bp, sizeof(float) * kLayers * kLayerB) != hipSuccess ||
      hipMalloc(&f->mom, sizeof(double) * (kD + kD * kD)) != hipSuccess ||
      hipMalloc(&f->kpart, sizeof(float) * kMaxSplit * kHid * kHid) != hipSuccess) {
    destroy(f);
    return PES_ENOMEM;
  }
  // padding of the BF16 and bias copies stays zero
  if (hipMemset(f->wb, 0, sizeof(__bf16) * kLayers * kLayerW) != hipSuccess ||
      hipMemset(f->bp, 0, sizeof(float) * kLayers * kLayerB) != hipSuccess ||
      hipMemset(f->G, 0, sizeof(float) * np) != hipSuccess || hipMemset(f->m1, 0, sizeof(float) * np) != hipSuccess ||
      hipMemset(f->m2, 0, sizeof(float) * np) != hipSuccess) {
    destroy(f);
    return PES_EHIP;
  }
  // Kaiming-uniform hidden layers, a small output layer (near-identity map), zero biases
  float* h = new (std::nothrow) float[np]();
  if (!h) {
    destroy(f);
    return PES_ENOMEM;
  }
  std::mt19937_64 rng(seed);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  for (int l = 0; l < kLayers; ++l) {
    const TensorDesc* td = &f->tt.t[6 * l];
    for (int q : {0, 2, 4}) {
      const double bound = q == 4 ? 1e-2 / sqrt((double)kHid) : sqrt(6.0 / td[q].rows);
      for (int64_t i = 0; i < (int64_t)td[q].rows * td[q].cols; ++i) h[td[q].off + i] = (float)(bound * U(rng));
    }
  }
  const hipError_t e = hipMemcpy(f->P, h, sizeof(float) * np, hipMemcpyHostToDevice);
  delete[] h;
  if (e != hipSuccess) {
    destroy(f);
    return PES_EHIP;
  }
  double mu[kD], sg[kD];
  for (int k = 0; k < kD; ++k) {
    mu[k] = 0.0;
    sg[k] = 1.0;
  }
  set_norm(f, mu, sg);
  if (refresh(f, false, 0.0f, nullptr) != PES_OK || hipDeviceSynchronize() != hipSuccess) {
    destroy(f);
    return PES_EHIP;
  }
  *out = f;
  return PES_OK;
}

int pes_flow_destroy(pes_flow* f) {
  if (!f) return PES_EINVAL;
  (void)hipDeviceSynchronize();
  destroy(f);
  return PES_OK;
}

int64_t pes_flow_num_params(void) {
  pes_flow tmp;
  build_spec(&tmp);
  return tmp.np;
}

int pes_flow_set_params(pes_flow* f, const float* params, void* stream) {
  if (!f || !params) return PES_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  FL_HIP(f, hipMemcpyAsync(f->P, params, sizeof(float) * f->np, hipMemcpyDeviceToDevice, s));
  FL_HIP(f, hipMemsetAsync(f->m1, 0, sizeof(float) * f->np, s));
  FL_HIP(f, hipMemsetAsync(f->m2, 0, sizeof(float) * f->np, s));
  f->t_adam = 0;
  return refresh(f, false, 0.0f, s);
}

int pes_flow_get_params(pes_flow* f, float* params, void* stream) {
  if (!f || !params) return PES_EINVAL;
  FL_HIP(f, hipMemcpyAsync(params, f->P, sizeof(float) * f->np, hipMemcpyDeviceToDevice, (hipStream_t)stream));
  return PES_OK;
}

int pes_flow_set_norm(pes_flow* f, const double* mu, const double* sigma) {
  if (!f || !mu || !sigma) return PES_EINVAL;
  return set_norm(f, mu, sigma);
}

int pes_flow_set_temperature(pes_flow* f, double tau) {
  if (!f || !(tau > 0.0) || !std::isfinite(tau)) return PES_EINVAL;
  f->tau = tau;
  return PES_OK;
}

int pes_flow_set_affine(pes_flow* f, const double* mu, const double* L) {
  if (!f || !mu || !L) return PES_EINVAL;
  return set_affine(f, mu, L);
}

int pes_flow_get_affine(pes_flow* f, double* mu, double* L) {
  if (!f || !mu || !L) return PES_EINVAL;
  for (int k = 0; k < kD; ++k) {
    mu[k] = f->nm.mu[k];
    for (int m = 0; m < kD; ++m) L[k * kD + m] = f->nm.L[k][m];
  }
  return PES_OK;
}

int pes_flow_forward(pes_flow* f, const double* theta, int64_t n, double* z, double* logq, void* stream) {
  if (!f || n < 0 || (n > 0 && (!theta || !logq))) return PES_EINVAL;
  int rc = ensure_ws(f, n);
  if (rc != PES_OK) return rc;
  return pes::flow_forward(f, theta, n, z, logq, (hipStream_t)stream);
}

int pes_flow_inverse(pes_flow* f, const double* z, int64_t n, double* theta, double* logdet, void* stream) {
  if (!f || n < 0 || (n > 0 && (!z || !theta))) return PES_EINVAL;
  int rc = ensure_ws(f, n);
  if (rc != PES_OK) return rc;
  return pes::flow_inverse(f, z, n, theta, logdet, (hipStream_t)stream);
}

int pes_flow_probe(pes_flow* f, const double* in, int64_t n, int inverse, double* out, double* lq,
                   float* states, float* logdet, float* acts, void* stream) {
  if (!f || n < 0 || (inverse != 0 && inverse != 1)) return PES_EINVAL;
  if (n > 0 && (!in || !out || !states || !logdet || (!inverse && !lq))) return PES_EINVAL;
  int rc = ensure_ws(f, n);
  if (rc != PES_OK) return rc;
  const StateProbe pr{n, states, logdet, acts};
  return inverse ? pes::flow_inverse(f, in, n, out, lq, (hipStream_t)stream, &pr)
                 : pes::flow_forward(f, in, n, out, lq, (hipStream_t)stream, &pr);
}

int pes_flow_nll_grad(pes_flow* f, const double* theta, int64_t n, double* nll, float* grad, void* stream) {
  if (!f || n <= 0 || !theta || !grad) return PES_EINVAL;
  int rc = ensure_ws(f, n);
  if (rc != PES_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t Mp = pad_rows(n);
  hipLaunchKernelGGL(standardize_kernel, dim3(nblk(Mp, 256)), dim3(256), 0, s, theta, n, Mp, f->nm, f->x,
                     f->logdet);
  FL_HIP(f, hipGetLastError());
  rc = pass_forward(f, Mp, true, s);
  if (rc != PES_OK) return rc;
  rc = pass_backward(f, n, Mp, nll, s);
  if (rc != PES_OK) return rc;
  FL_HIP(f, hipMemcpyAsync(grad, f->G, sizeof(float) * f->np, hipMemcpyDeviceToDevice, s));
  return PES_OK;
}

int pes_flow_adam_step(pes_flow* f, const float* grad, float lr, void* stream) {
  if (!f || !(lr >= 0.0f)) return PES_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (grad) FL_HIP(f, hipMemcpyAsync(f->G, grad, sizeof(float) * f->np, hipMemcpyDeviceToDevice, s));
  return refresh(f, true, lr, s);
}

int pes_flow_fit(pes_flow* f, const double* samples, int64_t n, int64_t steps, int64_t batch, float lr,
                 uint64_t seed, int standardize, double* loss, void* stream) {
  if (!f || !samples || n < 2 || steps < 0 || batch < 1 || batch > n || !(lr > 0.0f)) return PES_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int rc = ensure_ws(f, batch);
  if (rc != PES_OK) return rc;
  if (standardize) {   // whitening by the samples' mean and covariance (Cholesky factor)
    hipLaunchKernelGGL(mean_kernel, dim3(kD), dim3(256), 0, s, samples, n, f->mom);
    hipLaunchKernelGGL(cov_kernel, dim3(kD * kD), dim3(256), 0, s, samples, n, f->mom);
    FL_HIP(f, hipGetLastError());
    double h[kD + kD * kD], L[kD * kD];
    FL_HIP(f, hipMemcpyAsync(h, f->mom, sizeof(h), hipMemcpyDeviceToHost, s));
    FL_HIP(f, hipStreamSynchronize(s));
    if (!cholesky(h + kD, L) || set_affine(f, h, L) != PES_OK) {
      snprintf(f->err, sizeof(f->err), "the training samples' covariance is not positive definite");
      return PES_EINVAL;
    }
  }
  const int64_t Mp = pad_rows(batch);
  for (int64_t it = 0; it < steps; ++it) {
    hipLaunchKernelGGL(batch_kernel, dim3(nblk(batch, 256)), dim3(256), 0, s, samples, n, batch, seed,
                       (uint64_t)it, f->batchbuf);
    hipLaunchKernelGGL(standardize_kernel, dim3(nblk(Mp, 256)), dim3(256), 0, s, f->batchbuf, batch, Mp, f->nm,
                       f->x, f->logdet);
    FL_HIP(f, hipGetLastError());
    rc = pass_forward(f, Mp, true, s);
    if (rc != PES_OK) return rc;
    rc = pass_backward(f, batch, Mp, loss ? loss + it : nullptr, s);
    if (rc != PES_OK) return rc;
    const float lr_t = (float)(0.5 * lr * (1.0 + cos(M_PI * (double)it / (double)steps)));   // cosine decay
    rc = refresh(f, true, lr_t, s);
    if (rc != PES_OK) return rc;
  }
  return PES_OK;
}

const char* pes_flow_last_error(pes_flow* f) { return f ? f->err : "null flow"; }

}  // extern "C"
