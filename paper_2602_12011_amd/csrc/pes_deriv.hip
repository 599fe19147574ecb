// Derivative kernels of libpes (gfx950): the reverse-mode gradient
// (adj_kernel), the forward-mode Fisher matrix (fisher_dense_body: one (bin,
// parameter) tangent per lane, the J^T J contraction on the FP64 matrix cores)
// and gradient (forward_grad_body), and their per-walker reductions.  Walker
// tangents come from setup_tan_kernel (pes_kernels.hip).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pes_adjoint.hpp"
#include "pes_eval.hpp"
#include "pes_launch.hpp"

namespace pes {

// ---------------------------------------------------------------- derivatives
__device__ __forceinline__ int64_t active_bins(double fmx, double f0, double df, int64_t N) {
  double nb = ceil((fmx - f0) / df) + 1.0;
  nb = fmin(fmax(nb, 0.0), (double)N);
  return (int64_t)nb;
}

// Exact Kepler orbits in the tangent kernels: the walker's projected series
// derivatives in the three sky angles for every detector, staged in LDS
// ([det][angle][KW_STRIDE], then one zero row for the other directions).
constexpr int kKwtRows = kMaxDet * 3;
__device__ __forceinline__ void stage_kw_tangents(const JacArgs& A, int b, double* kwt_s) {
  const double* __restrict__ src = A.wkept + (int64_t)b * A.n_det * 3 * KW_STRIDE;
  const int n = A.n_det * 3 * KW_STRIDE;
  for (int i = threadIdx.x; i < (kKwtRows + 1) * KW_STRIDE; i += blockDim.x) kwt_s[i] = i < n ? src[i] : 0.0;
}
// This lane's accessor of a heliocentric detector's series (direction p).
__device__ __forceinline__ KwLane kw_lane(const JacArgs& A, int b, int det, int p, const double* kwt_s) {
  const int row = (p >= 7 && p <= 9) ? det * 3 + (p - 7) : kKwtRows;
  return KwLane{A.wkep + ((int64_t)b * A.n_det + det) * KW_STRIDE, kwt_s + row * KW_STRIDE};
}

// Dual-number channels of one (bin, detector) for the lane's direction p.
template <bool LS, bool KEP>
__device__ __forceinline__ ChanT<Dual<1>> eval_tangent(const TanTabLane& T, const JacArgs& A, const DetParams& P,
                                                       int b, int det, int p, const double* kwt_s,
                                                       const BinRegs& br, double a, double zr, double zi) {
  if (P.kind == 2)
    return eval_channels_t<true, LS, 1, Dual<1>>(T, det, A.plan, P.inv_year, P.inv_ptq, br, a, zr, zi);
  if constexpr (KEP)
    return eval_channels_t<false, LS, 1, Dual<1>, TanTabLane, NoProbe, true, KwLane>(
        T, det, A.plan, P.inv_year, P.inv_ptq, br, a, zr, zi, NoProbe(), kw_lane(A, b, det, p, kwt_s),
        A.kep + det * KV_STRIDE + KV_INVL);
  return eval_channels_t<false, LS, 1, Dual<1>>(T, det, A.plan, P.inv_year, P.inv_ptq, br, a, zr, zi);
}

// Forward-mode gradient (the cross-check of the reverse sweep), one (bin,
// parameter) pair per lane: lane l of a wavefront carries the tangent
// direction p = l % 16 (p < 11; the other five lanes contribute zeros) of bin
// l / 16 of its group of four bins and accumulates sum_r (D - W C)_r
// dC_r/dtheta_p; the p = 0 lanes also <d|h> and <h|h>, and the block reduces
// them to the per-tile partials of the gradient.  The walker's tangent table
// is staged in LDS once per block (the lanes read different directions of the
// same entry); the four wavefronts of a block take interleaved groups of the
// block's bin tile.
template <bool LS, bool KEP>
__device__ __forceinline__ void forward_grad_body(const double* __restrict__ bins, const double* __restrict__ tabs,
                                                  const double* __restrict__ wtab, const double* __restrict__ wtan,
                                                  double* __restrict__ partial, const JacArgs& A) {
  __shared__ double red[4][256];
  __shared__ double tan_s[W_STRIDE * kNParams];   // the walker's tangent table, 25 KiB
  __shared__ double kwt_s[KEP ? (kKwtRows + 1) * KW_STRIDE : 1];
  const int t = blockIdx.x;
  const int b = blockIdx.y;
  const double* __restrict__ wt = wtab + (int64_t)b * W_STRIDE;
  const double* __restrict__ wtn = wtan + (int64_t)b * W_STRIDE * kNParams;
  if (wt[W_VALID] == 0.0) return;
  const int64_t nact = active_bins(wt[W_FMAX], A.f0, A.df, A.N);
  const int64_t k0 = (int64_t)t * A.tile;
  if (k0 >= nact) return;
  for (int i = threadIdx.x; i < W_STRIDE * kNParams; i += 256) tan_s[i] = wtn[i];
  if (KEP) stage_kw_tangents(A, b, kwt_s);
  __syncthreads();
  const int64_t kend = k0 + A.tile < nact ? k0 + A.tile : nact;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int p = lane & 15, sub = lane >> 4;
  const bool pin = p < kNParams;
  const int64_t N = A.N;
  double gacc = 0.0, dh = 0.0, hh = 0.0;
  for (int64_t s0 = k0 + 4 * wv; s0 < kend; s0 += 16) {
    const int64_t k = s0 + sub;
    const bool in = pin && k < kend;
    const int64_t kk = k < kend ? k : kend - 1;
    BinRegs br;
    br.f = bins[B_F * N + kk];
    br.f13 = bins[B_F13 * N + kk];
    br.fm13 = bins[B_FM13 * N + kk];
    br.fm76 = bins[B_FM76 * N + kk];
    br.lnf = bins[B_LNF * N + kk];
    for (int det = 0; det < A.n_det; ++det) {
      const double* __restrict__ tb = tabs + (int64_t)det * T_NFIELDS * N;
      const double zr = tb[T_ZR * N + kk], zi = tb[T_ZI * N + kk], a = tb[T_A * N + kk];
      const double wA = in ? tb[T_WA * N + kk] : 0.0;
      const double wT = in ? tb[T_WT * N + kk] : 0.0;
      const DetParams& P = A.dt.p[det];
      const TanTabLane T{wt, tan_s, pin ? p : 0};
      const ChanT<Dual<1>> c = eval_tangent<LS, KEP>(T, A, P, b, det, pin ? p : 0, kwt_s, br, a, zr, zi);
      const double W[6] = {wA, wA, wA * (1.0 / 3.0), wA * (1.0 / 3.0), wT, wT};
      const double D[6] = {in ? tb[T_DAR * N + kk] : 0.0, in ? tb[T_DAI * N + kk] : 0.0,
                           in ? tb[T_DER * N + kk] : 0.0, in ? tb[T_DEI * N + kk] : 0.0,
                           in ? tb[T_DTR * N + kk] : 0.0, in ? tb[T_DTI * N + kk] : 0.0};
      const double cv[6] = {c.ar.v, c.ai.v, c.er.v, c.ei.v, c.tr.v, c.ti.v};
      const double cd[6] = {c.ar.d[0], c.ai.d[0], c.er.d[0], c.ei.d[0], c.tr.d[0], c.ti.d[0]};
      const bool first = p == 0;
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        gacc = fma(fma(-W[r], cv[r], D[r]), cd[r], gacc);
        dh = first ? fma(D[r], cv[r], dh) : dh;
        hh = first ? fma(W[r] * cv[r], cv[r], hh) : hh;
      }
    }
  }
  // lane (sub, p) of wave w holds its share of d l / d theta_p; <d|h>, <h|h>
  // sit in the p = 0 lanes.  Fixed-order sums over waves and sub-lanes.
  const int e = threadIdx.x;
  red[wv][lane] = gacc;
  red[wv][64 + lane] = dh;
  red[wv][128 + lane] = hh;
  __syncthreads();
  if (e < kNParams + 2) {
    const int base = e < kNParams ? 0 : (e == kNParams ? 64 : 128);
    const int col = e < kNParams ? e : 0;
    double sum = 0.0;
    for (int w = 0; w < 4; ++w)
      for (int q = 0; q < 4; ++q) sum += red[w][base + 16 * q + col];
    partial[((int64_t)t * A.B + b) * (kNParams + 2) + e] = sum;
  }
}

// Fisher matrix with every lane busy: the 11 tangent directions of a bin are
// spread over consecutive lanes, pair i = 64 r + lane of a wave's chunk of 64
// bins is (bin i / 11, direction i % 11), so eleven rounds of 64 lanes cover
// the chunk with no idle lane.  After each round the lanes write
// sqrt(W) dC_r/dtheta_p into a per-wave LDS ring of bins, and every complete
// group of four bins is read back in the 16 x 16 x 4 matrix-core layout
// (lane 16 sub + p: bin sub, direction p; p >= 11 reads zero) for the six
// products of the contraction.  A round completes floor(64 (r + 1) / 11) bins,
// so at most three complete bins wait for a group, six more complete in a
// round and one is partly written: twelve ring slots suffice.
constexpr int kRing = 12;

template <bool LS, bool KEP>
__device__ __forceinline__ void fisher_dense_body(const double* __restrict__ bins, const double* __restrict__ tabs,
                                                  const double* __restrict__ wtab, const double* __restrict__ wtan,
                                                  double* __restrict__ partial, const JacArgs& A) {
  __shared__ double tan_s[W_STRIDE * kNParams];             // the walker's tangent table, 25 KiB
  __shared__ double ring[4][kRing][6][kNParams];            // per wave; reused for the final sums
  __shared__ double kwt_s[KEP ? (kKwtRows + 1) * KW_STRIDE : 1];
  const int t = blockIdx.x;
  const int b = blockIdx.y;
  const double* __restrict__ wt = wtab + (int64_t)b * W_STRIDE;
  const double* __restrict__ wtn = wtan + (int64_t)b * W_STRIDE * kNParams;
  if (wt[W_VALID] == 0.0) return;
  const int64_t nact = active_bins(wt[W_FMAX], A.f0, A.df, A.N);
  const int64_t k0 = (int64_t)t * A.tile;
  if (k0 >= nact) return;
  for (int i = threadIdx.x; i < W_STRIDE * kNParams; i += 256) tan_s[i] = wtn[i];
  if (KEP) stage_kw_tangents(A, b, kwt_s);
  __syncthreads();
  const int64_t kend = k0 + A.tile < nact ? k0 + A.tile : nact;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int sub = lane >> 4, pq = lane & 15;
  const int64_t N = A.N;
  typedef double v4d __attribute__((ext_vector_type(4)));
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  double(*rw)[6][kNParams] = ring[wv];
  for (int det = 0; det < A.n_det; ++det) {   // each detector's channels are rows of their own
    const double* __restrict__ tb = tabs + (int64_t)det * T_NFIELDS * N;
    const DetParams& P = A.dt.p[det];
    for (int64_t c0 = k0 + 64 * wv; c0 < kend; c0 += 256) {   // this wave's chunks of 64 bins
      int used = 0;
      for (int r = 0; r < kNParams; ++r) {
        const int i = 64 * r + lane;
        const int bl = i / kNParams, p = i - kNParams * bl;
        const int64_t k = c0 + bl;
        const bool in = k < kend;
        const int64_t kk = in ? k : kend - 1;
        BinRegs br;
        br.f = bins[B_F * N + kk];
        br.f13 = bins[B_F13 * N + kk];
        br.fm13 = bins[B_FM13 * N + kk];
        br.fm76 = bins[B_FM76 * N + kk];
        br.lnf = bins[B_LNF * N + kk];
        const double zr = tb[T_ZR * N + kk], zi = tb[T_ZI * N + kk], a = tb[T_A * N + kk];
        const double sA = in ? sqrt(tb[T_WA * N + kk]) : 0.0;
        const double sT = in ? sqrt(tb[T_WT * N + kk]) : 0.0;
        const TanTabLane T{wt, tan_s, p};
        const ChanT<Dual<1>> c = eval_tangent<LS, KEP>(T, A, P, b, det, p, kwt_s, br, a, zr, zi);
        const double sE = sA * 0.5773502691896258;   // W_E = W_A / 3
        const double v[6] = {sA * c.ar.d[0], sA * c.ai.d[0], sE * c.er.d[0],
                             sE * c.ei.d[0], sT * c.tr.d[0], sT * c.ti.d[0]};
        const int slot = bl % kRing;
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int q = 0; q < 6; ++q) rw[slot][q][p] = v[q];
        __builtin_amdgcn_wave_barrier();
        // bins whose 11 directions are all written, contracted four at a time
        const int done = (64 * (r + 1)) / kNParams;
        for (; used + 4 <= done; used += 4) {
          const int bs = (used + sub) % kRing;
#pragma unroll
          for (int q = 0; q < 6; ++q) {
            const double x = pq < kNParams ? rw[bs][q][pq] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
          }
        }
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
  __syncthreads();
  double* red = &ring[0][0][0][0];   // [4 waves][256]
#pragma unroll
  for (int r = 0; r < 4; ++r) red[wv * 256 + 4 * lane + r] = acc[r];
  __syncthreads();
  // accumulator element e: lane e / 4, register e % 4 <-> (row 4 (e % 4) + (e / 4) / 16,
  // column (e / 4) % 16); the 11 x 11 block is kept, row-major
  const int e = threadIdx.x;
  const double sum = (red[e] + red[256 + e]) + (red[512 + e] + red[768 + e]);
  const int row = 4 * (e & 3) + ((e >> 2) >> 4), col = (e >> 2) & 15;
  if (row < kNParams && col < kNParams)
    partial[((int64_t)t * A.B + b) * (kNParams * kNParams) + row * kNParams + col] = sum;
}

// Three waves per SIMD for the dense Fisher body: with the detector entries
// loaded per geometry section (opaque_u in eval_channels_t) it fits 168
// registers with two spilled values (before that, 200; the third wave is
// worth 7% here); 3 blocks of 50 KiB of LDS per CU.  The gradient variant
// holds the residual as well and runs two without spilling.
template <bool LS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
    forward_fisher_kernel(const double* __restrict__ bins, const double* __restrict__ tabs,
                          const double* __restrict__ wtab, const double* __restrict__ wtan,
                          double* __restrict__ partial, JacArgs A) {
  fisher_dense_body<LS, false>(bins, tabs, wtab, wtan, partial, A);
}
template <bool LS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    forward_grad_kernel(const double* __restrict__ bins, const double* __restrict__ tabs,
                        const double* __restrict__ wtab, const double* __restrict__ wtan,
                        double* __restrict__ partial, JacArgs A) {
  forward_grad_body<LS, false>(bins, tabs, wtab, wtan, partial, A);
}
// The same on exact Kepler orbits (9 KiB more LDS for the series derivatives:
// two blocks per CU).
template <bool LS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    forward_fisher_kep_kernel(const double* __restrict__ bins, const double* __restrict__ tabs,
                              const double* __restrict__ wtab, const double* __restrict__ wtan,
                              double* __restrict__ partial, JacArgs A) {
  fisher_dense_body<LS, true>(bins, tabs, wtab, wtan, partial, A);
}
template <bool LS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
    forward_grad_kep_kernel(const double* __restrict__ bins, const double* __restrict__ tabs,
                            const double* __restrict__ wtab, const double* __restrict__ wtan,
                            double* __restrict__ partial, JacArgs A) {
  forward_grad_body<LS, true>(bins, tabs, wtab, wtan, partial, A);
}

// Reverse-mode gradient: for each (walker, bin, detector) one forward
// evaluation gives the channels and the weighted residual, adj_links turns it
// into link adjoints, and adj_unit recomputes and back-propagates every active
// mode, contracting table-entry adjoints with the setup's theta-derivatives.
template <bool LS, bool GEO, bool KEP = false>
__device__ __forceinline__ void adj_det(const double* __restrict__ bins, const double* __restrict__ tb,
                                        const double* __restrict__ wt, const double* __restrict__ wtn,
                                        const JacArgs& A, int det, int64_t k, bool in, double* g,
                                        double& dh, double& hh, double* __restrict__ ybs,
                                        const double* __restrict__ kw = nullptr,
                                        const double* __restrict__ kinv = nullptr) {
  const int64_t N = A.N;
  const int64_t kk = in ? k : N - 1;
  BinRegs br;
  br.f = bins[B_F * N + kk];
  br.f13 = bins[B_F13 * N + kk];
  br.fm13 = bins[B_FM13 * N + kk];
  br.fm76 = bins[B_FM76 * N + kk];
  br.lnf = bins[B_LNF * N + kk];
  const double zr = tb[T_ZR * N + kk], zi = tb[T_ZI * N + kk], a = tb[T_A * N + kk];
  const double wA = in ? tb[T_WA * N + kk] : 0.0;
  const double wT = in ? tb[T_WT * N + kk] : 0.0;
  double D[6];
  D[0] = in ? tb[T_DAR * N + kk] : 0.0;
  D[1] = in ? tb[T_DAI * N + kk] : 0.0;
  D[2] = in ? tb[T_DER * N + kk] : 0.0;
  D[3] = in ? tb[T_DEI * N + kk] : 0.0;
  D[4] = in ? tb[T_DTR * N + kk] : 0.0;
  D[5] = in ? tb[T_DTI * N + kk] : 0.0;
  const DetParams& P = A.dt.p[det];
  const Chan c =
      eval_channels<GEO, LS, 1, KEP, KwScalar>(wt, det, A.plan, P.inv_year, P.inv_ptq, br, a, zr, zi, KwScalar{kw}, kinv);
  dh = fma(D[0], c.ar, dh);
  dh = fma(D[1], c.ai, dh);
  dh = fma(D[2], c.er, dh);
  dh = fma(D[3], c.ei, dh);
  dh = fma(D[4], c.tr, dh);
  dh = fma(D[5], c.ti, dh);
  const double a2 = fma(c.ar, c.ar, c.ai * c.ai) + (1.0 / 3.0) * fma(c.er, c.er, c.ei * c.ei);
  const double t2 = fma(c.tr, c.tr, c.ti * c.ti);
  hh = fma(wA, a2, fma(wT, t2, hh));
  {   // the link adjoints wait in LDS (this lane's 12 slots) while the modes run
    double yb[3][4];
    adj_links(c, D, wA, wT, zr, zi, yb);
#pragma unroll
    for (int q = 0; q < 12; ++q) ybs[q] = yb[q / 4][q % 4];
  }
  const double ftc = frac_prod(br.f, wt[W_TC]);
  const double L3 = P.L * (1.0 / 3.0);
#pragma unroll 1
  for (int u = 0; u < A.plan.n_pairs; ++u)
    adj_unit<GEO, LS, true, KEP>(wt, wtn, det, A.plan.lead[u], A.plan.member[u], P.inv_year, P.inv_ptq, L3, br, a,
                                 ftc, ybs, g, kw, kinv);
#pragma unroll 1
  for (int u = A.plan.n_pairs; u < A.plan.n_units; ++u)
    adj_unit<GEO, LS, false, KEP>(wt, wtn, det, A.plan.lead[u], 0, P.inv_year, P.inv_ptq, L3, br, a, ftc, ybs, g,
                                  kw, kinv);
}

// The walker's tangents are staged in LDS in the compact layout (4.6 KiB,
// written once per walker by compact_tan_kernel): the contraction reads the
// mode entries' ones as wave-uniform LDS broadcasts, which keeps them out of
// the scalar registers and their spills (the walker table itself stays on
// scalar loads: staging it too moves the pressure into vector registers).
// Two waves per SIMD: the reverse sweep fits 254 registers (a couple of
// spilled values); one wave per SIMD leaves its long dependency chains exposed.
template <bool LS, bool KEP>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 2)))
    adj_kernel(const double* __restrict__ bins, const double* __restrict__ tabs,
               const double* __restrict__ wtab, const double* __restrict__ wtan,
               double* __restrict__ partial, JacArgs A) {
  __shared__ double tan_s[kTanSlots];
  __shared__ double yb_s[64 * 12];
  const int t = blockIdx.x;
  const int b = blockIdx.y;
  const double* __restrict__ wt = wtab + (int64_t)b * W_STRIDE;
  if (wt[W_VALID] == 0.0) return;
  const int64_t nact = active_bins(wt[W_FMAX], A.f0, A.df, A.N);
  const int64_t k0 = (int64_t)t * A.tile;
  if (k0 >= nact) return;
  const int lane = threadIdx.x;
  {
    const double* __restrict__ src = wtan + (int64_t)b * kTanSlots;
    for (int i = lane; i < kTanSlots; i += 64) tan_s[i] = src[i];
    __syncthreads();
  }
  const double* wtn = tan_s;
  const int64_t kend = k0 + A.tile < nact ? k0 + A.tile : nact;
  double g[kNParams + 3];
#pragma unroll
  for (int i = 0; i < kNParams + 3; ++i) g[i] = 0.0;
  double dh = 0.0, hh = 0.0;
  for (int64_t s0 = k0; s0 < kend; s0 += 64) {
    const int64_t k = s0 + lane;
    const bool in = k < kend;
    for (int det = 0; det < A.n_det; ++det) {
      const double* __restrict__ tb = tabs + (int64_t)det * T_NFIELDS * A.N;
      if (A.dt.p[det].kind == 2)
        adj_det<LS, true>(bins, tb, wt, wtn, A, det, k, in, g, dh, hh, yb_s + 12 * lane);
      else if (KEP)
        adj_det<LS, false, true>(bins, tb, wt, wtn, A, det, k, in, g, dh, hh, yb_s + 12 * lane,
                                 A.wkep + ((int64_t)b * A.n_det + det) * KW_STRIDE, A.kep + det * KV_STRIDE + KV_INVL);
      else
        adj_det<LS, false>(bins, tb, wt, wtn, A, det, k, in, g, dh, hh, yb_s + 12 * lane);
    }
  }
  {
    // the sky sums: g_J += (p.dk_J) S_a + (q.dk_J) S_b + (q.dp_J) S_c for
    // J = (lambda, beta, psi).  With the basis of sky_basis (k = -(cos b cos l,
    // cos b sin l, sin b), u = (-sin l, cos l, 0), v = (-sin b cos l,
    // -sin b sin l, cos b), p = cos psi u + sin psi v, q = -sin psi u + cos psi v):
    // dk/dl = -cos b u, dk/db = -v, dp/dl = cos psi (cos b k + sin b v) - sin psi sin b u,
    // dp/db = sin psi k, dp/dpsi = q; hence p.dk = (-cos b cos psi, -sin psi, 0),
    // q.dk = (cos b sin psi, -cos psi, 0), q.dp = (sin b, 0, 1).
    const double* th = A.theta + (int64_t)b * kNParams;
    const double sb = sin(th[8]), cb = cos(th[8]), sps = sin(th[9]), cps = cos(th[9]);
    g[7] = fma(-cb * cps, g[kNParams], fma(cb * sps, g[kNParams + 1], fma(sb, g[kNParams + 2], g[7])));
    g[8] = fma(-sps, g[kNParams], fma(-cps, g[kNParams + 1], g[8]));
    g[9] += g[kNParams + 2];
  }
  double red[kNParams + 2];
#pragma unroll
  for (int i = 0; i < kNParams; ++i) red[i] = wave_sum_dpp(g[i]);
  red[kNParams] = wave_sum_dpp(dh);
  red[kNParams + 1] = wave_sum_dpp(hh);
  if (lane == 0) {
    double* p = partial + ((int64_t)t * A.B + b) * (kNParams + 2);
#pragma unroll
    for (int i = 0; i < kNParams + 2; ++i) p[i] = red[i];
  }
}

// The compact tangent table of each walker (one block of 64 per walker).
__global__ void __launch_bounds__(64) compact_tan_kernel(const double* __restrict__ wtan, double* __restrict__ wtanc) {
  const int b = blockIdx.x;
  compact_tangents(wtan + (int64_t)b * W_STRIDE * kNParams, wtanc + (int64_t)b * kTanSlots, threadIdx.x, 64);
}

// Per walker, tiles summed in order.  logl = <d|h> - <h|h>/2 - <d|d>/2.
__global__ void grad_finalize_kernel(const double* __restrict__ partial, const double* __restrict__ wtab,
                                     const double* __restrict__ dd, JacArgs A, double* __restrict__ logl,
                                     double* __restrict__ grad) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= A.B) return;
  const double* wt = wtab + (int64_t)b * W_STRIDE;
  if (wt[W_VALID] == 0.0) {
    if (logl) logl[b] = -INFINITY;
    for (int i = 0; i < kNParams; ++i) grad[(int64_t)b * kNParams + i] = 0.0;
    return;
  }
  const int64_t nact = active_bins(wt[W_FMAX], A.f0, A.df, A.N);
  const int nt = (int)((nact + A.tile - 1) / A.tile);
  double s[kNParams + 2];
  for (int i = 0; i < kNParams + 2; ++i) s[i] = 0.0;
  for (int t = 0; t < nt; ++t) {
    const double* p = partial + ((int64_t)t * A.B + b) * (kNParams + 2);
    for (int i = 0; i < kNParams + 2; ++i) s[i] += p[i];
  }
  for (int i = 0; i < kNParams; ++i) grad[(int64_t)b * kNParams + i] = s[i];
  if (logl) logl[b] = (s[kNParams] - 0.5 * s[kNParams + 1]) - 0.5 * dd[0];
}

// Fisher matrix: the per-tile 11 x 11 blocks summed in tile order.
__global__ void fisher_finalize_kernel(const double* __restrict__ partial, const double* __restrict__ wtab,
                                       JacArgs A, double* __restrict__ F) {
  const int b = blockIdx.x;
  const int e = threadIdx.x;   // row * 11 + column
  if (e >= kNParams * kNParams) return;
  const double* wt = wtab + (int64_t)b * W_STRIDE;
  double s = 0.0;
  if (wt[W_VALID] != 0.0) {
    const int64_t nact = active_bins(wt[W_FMAX], A.f0, A.df, A.N);
    const int nt = (int)((nact + A.tile - 1) / A.tile);
    for (int t = 0; t < nt; ++t) s += partial[((int64_t)t * A.B + b) * (kNParams * kNParams) + e];
  } else {
    s = NAN;
  }
  F[(int64_t)b * kNParams * kNParams + e] = s;
}

hipError_t launch_grad(const double* bins, const double* tabs, const double* wtab, const double* wtan,
                       double* partial, const double* dd, const JacArgs& A, bool long_sinc, bool adjoint,
                       double* logl, double* grad, hipStream_t s) {
  const dim3 grid((unsigned)((A.N + A.tile - 1) / A.tile), (unsigned)A.B);
  const bool kep = A.wkep != nullptr;
  if (kep && (!A.kep || (!adjoint && !A.wkept))) return hipErrorInvalidValue;
  if (adjoint) {
    if (!A.theta) return hipErrorInvalidValue;
    // the compact tables follow the full ones of the batch in the same buffer
    double* wtanc = const_cast<double*>(wtan) + (int64_t)A.B * W_STRIDE * kNParams;
    hipLaunchKernelGGL(compact_tan_kernel, dim3((unsigned)A.B), dim3(64), 0, s, wtan, wtanc);
    if (long_sinc && kep)
      hipLaunchKernelGGL((adj_kernel<true, true>), grid, dim3(64), 0, s, bins, tabs, wtab, wtanc, partial, A);
    else if (long_sinc)
      hipLaunchKernelGGL((adj_kernel<true, false>), grid, dim3(64), 0, s, bins, tabs, wtab, wtanc, partial, A);
    else if (kep)
      hipLaunchKernelGGL((adj_kernel<false, true>), grid, dim3(64), 0, s, bins, tabs, wtab, wtanc, partial, A);
    else
      hipLaunchKernelGGL((adj_kernel<false, false>), grid, dim3(64), 0, s, bins, tabs, wtab, wtanc, partial, A);
  } else if (kep && long_sinc) {
    hipLaunchKernelGGL((forward_grad_kep_kernel<true>), grid, dim3(256), 0, s, bins, tabs, wtab, wtan, partial, A);
  } else if (kep) {
    hipLaunchKernelGGL((forward_grad_kep_kernel<false>), grid, dim3(256), 0, s, bins, tabs, wtab, wtan, partial, A);
  } else if (long_sinc) {
    hipLaunchKernelGGL((forward_grad_kernel<true>), grid, dim3(256), 0, s, bins, tabs, wtab, wtan, partial, A);
  } else {
    hipLaunchKernelGGL((forward_grad_kernel<false>), grid, dim3(256), 0, s, bins, tabs, wtab, wtan, partial, A);
  }
  hipLaunchKernelGGL(grad_finalize_kernel, dim3((A.B + 255) / 256), dim3(256), 0, s, partial, wtab, dd, A, logl,
                     grad);
  return hipGetLastError();
}

hipError_t launch_fisher(const double* bins, const double* tabs, const double* wtab, const double* wtan,
                         double* partial, const JacArgs& A, bool long_sinc, double* F, hipStream_t s) {
  const dim3 grid((unsigned)((A.N + A.tile - 1) / A.tile), (unsigned)A.B);
  const bool kep = A.wkep != nullptr;
  if (kep && (!A.kep || !A.wkept)) return hipErrorInvalidValue;
  if (kep && long_sinc)
    hipLaunchKernelGGL((forward_fisher_kep_kernel<true>), grid, dim3(256), 0, s, bins, tabs, wtab, wtan, partial, A);
  else if (kep)
    hipLaunchKernelGGL((forward_fisher_kep_kernel<false>), grid, dim3(256), 0, s, bins, tabs, wtab, wtan, partial, A);
  else if (long_sinc)
    hipLaunchKernelGGL((forward_fisher_kernel<true>), grid, dim3(256), 0, s, bins, tabs, wtab, wtan, partial, A);
  else
    hipLaunchKernelGGL((forward_fisher_kernel<false>), grid, dim3(256), 0, s, bins, tabs, wtab, wtan, partial, A);
  hipLaunchKernelGGL(fisher_finalize_kernel, dim3(A.B), dim3(128), 0, s, partial, wtab, A, F);
  return hipGetLastError();
}

}  // namespace pes
