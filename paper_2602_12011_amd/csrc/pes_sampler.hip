// Ensemble sampler on the device: counter-based random numbers (Philox4x32-10),
// differential-evolution proposals over the half-ensemble, Metropolis-Hastings
// acceptance with the exact FP64 likelihood of pes_loglike, and capture of a
// whole sampler step in a HIP graph.  The paper leaves sampling to an
// external sampler through the prior/likelihood split of Bayes' theorem
// (Sec. 2.2); this is the batched sampler that drives the likelihood kernels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>

#include "../../include/pes.h"
#include "pes_layout.hpp"
#include "pes_sampler.hpp"

namespace pes {

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): ten rounds of two 32x32 -> 64-bit multiplications with the
// multipliers 0xD2511F53, 0xCD9E8D57 and the Weyl key increments 0x9E3779B9,
// 0xBB67AE85.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Uniform in (0, 1) from two 32-bit words: 52 bits plus one half, so the
// largest value is 1 - 2^-53 (exactly representable) and 0 never occurs.
__device__ __forceinline__ double u01(uint32_t a, uint32_t b) {
  const uint64_t m = ((uint64_t)a << 20) ^ (uint64_t)(b >> 12);
  return ((double)(m & ((1ull << 52) - 1)) + 0.5) * (1.0 / 4503599627370496.0);
}

// Counter (walker, step, purpose) -> one Philox block.
__device__ __forceinline__ uint4 draw(uint64_t seed, uint64_t walker, uint64_t step, uint32_t purpose) {
  return philox4x32_10(make_uint4((uint32_t)walker, (uint32_t)step, (uint32_t)(step >> 32), purpose),
                       (uint32_t)seed, (uint32_t)(seed >> 32));
}

__global__ void philox_kernel(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                              uint32_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint4 r = philox4x32_10(make_uint4(c0 + (uint32_t)i, c1, c2, c3), (uint32_t)key, (uint32_t)(key >> 32));
  out[4 * i] = r.x;
  out[4 * i + 1] = r.y;
  out[4 * i + 2] = r.z;
  out[4 * i + 3] = r.w;
}

// ---------------------------------------------------------------- prior
__device__ double log_prior(const double* th, const PriorArgs& p) {
  double lp = 0.0;
  for (int j = 0; j < kNParams; ++j) {
    const double x = th[j], lo = p.lo[j], hi = p.hi[j];
    switch (p.kind[j]) {
      case PES_PRIOR_UNIFORM:
        if (!(x >= lo && x <= hi)) return -INFINITY;
        break;
      case PES_PRIOR_LOGUNIFORM:
        if (!(x >= lo && x <= hi)) return -INFINITY;
        lp -= log(x);
        break;
      case PES_PRIOR_SIN:
        if (!(x > lo && x < hi)) return -INFINITY;
        lp += log(sin(x));
        break;
      case PES_PRIOR_COS:
        if (!(x > lo && x < hi)) return -INFINITY;
        lp += log(cos(x));
        break;
      default:  // periodic (wrapped by the proposal) and fixed
        if (!isfinite(x)) return -INFINITY;
        break;
    }
  }
  return lp;
}

__device__ double wrap(double x, double lo, double hi) {
  const double w = hi - lo;
  double y = fmod(x - lo, w);
  if (y < 0.0) y += w;
  return lo + y;
}

// ---------------------------------------------------------------- DE proposal
// For walker i of half h (the half being updated), two distinct walkers r1, r2
// of the other half: theta' = theta_i + gamma (theta_r1 - theta_r2) + eps with
// gamma = 2.38 / sqrt(2 d) (d = number of free parameters), gamma = 1 with
// probability 0.1, eps_j ~ N(0, (1e-6 width_j)^2).  Symmetric: log q ratio 0.
// Random numbers: Philox block (walker, 2 step + half, purpose) with purposes
// 0 (r1, r2), 1 (gamma), 2 + j (jitter of parameter j), 16 (acceptance).
__global__ void de_propose_kernel(const double* __restrict__ theta, double* __restrict__ prop,
                                  double* __restrict__ qratio, const uint64_t* __restrict__ step_ctr,
                                  DeArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // index within the half
  if (j >= a.n_upd) return;
  const int64_t i = a.upd0 + j;                                      // walker index
  const uint64_t step = step_ctr[0] * 2 + a.half;
  const uint4 r = draw(a.seed, (uint64_t)i, step, 0u);
  const int64_t n = a.n_ref;
  // u n can round up to n: clamp so r1 < n and r2 < n - 1 before the shift
  const int64_t r1 = min((int64_t)(u01(r.x, r.y) * (double)n), n - 1);
  int64_t r2 = min((int64_t)(u01(r.z, r.w) * (double)(n - 1)), n - 2);
  if (r2 >= r1) ++r2;   // distinct from r1, still < n
  const uint4 r3 = draw(a.seed, (uint64_t)i, step, 1u);
  const double gamma = (u01(r3.x, r3.y) < 0.1) ? 1.0 : a.gamma;
  const double* ti = theta + 11 * i;
  const double* ta = theta + 11 * (a.ref0 + r1);
  const double* tb = theta + 11 * (a.ref0 + r2);
  double* tp = prop + 11 * j;
  for (int k = 0; k < kNParams; ++k) {
    double x = ti[k];
    if (a.prior.kind[k] != PES_PRIOR_FIXED) {
      // jitter: Box-Muller normal from the block of purpose 2 + k
      const uint4 rz = draw(a.seed, (uint64_t)i, step, 2u + (uint32_t)k);
      const double u1 = u01(rz.x, rz.y);
      const double u2 = u01(rz.z, rz.w);
      const double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
      x = fma(gamma, ta[k] - tb[k], x) + 1e-6 * a.width[k] * z;
      if (a.prior.kind[k] == PES_PRIOR_PERIODIC) x = wrap(x, a.prior.lo[k], a.prior.hi[k]);
    }
    tp[k] = x;
  }
  qratio[j] = 0.0;
}

// ---------------------------------------------------------------- accept
// log u < (L' + log pi') - (L + log pi) + log q ratio  ->  take the proposal.
__global__ void accept_kernel(double* __restrict__ theta, double* __restrict__ logl, double* __restrict__ logp,
                              const double* __restrict__ prop, const double* __restrict__ prop_logl,
                              const double* __restrict__ qratio, int64_t* __restrict__ accepts,
                              const uint64_t* __restrict__ step_ctr, DeArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t step = step_ctr[0];
  if (j < a.n_upd) {
    const int64_t i = a.upd0 + j;
    const double* tp = prop + 11 * j;
    const double lp = log_prior(tp, a.prior);
    const double Lp = prop_logl[j];
    const double delta = (Lp + lp) - (logl[i] + logp[i]) + qratio[j];
    const uint4 r = draw(a.seed, (uint64_t)i, step * 2 + a.half, 16u);
    const double lu = log(u01(r.x, r.y));
    if (isfinite(lp) && Lp > -INFINITY && lu < delta) {
      for (int k = 0; k < kNParams; ++k) theta[11 * i + k] = tp[k];
      logl[i] = Lp;
      logp[i] = lp;
      accepts[i] += 1;
    }
  }
}

// Chain append (all walkers) and counter advance, after both halves.
__global__ void end_step_kernel(const double* __restrict__ theta, uint64_t* __restrict__ step_ctr,
                                double* __restrict__ chain, int64_t n_chain, int64_t B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t step = step_ctr[0];
  if (n_chain > 0 && t < B * 11) chain[(int64_t)(step % (uint64_t)n_chain) * B * 11 + t] = theta[t];
  if (t == 0) step_ctr[1] = step + 1;   // committed by the next kernel (other blocks still read [0])
}

__global__ void commit_step_kernel(uint64_t* __restrict__ step_ctr) {
  step_ctr[0] = step_ctr[1];
}

__global__ void init_state_kernel(const double* __restrict__ theta, double* __restrict__ logp, int64_t B,
                                  PriorArgs p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) logp[i] = log_prior(theta + 11 * i, p);
}

// ---------------------------------------------------------------- flow proposal
// Latent draws of the independence proposal: z_k ~ N(0, 1) by Box-Muller from
// the Philox block of purpose 20 + k.
__global__ void flow_latent_kernel(double* __restrict__ z, const uint64_t* __restrict__ step_ctr, DeArgs a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_upd) return;
  const int64_t i = a.upd0 + j;
  const uint64_t step = step_ctr[0] * 2 + a.half;
  for (int k = 0; k < kNParams; ++k) {
    const uint4 r = draw(a.seed, (uint64_t)i, step, 20u + (uint32_t)k);
    const double u1 = u01(r.x, r.y), u2 = u01(r.z, r.w);
    z[11 * j + k] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

// Mixture: with probability p_flow (purpose 19) the walker takes the flow's
// proposal and the Hastings term log q(current) - log q(proposal); otherwise
// it keeps the DE proposal already in prop (log q ratio 0).  A flow proposal
// outside the range of a periodic parameter is rejected (log q ratio -inf).
__global__ void flow_mix_kernel(const double* __restrict__ fprop, const double* __restrict__ lq_prop,
                                const double* __restrict__ lq_cur, double* __restrict__ prop,
                                double* __restrict__ qratio, const uint64_t* __restrict__ step_ctr, DeArgs a,
                                double p_flow) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= a.n_upd) return;
  const int64_t i = a.upd0 + j;
  const uint64_t step = step_ctr[0] * 2 + a.half;
  const uint4 r = draw(a.seed, (uint64_t)i, step, 19u);
  if (!(u01(r.x, r.y) < p_flow)) return;
  bool ok = isfinite(lq_prop[j]) && isfinite(lq_cur[j]);
  for (int k = 0; k < kNParams; ++k) {
    const double x = fprop[11 * j + k];
    prop[11 * j + k] = x;
    if (a.prior.kind[k] == PES_PRIOR_PERIODIC && !(x >= a.prior.lo[k] && x < a.prior.hi[k])) ok = false;
  }
  qratio[j] = ok ? lq_cur[j] - lq_prop[j] : -INFINITY;
}

// ---------------------------------------------------------------- launchers
// Stationary Gaussian noise: Re, Im ~ N(0, 1 / w) with w = 4 df / S_c the
// channel's weight (0 where S_c = 0: no noise there).
__global__ void noise_kernel(const double* __restrict__ tabs, int64_t N, int n_det, uint64_t seed,
                             double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  for (int det = 0; det < n_det; ++det) {
    const double* t = tabs + (int64_t)det * T_NFIELDS * N;
    const double wae = t[T_WAE * N + k], wtt = t[T_WTT * N + k];
    for (int c = 0; c < 3; ++c) {
      const double w = c < 2 ? wae : wtt;
      const uint4 r = philox4x32_10(make_uint4((uint32_t)k, (uint32_t)det, (uint32_t)c, 0xD0u),
                                    (uint32_t)seed, (uint32_t)(seed >> 32));
      const double rad = sqrt(-2.0 * log(u01(r.x, r.y)));
      double sn, cs;
      sincos(6.283185307179586 * u01(r.z, r.w), &sn, &cs);
      const double sig = w > 0.0 ? sqrt(1.0 / w) : 0.0;
      double* o = out + (((int64_t)det * 3 + c) * N + k) * 2;
      o[0] = sig * rad * cs;
      o[1] = sig * rad * sn;
    }
  }
}

hipError_t launch_noise(const double* tabs, int64_t N, int n_det, uint64_t seed, double* out, hipStream_t s) {
  hipLaunchKernelGGL(noise_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, tabs, N, n_det, seed, out);
  return hipGetLastError();
}

hipError_t launch_philox(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n, uint32_t* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(philox_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, key, c0, c1, c2, c3, n,
                     out);
  return hipGetLastError();
}

hipError_t launch_de_propose(const double* theta, double* prop, double* qratio, const uint64_t* step,
                             const DeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(de_propose_kernel, dim3((unsigned)((a.n_upd + 127) / 128)), dim3(128), 0, s, theta, prop,
                     qratio, step, a);
  return hipGetLastError();
}

hipError_t launch_accept(double* theta, double* logl, double* logp, const double* prop, const double* prop_logl,
                         const double* qratio, int64_t* accepts, uint64_t* step, const DeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(accept_kernel, dim3((unsigned)((a.n_upd + 127) / 128)), dim3(128), 0, s, theta, logl, logp,
                     prop, prop_logl, qratio, accepts, step, a);
  return hipGetLastError();
}

hipError_t launch_end_step(const double* theta, uint64_t* step, double* chain, int64_t n_chain, int64_t B,
                           hipStream_t s) {
  const int64_t n = std::max<int64_t>(B * 11, 1);
  hipLaunchKernelGGL(end_step_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, step, chain,
                     n_chain, B);
  hipLaunchKernelGGL(commit_step_kernel, dim3(1), dim3(1), 0, s, step);
  return hipGetLastError();
}

hipError_t launch_flow_latent(double* z, const uint64_t* step, const DeArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(flow_latent_kernel, dim3((unsigned)((a.n_upd + 127) / 128)), dim3(128), 0, s, z, step, a);
  return hipGetLastError();
}

hipError_t launch_flow_mix(const double* fprop, const double* lq_prop, const double* lq_cur, double* prop,
                           double* qratio, const uint64_t* step, const DeArgs& a, double p_flow, hipStream_t s) {
  hipLaunchKernelGGL(flow_mix_kernel, dim3((unsigned)((a.n_upd + 127) / 128)), dim3(128), 0, s, fprop, lq_prop,
                     lq_cur, prop, qratio, step, a, p_flow);
  return hipGetLastError();
}

hipError_t launch_init_state(const double* theta, double* logp, int64_t B, const PriorArgs& p, hipStream_t s) {
  hipLaunchKernelGGL(init_state_kernel, dim3((unsigned)((B + 127) / 128)), dim3(128), 0, s, theta, logp, B, p);
  return hipGetLastError();
}

}  // namespace pes
