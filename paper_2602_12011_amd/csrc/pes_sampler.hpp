// Argument blocks of the sampler kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pes_layout.hpp"

namespace pes {

struct PriorArgs {
  int kind[kNParams];
  double lo[kNParams], hi[kNParams];
};

struct DeArgs {
  int64_t upd0, n_upd;   // walkers being updated: [upd0, upd0 + n_upd)
  int64_t ref0, n_ref;   // reference half: [ref0, ref0 + n_ref)
  int half;              // 0 or 1 (the position within the step)
  double gamma;          // 2.38 / sqrt(2 d)
  uint64_t seed;
  double width[kNParams];
  PriorArgs prior;
};

hipError_t launch_noise(const double* tabs, int64_t N, int n_det, uint64_t seed, double* out, hipStream_t s);
hipError_t launch_philox(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n, uint32_t* out,
                         hipStream_t s);
hipError_t launch_de_propose(const double* theta, double* prop, double* qratio, const uint64_t* step,
                             const DeArgs& a, hipStream_t s);
hipError_t launch_accept(double* theta, double* logl, double* logp, const double* prop, const double* prop_logl,
                         const double* qratio, int64_t* accepts, uint64_t* step, const DeArgs& a, hipStream_t s);
hipError_t launch_end_step(const double* theta, uint64_t* step, double* chain, int64_t n_chain, int64_t B,
                           hipStream_t s);
hipError_t launch_init_state(const double* theta, double* logp, int64_t B, const PriorArgs& p, hipStream_t s);
hipError_t launch_flow_latent(double* z, const uint64_t* step, const DeArgs& a, hipStream_t s);
hipError_t launch_flow_mix(const double* fprop, const double* lq_prop, const double* lq_cur, double* prop,
                           double* qratio, const uint64_t* step, const DeArgs& a, double p_flow, hipStream_t s);

}  // namespace pes
