// Kernel argument blocks and launchers (host side of the kernels TU).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pes_layout.hpp"

namespace pes {

constexpr int kMaxGroup = 64;   // walkers per work item, upper bound

struct DetTable {
  DetParams p[kMaxDet];
};

struct SetupArgs {
  int n_modes, n_det;
  ModeSpec modes[kMaxModes];
  DetTable dt;
  double f0, df;
  int64_t N;
  int tile;
  int full_tiles;   // 1: every valid walker covers the whole grid (plain-grid schedule)
};

struct LoglikeArgs {
  const double* bins;
  const double* tabs;
  const double* wtab;
  const float* wtab32;   // FP32 copy of the walker tables (single-precision kernels only)
  const double* wkep;    // [B][n_det][KW_STRIDE] projected orbit series (exact Kepler orbits only)
  const double* kep;     // [n_det][KV_STRIDE] orbit series of the detectors (exact Kepler orbits only)
  const int* ntiles;
  const int* perm;
  const int* gstart;
  int* counters;
  double* partial;
  int64_t N;
  int B, wg, n_groups, ntmax, n_modes, n_det;
  ModePlan plan;
  int grid_mode;   // 1: block i takes work item i (plain grid); 0: atomic ticket
  DetTable dt;
  const float* wkep32;   // FP32 copies of wkep and kep (single precision on exact Kepler orbits only)
  const float* kep32;
};

struct ResponseArgs {
  const double* bins;
  const double* tabs;
  const double* wtab;
  const float* wtab32;   // FP32 copy of the walker tables (single-precision kernels only)
  const double* wkep;    // [B][n_det][KW_STRIDE] projected orbit series (exact Kepler orbits only)
  const double* kep;     // [n_det][KV_STRIDE] orbit series of the detectors (exact Kepler orbits only)
  double* out;
  int64_t N;
  int n_modes, n_det;
  ModePlan plan;
  DetTable dt;
  const float* wkep32;   // FP32 copies of wkep and kep (single precision on exact Kepler orbits only)
  const float* kep32;
};

// Doubles per walker of the compact tangent table of the reverse sweep.
constexpr int kTanCompactSlots = 584;

struct JacArgs {
  int64_t N;
  int B, n_modes, n_det;
  ModePlan plan;
  int tile;           // bins per block (a multiple of 64)
  double f0, df;
  DetTable dt;
  const double* theta;   // [B][11] (the reverse sweep's sky contraction)
  // exact Kepler orbits (null otherwise): the detectors' series [kMaxDet][KV_STRIDE],
  // the walkers' projected series [B][n_det][KW_STRIDE] and their derivatives
  // in lambda, beta, psi [B][n_det][3][KW_STRIDE]
  const double* kep;
  const double* wkep;
  const double* wkept;
};

hipError_t launch_grad(const double* bins, const double* tabs, const double* wtab, const double* wtan,
                       double* partial, const double* dd, const JacArgs& A, bool long_sinc, bool adjoint,
                       double* logl, double* grad, hipStream_t s);
hipError_t launch_fisher(const double* bins, const double* tabs, const double* wtab, const double* wtan,
                         double* partial, const JacArgs& A, bool long_sinc, double* F, hipStream_t s);

hipError_t launch_bin_tables(double* bins, double* tabs, int64_t N, double f0, double df, int n_det,
                             const DetTable& dt, hipStream_t s);
hipError_t launch_set_data(const double* d, double* tabs, double* dd_part, double* dd, int64_t N,
                           int n_det, hipStream_t s);
hipError_t launch_setup(const double* theta, int64_t B, double* wtab, int* ntiles, const SetupArgs& sa,
                        hipStream_t s);
hipError_t launch_setup_tan(const double* theta, int64_t B, double* wtab, double* wtan, int* ntiles,
                            const SetupArgs& sa, hipStream_t s);
hipError_t launch_plan(const int* ntiles, int B, int wg, int ntmax, bool sorted, int* perm, int* gstart,
                       int* counters, hipStream_t s);
hipError_t launch_loglike(const LoglikeArgs& a, int bpl, bool long_sinc, bool f32, bool kep, int grid,
                          hipStream_t s);
hipError_t launch_kepler_proj(const double* theta, int64_t B, const double* kep, const SetupArgs& sa,
                              double* wkep, hipStream_t s);
hipError_t launch_kepler_proj_tan(const double* theta, int64_t B, const double* kep, const SetupArgs& sa,
                                  double* wkept, hipStream_t s);
hipError_t launch_table32(const double* wtab, int64_t B, float* wtab32, hipStream_t s);
hipError_t launch_copy_f32(const double* src, int64_t n, float* dst, hipStream_t s);
hipError_t launch_finalize(const double* partial, const int* ntiles, const double* wtab, const double* dd,
                           int64_t B, double* logl, hipStream_t s);
hipError_t launch_probe(const ResponseArgs& a, int64_t B, bool long_sinc, bool kep, int stage, hipStream_t s);
hipError_t launch_response(const ResponseArgs& a, int64_t B, bool long_sinc, bool f32, bool kep, hipStream_t s);
int loglike_blocks_per_cu(int bpl, bool long_sinc, bool f32, bool kep);

}  // namespace pes
