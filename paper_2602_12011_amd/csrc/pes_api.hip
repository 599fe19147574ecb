// C-ABI of libpes: context management, argument validation and the launch
// sequences of each entry point (declared in include/pes.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "../../include/pes.h"
#include "pes_launch.hpp"
#include "pes_flow.hpp"
#include "pes_sampler.hpp"

using namespace pes;

// Device scratch of pes_loglike_noalloc: one copy per GPU, held until the
// process ends.  Host code never uses the array's name as an address: the
// address on each device is looked up once (scratch_address) and kept.
constexpr int64_t kScratchBytes = int64_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Address of this device's copy of the scratch array (the device must be
// current); null if the lookup fails.
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch[device] = p;
  }
  return g_scratch[device];
}

constexpr double kC = 299792458.0;
constexpr double kAU = 149597870700.0;
constexpr double kYear = 31557600.0;   // Julian year [s]

}  // namespace

struct pes_ctx {
  pes_config cfg;
  int device = 0;
  int n_cu = 0;
  DetTable dt;
  ModeSpec modes[kMaxModes];
  int64_t N = 0;
  // tables
  double* bins = nullptr;
  double* tabs = nullptr;
  double* dd_part = nullptr;
  double* dd = nullptr;
  bool has_data = false;
  // tuning
  int bpl = 1;              // bins per lane (1 or 2)
  bool long_sinc = false;   // a detector's largest sinc argument exceeds the short fit
  int wg = 16;              // walkers per work item
  int bpc = 0;              // resident blocks per CU requested (0: occupancy limit)
  // occupancy limit per variant (FP64, FP32, Kepler FP64, Kepler FP32) and bins per lane
  int occ[4][3] = {{1, 1, 1}, {1, 1, 1}, {1, 1, 1}, {1, 1, 1}};
  bool f32 = false;         // single-precision log-likelihood and response kernels
  bool kep = false;         // heliocentric detectors on exact Kepler ellipses
  double* kep_tab = nullptr;  // [n_det][KV_STRIDE] orbit series (Kepler detectors)
  float* kep_tab32 = nullptr; // its FP32 copy (single precision)
  int tile = 256;
  int grad_method = PES_GRAD_ADJOINT;
  int schedule = PES_SCHED_QUEUE;
  ModePlan plan;            // evaluation units: one per distinct m
  int ntmax = 0;            // tiles per walker at the current tile size
  int ntmax_alloc = 0;      // tiles at the smallest tile (partial-buffer sizing)
  // workspace
  int64_t cap = 0;
  double* wtab = nullptr;
  float* wtab32 = nullptr;    // FP32 copy of wtab (single-precision kernels)
  double* wkep = nullptr;     // [cap][n_det][KW_STRIDE] projected orbit series (Kepler contexts)
  float* wkep32 = nullptr;    // its FP32 copy (Kepler contexts, single precision)
  double* wkept = nullptr;    // [jcap][n_det][3][KW_STRIDE] their sky-angle derivatives (Kepler contexts)
  int* ntiles = nullptr;
  int* perm = nullptr;
  int* gstart = nullptr;
  int* counters = nullptr;
  double* partial = nullptr;
  uint64_t ws_gen = 0;        // bumped whenever the workspace above is reallocated
  void* scratch = nullptr;    // this device's scratch array (pes_loglike_noalloc)
  // derivative workspace
  int64_t jcap = 0;
  double* wtan = nullptr;      // [jcap][W_STRIDE][11]
  double* jpart = nullptr;     // per-tile partial sums of the derivative kernels
  int64_t jpart_n = 0;
  // measurement
  bool timing = false;
  int n_ev = 0;
  hipEvent_t* ev = nullptr;   // [kMaxEv][2]
  char err[256] = {0};
};

namespace {

constexpr int kMaxEv = 4096;

int fail_hip(pes_ctx* c, hipError_t e, const char* where) {
  if (c) snprintf(c->err, sizeof(c->err), "%s: %s", where, hipGetErrorString(e));
  return PES_EHIP;
}

#define PES_HIP(ctx, call)                                   \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return fail_hip((ctx), e_, #call); \
  } while (0)

// Kernel variant of the log-likelihood: 0 FP64, 1 FP32, 2 FP64 and 3 FP32 on exact Kepler orbits.
int occ_var(const pes_ctx* c) { return (c->kep ? 2 : 0) + (c->f32 ? 1 : 0); }

bool mode_ok(int l, int m) {
  return (l == 2 && (m == 2 || m == 1)) || (l == 3 && (m == 3 || m == 2)) || (l == 4 && m == 4);
}

void free_workspace(pes_ctx* c) {
  (void)hipFree(c->wtab);
  (void)hipFree(c->wtab32);
  (void)hipFree(c->wkep);
  (void)hipFree(c->wkep32);
  (void)hipFree(c->ntiles);
  (void)hipFree(c->perm);
  (void)hipFree(c->gstart);
  (void)hipFree(c->counters);
  (void)hipFree(c->partial);
  c->wtab = nullptr;
  c->wtab32 = nullptr;
  c->wkep = nullptr;
  c->wkep32 = nullptr;
  c->ntiles = c->perm = c->gstart = c->counters = nullptr;
  c->partial = nullptr;
  c->cap = 0;
}

int ensure_workspace(pes_ctx* c, int64_t B) {
  if (B <= c->cap) return PES_OK;
  const int64_t cap = std::max<int64_t>(B, 64);
  free_workspace(c);
  const int64_t ng = (cap + 1) / 1 + 1;  // groups <= walkers
  if (hipMalloc(&c->wtab, sizeof(double) * cap * W_STRIDE) != hipSuccess ||
      hipMalloc(&c->wtab32, sizeof(float) * cap * W_STRIDE) != hipSuccess ||
      (c->kep && hipMalloc(&c->wkep, sizeof(double) * cap * c->cfg.n_det * KW_STRIDE) != hipSuccess) ||
      (c->kep && hipMalloc(&c->wkep32, sizeof(float) * cap * c->cfg.n_det * KW_STRIDE) != hipSuccess) ||
      hipMalloc(&c->ntiles, sizeof(int) * cap) != hipSuccess ||
      hipMalloc(&c->perm, sizeof(int) * cap) != hipSuccess ||
      hipMalloc(&c->gstart, sizeof(int) * (ng + 1)) != hipSuccess ||
      hipMalloc(&c->counters, sizeof(int) * 4) != hipSuccess ||
      hipMalloc(&c->partial, sizeof(double) * 2 * cap * (int64_t)c->ntmax_alloc) != hipSuccess) {
    free_workspace(c);
    snprintf(c->err, sizeof(c->err), "workspace allocation for %lld walkers failed", (long long)cap);
    return PES_ENOMEM;
  }
  c->cap = cap;
  ++c->ws_gen;
  return PES_OK;
}

constexpr int kGradTile = 1024;
constexpr int64_t kMaxDerivBatch = 65535;   // batch limit of pes_grad and pes_fisher
constexpr int kFisherTile = 1024;

void free_jac(pes_ctx* c) {
  (void)hipFree(c->wtan);
  (void)hipFree(c->jpart);
  (void)hipFree(c->wkept);
  c->wtan = c->jpart = c->wkept = nullptr;
  c->jcap = 0;
  c->jpart_n = 0;
}

int ensure_jac(pes_ctx* c, int64_t B) {
  int st = ensure_workspace(c, B);
  if (st != PES_OK) return st;
  const int64_t ng = (c->N + kGradTile - 1) / kGradTile, nf = (c->N + kFisherTile - 1) / kFisherTile;
  const int64_t cap = std::max<int64_t>(B, 16);
  const int64_t need = std::max(ng * cap * (kNParams + 2), nf * cap * kNParams * kNParams);
  if (B <= c->jcap && need <= c->jpart_n) return PES_OK;
  free_jac(c);
  if (hipMalloc(&c->wtan, sizeof(double) * cap * (W_STRIDE * kNParams + kTanCompactSlots)) != hipSuccess ||
      hipMalloc(&c->jpart, sizeof(double) * need) != hipSuccess ||
      (c->kep && hipMalloc(&c->wkept, sizeof(double) * cap * c->cfg.n_det * 3 * KW_STRIDE) != hipSuccess)) {
    free_jac(c);
    snprintf(c->err, sizeof(c->err), "derivative workspace for %lld walkers failed", (long long)cap);
    return PES_ENOMEM;
  }
  c->jcap = cap;
  c->jpart_n = need;
  return PES_OK;
}

void fill_geometry(const pes_detector& d, DetParams& p) {
  memset(&p, 0, sizeof(p));
  p.kind = d.kind;
  p.tdi_gen = d.tdi_gen;
  p.L = d.arm_m / kC;
  p.inv_year = 1.0 / kYear;
  p.inv_ptq = d.kind == PES_TIANQIN ? 1.0 / d.tq_period_s : 0.0;
  p.phase0_cyc = d.phase0 / (2.0 * M_PI);
  p.AUc = kAU / kC;
  p.oms2 = d.oms_asd * d.oms_asd;
  p.acc2 = d.acc_asd * d.acc_asd;
  for (int s = 0; s < 3; ++s) {
    const double b = 2.0 * M_PI * s / 3.0, cb = cos(b), sb = sin(b);
    if (d.kind == PES_TIANQIN) {
      // ring of radius L/sqrt3 in the plane normal to (lon, lat)
      const double R = p.L / sqrt(3.0);
      const double nh[3] = {cos(d.tq_lat) * cos(d.tq_lon), cos(d.tq_lat) * sin(d.tq_lon), sin(d.tq_lat)};
      const double u[3] = {-sin(d.tq_lon), cos(d.tq_lon), 0.0};
      const double w[3] = {nh[1] * u[2] - nh[2] * u[1], nh[2] * u[0] - nh[0] * u[2], nh[0] * u[1] - nh[1] * u[0]};
      for (int c = 0; c < 3; ++c) {
        p.G[s][c][0] = R * (cb * u[c] + sb * w[c]);     // x cos(phi)
        p.G[s][c][1] = R * (-sb * u[c] + cb * w[c]);    // x sin(phi)
      }
    } else {
      // first-order-in-eccentricity heliocentric orbit, rho = e AU / c = L / (2 sqrt3)
      const double rho = p.L / (2.0 * sqrt(3.0));
      p.G[s][0][0] = rho * 0.5 * cb;
      p.G[s][0][1] = rho * 0.5 * sb;
      p.G[s][0][4] = -rho * 1.5 * cb;
      p.G[s][1][0] = -rho * 0.5 * sb;
      p.G[s][1][1] = rho * 0.5 * cb;
      p.G[s][1][4] = -rho * 1.5 * sb;
      p.G[s][2][2] = -rho * sqrt(3.0) * cb;
      p.G[s][2][3] = -rho * sqrt(3.0) * sb;
    }
  }
}

// Fourier series (harmonics 0..kKepH of the revolution phase alpha) of the
// orbit vectors of a heliocentric detector on exact Kepler ellipses:
// semi-major axis 1 AU, eccentricity e = L / (2 sqrt3 AU), inclination
// sin i = sqrt3 e, longitude of perihelion b_n = 2 pi n / 3, ascending node
// b_n + pi/2, mean anomaly alpha - b_n (the ellipses whose first-order
// expansion in e is the triangle of fill_geometry).  Sampled at 64 phases in
// long double (Kepler's equation by Newton's method) and transformed
// exactly; the series converge as e^k, so harmonic 7 and up are below 1e-13 s.
void kepler_table(const pes_detector& d, double* out) {
  constexpr int NS = 64;
  const long double PI = 3.14159265358979323846264338327950288L;
  const long double R = (long double)kAU / (long double)kC;
  const long double e = (long double)d.arm_m / (2.0L * sqrtl(3.0L) * (long double)kAU);
  const long double si = sqrtl(3.0L) * e, ci = sqrtl(1.0L - si * si), sq = sqrtl(1.0L - e * e);
  // samples: 15 vector components (Delta_0, Delta_1, x_0 - c, x_1 - c, c) and 3 inverse lengths
  long double v[NS][18];
  for (int j = 0; j < NS; ++j) {
    const long double al = 2.0L * PI * j / NS;
    long double x[3][3];
    for (int n = 0; n < 3; ++n) {
      const long double b = 2.0L * PI * n / 3.0L;
      const long double M = al - b;
      long double E = M + e * sinl(M);
      for (int it = 0; it < 12; ++it) E -= (E - e * sinl(E) - M) / (1.0L - e * cosl(E));
      const long double xo = R * (cosl(E) - e), yo = R * sq * sinl(E);
      const long double u = yo, w = -xo;                 // argument of perihelion -pi/2
      const long double Om = b + 0.5L * PI;
      x[n][0] = u * cosl(Om) - w * ci * sinl(Om);
      x[n][1] = u * sinl(Om) + w * ci * cosl(Om);
      x[n][2] = w * si;
    }
    long double c[3], d0[3], d1[3], d2[3];
    for (int k = 0; k < 3; ++k) {
      c[k] = (x[0][k] + x[1][k] + x[2][k]) / 3.0L;
      d0[k] = x[2][k] - x[1][k];
      d1[k] = x[0][k] - x[2][k];
      d2[k] = x[1][k] - x[0][k];
    }
    for (int k = 0; k < 3; ++k) {
      v[j][k] = d0[k];
      v[j][3 + k] = d1[k];
      v[j][6 + k] = x[0][k] - c[k];
      v[j][9 + k] = x[1][k] - c[k];
      v[j][12 + k] = c[k];
    }
    const long double* dd[3] = {d0, d1, d2};
    for (int t = 0; t < 3; ++t)
      v[j][15 + t] = 1.0L / sqrtl(dd[t][0] * dd[t][0] + dd[t][1] * dd[t][1] + dd[t][2] * dd[t][2]);
  }
  for (int i = 0; i < KV_STRIDE; ++i) out[i] = 0.0;
  for (int q = 0; q < 18; ++q) {
    double* o = out + q * kKepT;   // 15 vector components, then the 3 inverse lengths (KV_INVL)
    long double a0 = 0.0L;
    for (int j = 0; j < NS; ++j) a0 += v[j][q];
    o[0] = (double)(a0 / NS);
    for (int h = 1; h <= kKepH; ++h) {
      long double ac = 0.0L, as = 0.0L;
      for (int j = 0; j < NS; ++j) {
        const long double al = 2.0L * PI * j / NS;
        ac += v[j][q] * cosl(h * al);
        as += v[j][q] * sinl(h * al);
      }
      o[2 * h - 1] = (double)(2.0L * ac / NS);
      o[2 * h] = (double)(2.0L * as / NS);
    }
  }
}

}  // namespace

extern "C" {

const char* pes_strerror(int s) {
  switch (s) {
    case PES_OK: return "ok";
    case PES_EINVAL: return "invalid argument";
    case PES_ESHAPE: return "size inconsistent with the context";
    case PES_ENOMEM: return "device allocation failed";
    case PES_EHIP: return "HIP runtime error";
    case PES_ESTATE: return "call order violated";
    default: return "unknown status";
  }
}

const char* pes_last_error(pes_ctx* ctx) { return ctx ? ctx->err : "null context"; }

// Evaluation units: each mode is paired with the next unpaired mode of the
// same m (the rotated polarization factors of the table refer to the first
// mode with that m, so only that one leads a pair); pairs first, then the
// modes left alone, in the order of the configuration.
static ModePlan make_mode_plan(const ModeSpec* modes, int n) {
  ModePlan p;
  memset(&p, 0, sizeof(p));
  bool used[kMaxModes] = {false, false, false, false, false};
  for (int j = 0; j < n; ++j) {
    bool first_of_m = true;
    for (int i = 0; i < j; ++i)
      if (modes[i].m == modes[j].m) first_of_m = false;
    if (!first_of_m) continue;
    for (int i = j + 1; i < n; ++i)
      if (modes[i].m == modes[j].m) {
        p.lead[p.n_pairs] = j;
        p.member[p.n_pairs] = i;
        used[j] = used[i] = true;
        ++p.n_pairs;
        break;
      }
  }
  p.n_units = p.n_pairs;
  for (int j = 0; j < n; ++j)
    if (!used[j]) {
      p.lead[p.n_units] = j;
      p.member[p.n_units] = -1;
      ++p.n_units;
    }
  return p;
}

int pes_create(const pes_config* cfg, pes_ctx** out) {
  if (!cfg || !out) return PES_EINVAL;
  *out = nullptr;
  if (cfg->n_det < 1 || cfg->n_det > 3 || cfg->n_bins < 1 || cfg->n_bins > (int64_t(1) << 26) ||
      !(cfg->f0 > 0) || !(cfg->df > 0) || cfg->n_modes < 1 || cfg->n_modes > 5)
    return PES_EINVAL;
  for (int i = 0; i < cfg->n_modes; ++i)
    if (!mode_ok(cfg->modes[i][0], cfg->modes[i][1])) return PES_EINVAL;
  for (int i = 0; i < cfg->n_det; ++i) {
    const pes_detector& d = cfg->det[i];
    if (d.kind < 0 || d.kind > 2 || (d.tdi_gen != 15 && d.tdi_gen != 20) || !(d.arm_m > 0) ||
        !(d.oms_asd >= 0) || !(d.acc_asd >= 0) || (d.kind == PES_TIANQIN && !(d.tq_period_s > 0)) ||
        (d.orbit != PES_ORBIT_FIRST_ORDER && d.orbit != PES_ORBIT_KEPLER) ||
        (d.kind == PES_TIANQIN && d.orbit != PES_ORBIT_FIRST_ORDER))
      return PES_EINVAL;
  }
  // every heliocentric detector of a context takes the same orbit model
  bool any_kep = false, any_first = false;
  for (int i = 0; i < cfg->n_det; ++i) {
    if (cfg->det[i].kind == PES_TIANQIN) continue;
    (cfg->det[i].orbit == PES_ORBIT_KEPLER ? any_kep : any_first) = true;
  }
  if (any_kep && any_first) return PES_EINVAL;
  pes_ctx* c = new (std::nothrow) pes_ctx();
  if (!c) return PES_ENOMEM;
  c->cfg = *cfg;
  c->N = cfg->n_bins;
  c->kep = any_kep;
  if (hipGetDevice(&c->device) != hipSuccess ||
      hipDeviceGetAttribute(&c->n_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
      c->n_cu < 1) {
    delete c;
    return PES_EHIP;
  }
  c->scratch = scratch_address(c->device);
  for (int i = 0; i < cfg->n_det; ++i) fill_geometry(cfg->det[i], c->dt.p[i]);
  // largest link sinc argument pi f L (1 + |k.n|) <= 2 pi f_max L per detector
  const double fmax_grid = cfg->f0 + (double)(cfg->n_bins - 1) * cfg->df;
  for (int i = 0; i < cfg->n_det; ++i) {
    const double bmax = 2.0 * M_PI * fmax_grid * c->dt.p[i].L;
    if (bmax * bmax > 16.0) {   // beyond the long sinc fit (f L > 0.64)
      delete c;
      return PES_EINVAL;
    }
    if (bmax * bmax > 4.9) c->long_sinc = true;
  }
  for (int i = 0; i < cfg->n_modes; ++i) c->modes[i] = ModeSpec{cfg->modes[i][0], cfg->modes[i][1]};
  c->plan = make_mode_plan(c->modes, cfg->n_modes);
  c->tile = 256 * c->bpl;
  c->ntmax = (int)((c->N + c->tile - 1) / c->tile);
  c->ntmax_alloc = (int)((c->N + 255) / 256);
  for (int p = 0; p < 4; ++p)
    for (int bpl = 1; bpl <= 2; ++bpl)
      c->occ[p][bpl] = std::max(1, loglike_blocks_per_cu(bpl, c->long_sinc, (p & 1) != 0, p >= 2));
  const int64_t nb = (c->N + 255) / 256;
  if (hipMalloc(&c->bins, sizeof(double) * B_NFIELDS * c->N) != hipSuccess ||
      hipMalloc(&c->tabs, sizeof(double) * T_NFIELDS * c->N * cfg->n_det) != hipSuccess ||
      hipMalloc(&c->dd_part, sizeof(double) * nb) != hipSuccess ||
      hipMalloc(&c->dd, sizeof(double)) != hipSuccess) {
    pes_destroy(c);
    return PES_ENOMEM;
  }
  if (c->kep) {
    double host[kMaxDet * KV_STRIDE] = {0};
    for (int i = 0; i < cfg->n_det; ++i)
      if (cfg->det[i].kind != PES_TIANQIN) kepler_table(cfg->det[i], host + i * KV_STRIDE);
    float host32[kMaxDet * KV_STRIDE];
    for (int i = 0; i < kMaxDet * KV_STRIDE; ++i) host32[i] = (float)host[i];
    if (hipMalloc(&c->kep_tab, sizeof(double) * kMaxDet * KV_STRIDE) != hipSuccess ||
        hipMemcpy(c->kep_tab, host, sizeof(host), hipMemcpyHostToDevice) != hipSuccess ||
        hipMalloc(&c->kep_tab32, sizeof(float) * kMaxDet * KV_STRIDE) != hipSuccess ||
        hipMemcpy(c->kep_tab32, host32, sizeof(host32), hipMemcpyHostToDevice) != hipSuccess) {
      pes_destroy(c);
      return PES_ENOMEM;
    }
  }
  hipError_t e = launch_bin_tables(c->bins, c->tabs, c->N, cfg->f0, cfg->df, cfg->n_det, c->dt, 0);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    pes_destroy(c);
    return PES_EHIP;
  }
  *out = c;
  return PES_OK;
}

int pes_destroy(pes_ctx* c) {
  if (!c) return PES_EINVAL;
  (void)hipDeviceSynchronize();
  pes_timing(c, 0);
  free_workspace(c);
  free_jac(c);
  (void)hipFree(c->bins);
  (void)hipFree(c->tabs);
  (void)hipFree(c->dd_part);
  (void)hipFree(c->dd);
  (void)hipFree(c->kep_tab);
  (void)hipFree(c->kep_tab32);
  delete c;
  return PES_OK;
}

int pes_timing(pes_ctx* c, int enable) {
  if (!c) return PES_EINVAL;
  if (enable && !c->ev) {
    c->ev = new (std::nothrow) hipEvent_t[2 * kMaxEv];
    if (!c->ev) return PES_ENOMEM;
    for (int i = 0; i < 2 * kMaxEv; ++i) {
      if (hipEventCreate(&c->ev[i]) != hipSuccess) {
        for (int j = 0; j < i; ++j) (void)hipEventDestroy(c->ev[j]);
        delete[] c->ev;
        c->ev = nullptr;
        return PES_EHIP;
      }
    }
  }
  if (!enable && c->ev) {
    (void)hipDeviceSynchronize();
    for (int i = 0; i < 2 * kMaxEv; ++i) (void)hipEventDestroy(c->ev[i]);
    delete[] c->ev;
    c->ev = nullptr;
  }
  c->timing = enable != 0;
  c->n_ev = 0;
  return PES_OK;
}

int pes_timing_read(pes_ctx* c, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return PES_EINVAL;
  double sum = 0.0;
  for (int i = 0; i < c->n_ev; ++i) {
    float ms = 0.f;
    PES_HIP(c, hipEventSynchronize(c->ev[2 * i + 1]));
    PES_HIP(c, hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]));
    sum += ms;
  }
  *total_ms = sum;
  *launches = c->n_ev;
  c->n_ev = 0;
  return PES_OK;
}

int pes_set_tuning(pes_ctx* c, int bins_per_lane, int walkers_per_group, int blocks_per_cu) {
  if (!c || (bins_per_lane != 1 && bins_per_lane != 2) || walkers_per_group < 1 ||
      walkers_per_group > kMaxGroup || blocks_per_cu < 0 || blocks_per_cu > 16)
    return PES_EINVAL;
  c->bpl = bins_per_lane;
  c->wg = walkers_per_group;
  c->bpc = blocks_per_cu;
  c->tile = 256 * c->bpl;
  c->ntmax = (int)((c->N + c->tile - 1) / c->tile);
  return PES_OK;
}

int pes_get_tuning(pes_ctx* c, int* bins_per_lane, int* walkers_per_group, int* blocks_per_cu) {
  if (!c || !bins_per_lane || !walkers_per_group || !blocks_per_cu) return PES_EINVAL;
  *bins_per_lane = c->bpl;
  *walkers_per_group = c->wg;
  *blocks_per_cu = c->bpc > 0 ? std::min(c->bpc, c->occ[occ_var(c)][c->bpl]) : c->occ[occ_var(c)][c->bpl];
  return PES_OK;
}

// Time n calls of pes_loglike on the stream; returns the least single-call
// time [ms] (n_each = 1) or the mean over the n calls (n_each = 0).
static int time_loglike(pes_ctx* c, const double* theta, int64_t B, double* logl, void* stream, hipEvent_t e0,
                        hipEvent_t e1, int n, bool n_each, double* ms_out) {
  hipStream_t s = (hipStream_t)stream;
  double best = 1e300, total = 0.0;
  for (int r = 0; r < (n_each ? n : 1); ++r) {
    if (hipEventRecord(e0, s) != hipSuccess) return PES_EHIP;
    for (int k = 0; k < (n_each ? 1 : n); ++k) {
      const int st = pes_loglike(c, theta, B, logl, stream);
      if (st != PES_OK) return st;
    }
    float ms = 0.f;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return PES_EHIP;
    best = std::min(best, (double)ms);
    total += ms;
  }
  *ms_out = n_each ? best : total / n;
  return PES_OK;
}

int pes_autotune(pes_ctx* c, const double* theta, int64_t B, double* logl, double* best_ms, void* stream) {
  if (!c || !theta || !logl || !best_ms || B < 1) return PES_EINVAL;
  if (!c->has_data) return PES_ESTATE;
  hipEvent_t e0, e1;
  PES_HIP(c, hipEventCreate(&e0));
  PES_HIP(c, hipEventCreate(&e1));
  // stage 1: every candidate, one warm-up and the mean of two calls;
  // stage 2: the three fastest again, the least of three single calls
  struct Cand {
    int bpl, wg, bpc;
    double ms;
  };
  Cand cand[16];
  int nc = 0;
  const int bpls[2] = {1, 2};
  const int wgs[4] = {8, 16, 32, 64};
  const int b0 = c->bpl, w0 = c->wg, c0 = c->bpc;
  int st = PES_OK;
  for (int ib = 0; ib < 2 && st == PES_OK; ++ib)
    for (int iw = 0; iw < 4 && st == PES_OK; ++iw)
      for (int half = 0; half < 2 && st == PES_OK; ++half) {
        const int occ = c->occ[occ_var(c)][bpls[ib]];
        const int bpc = half ? std::max(1, occ / 2) : 0;
        if (half && bpc == occ) continue;
        pes_set_tuning(c, bpls[ib], wgs[iw], bpc);
        st = pes_loglike(c, theta, B, logl, stream);   // warm-up
        double ms = 0.0;
        if (st == PES_OK) st = time_loglike(c, theta, B, logl, stream, e0, e1, 2, false, &ms);
        if (st == PES_OK) cand[nc++] = Cand{bpls[ib], wgs[iw], bpc, ms};
      }
  std::sort(cand, cand + nc, [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
  for (int k = 0; k < std::min(nc, 3) && st == PES_OK; ++k) {
    pes_set_tuning(c, cand[k].bpl, cand[k].wg, cand[k].bpc);
    st = time_loglike(c, theta, B, logl, stream, e0, e1, 3, true, &cand[k].ms);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != PES_OK || nc == 0) {
    pes_set_tuning(c, b0, w0, c0);
    return st != PES_OK ? st : PES_EHIP;
  }
  std::sort(cand, cand + std::min(nc, 3), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
  // among the finalists within 1% of the fastest, the one with the most
  // walkers per item: each item reads its tile's bin tables once, so that
  // choice moves the fewest bytes for the same time
  int pick = 0;
  for (int k = 1; k < std::min(nc, 3); ++k)
    if (cand[k].ms <= 1.01 * cand[0].ms && cand[k].wg > cand[pick].wg) pick = k;
  pes_set_tuning(c, cand[pick].bpl, cand[pick].wg, cand[pick].bpc);
  *best_ms = cand[pick].ms;
  return PES_OK;
}

int pes_reserve(pes_ctx* c, int64_t max_walkers) {
  if (!c || max_walkers < 0) return PES_EINVAL;
  const int st = ensure_workspace(c, max_walkers);
  if (st != PES_OK || max_walkers == 0) return st;
  return ensure_jac(c, std::min<int64_t>(max_walkers, kMaxDerivBatch));
}

int pes_set_data(pes_ctx* c, const double* d, void* stream) {
  if (!c || !d) return PES_EINVAL;
  PES_HIP(c, launch_set_data(d, c->tabs, c->dd_part, c->dd, c->N, c->cfg.n_det, (hipStream_t)stream));
  c->has_data = true;
  return PES_OK;
}

static SetupArgs setup_args(const pes_ctx* c) {
  SetupArgs sa;
  memset(&sa, 0, sizeof(sa));
  sa.n_modes = c->cfg.n_modes;
  sa.n_det = c->cfg.n_det;
  for (int i = 0; i < sa.n_modes; ++i) sa.modes[i] = c->modes[i];
  sa.dt = c->dt;
  sa.f0 = c->cfg.f0;
  sa.df = c->cfg.df;
  sa.N = c->N;
  sa.tile = c->tile;
  return sa;
}

int pes_noise(pes_ctx* c, uint64_t seed, double* out, void* stream) {
  if (!c || !out) return PES_EINVAL;
  PES_HIP(c, launch_noise(c->tabs, c->N, c->cfg.n_det, seed, out, (hipStream_t)stream));
  return PES_OK;
}

int pes_probe(pes_ctx* c, const double* theta, int64_t B, int stage, double* out, void* stream) {
  if (!c || (B > 0 && (!theta || !out)) || B < 0 || B > 65535 || stage < PES_PROBE_MODE || stage > PES_PROBE_LINKS)
    return PES_EINVAL;
  if (B == 0) return PES_OK;
  int st = ensure_workspace(c, B);
  if (st != PES_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  PES_HIP(c, launch_setup(theta, B, c->wtab, c->ntiles, setup_args(c), s));
  if (c->kep) PES_HIP(c, launch_kepler_proj(theta, B, c->kep_tab, setup_args(c), c->wkep, s));
  ResponseArgs ra;   // the stage probes evaluate in FP64 whatever the precision setting
  ra.bins = c->bins;
  ra.tabs = c->tabs;
  ra.wtab = c->wtab;
  ra.wtab32 = nullptr;
  ra.wkep = c->kep ? c->wkep : nullptr;
  ra.kep = c->kep ? c->kep_tab : nullptr;
  ra.wkep32 = nullptr;
  ra.kep32 = nullptr;
  ra.out = out;
  ra.N = c->N;
  ra.n_modes = c->cfg.n_modes;
  ra.n_det = c->cfg.n_det;
  ra.plan = c->plan;
  ra.dt = c->dt;
  PES_HIP(c, launch_probe(ra, B, c->long_sinc, c->kep, stage, s));
  return PES_OK;
}

int pes_response(pes_ctx* c, const double* theta, int64_t B, double* out, void* stream) {
  if (!c || (B > 0 && (!theta || !out)) || B < 0 || B > 65535) return PES_EINVAL;
  if (B == 0) return PES_OK;
  int st = ensure_workspace(c, B);
  if (st != PES_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  PES_HIP(c, launch_setup(theta, B, c->wtab, c->ntiles, setup_args(c), s));
  if (c->f32) PES_HIP(c, launch_table32(c->wtab, B, c->wtab32, s));
  if (c->kep) PES_HIP(c, launch_kepler_proj(theta, B, c->kep_tab, setup_args(c), c->wkep, s));
  if (c->kep && c->f32) PES_HIP(c, launch_copy_f32(c->wkep, B * c->cfg.n_det * KW_STRIDE, c->wkep32, s));
  ResponseArgs ra;
  ra.bins = c->bins;
  ra.tabs = c->tabs;
  ra.wtab = c->wtab;
  ra.wtab32 = c->f32 ? c->wtab32 : nullptr;
  ra.wkep = c->kep ? c->wkep : nullptr;
  ra.kep = c->kep_tab;
  ra.wkep32 = c->kep && c->f32 ? c->wkep32 : nullptr;
  ra.kep32 = c->kep_tab32;
  ra.out = out;
  ra.N = c->N;
  ra.n_modes = c->cfg.n_modes;
  ra.plan = c->plan;
  ra.n_det = c->cfg.n_det;
  ra.dt = c->dt;
  PES_HIP(c, launch_response(ra, B, c->long_sinc, c->f32, c->kep, s));
  return PES_OK;
}

}  // extern "C"

namespace {

// Device buffers one log-likelihood launch sequence works in.
struct LoglikeWork {
  double* wtab;
  float* wtab32;
  double* wkep;
  float* wkep32;
  int* ntiles;
  int* perm;
  int* gstart;
  int* counters;
  double* partial;
};

// Items of the (walker group, tile) plan are int32 in the plan, the queue and
// the ticket; a persistent grid of at most 16 blocks per CU takes one ticket
// per block beyond the last item, so the bound keeps that headroom too.
constexpr int64_t kMaxItems = int64_t(INT32_MAX) - 65536;

int check_items(pes_ctx* c, int64_t B) {
  const int64_t n_groups = (B + c->wg - 1) / c->wg;
  if (n_groups * (int64_t)c->ntmax > kMaxItems) {
    snprintf(c->err, sizeof(c->err), "%lld walker groups x %d tiles exceed the int32 work-item plan",
             (long long)n_groups, c->ntmax);
    return PES_ESHAPE;
  }
  return PES_OK;
}

// setup -> plan -> persistent log-likelihood kernel -> per-walker reduction
int run_loglike(pes_ctx* c, const double* theta, int64_t B, double* logl, const LoglikeWork& ws,
                hipStream_t s) {
  const bool grid_mode = c->schedule == PES_SCHED_GRID;
  const int64_t n_groups = (B + c->wg - 1) / c->wg;
  SetupArgs sa = setup_args(c);
  sa.full_tiles = grid_mode ? 1 : 0;
  PES_HIP(c, launch_setup(theta, B, ws.wtab, ws.ntiles, sa, s));
  if (c->f32) PES_HIP(c, launch_table32(ws.wtab, B, ws.wtab32, s));
  if (c->kep) PES_HIP(c, launch_kepler_proj(theta, B, c->kep_tab, sa, ws.wkep, s));
  if (c->kep && c->f32) PES_HIP(c, launch_copy_f32(ws.wkep, B * c->cfg.n_det * KW_STRIDE, ws.wkep32, s));
  PES_HIP(c, launch_plan(ws.ntiles, (int)B, c->wg, c->ntmax, !grid_mode, ws.perm, ws.gstart, ws.counters, s));
  LoglikeArgs a;
  a.bins = c->bins;
  a.tabs = c->tabs;
  a.wtab = ws.wtab;
  a.wtab32 = ws.wtab32;
  a.wkep = ws.wkep;
  a.kep = c->kep_tab;
  a.wkep32 = c->kep && c->f32 ? ws.wkep32 : nullptr;
  a.kep32 = c->kep_tab32;
  a.ntiles = ws.ntiles;
  a.perm = ws.perm;
  a.gstart = ws.gstart;
  a.counters = ws.counters;
  a.partial = ws.partial;
  a.N = c->N;
  a.B = (int)B;
  a.wg = c->wg;
  a.n_groups = (int)n_groups;
  a.ntmax = c->ntmax;
  a.n_modes = c->cfg.n_modes;
  a.plan = c->plan;
  a.n_det = c->cfg.n_det;
  a.dt = c->dt;
  const int bpc = c->bpc > 0 ? std::min(c->bpc, c->occ[occ_var(c)][c->bpl]) : c->occ[occ_var(c)][c->bpl];
  // persistent grid: the resident blocks, but never more than the items can be
  const int grid = grid_mode ? (int)(n_groups * c->ntmax)
                             : (int)std::min<int64_t>((int64_t)c->n_cu * bpc, n_groups * c->ntmax);
  a.grid_mode = grid_mode ? 1 : 0;
  const bool rec = c->timing && c->n_ev < kMaxEv;
  if (rec) PES_HIP(c, hipEventRecord(c->ev[2 * c->n_ev], s));
  PES_HIP(c, launch_loglike(a, c->bpl, c->long_sinc, c->f32, c->kep, grid, s));
  if (rec) {
    PES_HIP(c, hipEventRecord(c->ev[2 * c->n_ev + 1], s));
    ++c->n_ev;
  }
  PES_HIP(c, launch_finalize(ws.partial, ws.ntiles, ws.wtab, c->dd, B, logl, s));
  return PES_OK;
}

}  // namespace

extern "C" {

int pes_loglike(pes_ctx* c, const double* theta, int64_t B, double* logl, void* stream) {
  if (!c || B < 0 || (B > 0 && (!theta || !logl)) || B > (int64_t(1) << 24)) return PES_EINVAL;
  if (!c->has_data) return PES_ESTATE;
  if (B == 0) return PES_OK;
  int st = check_items(c, B);
  if (st != PES_OK) return st;
  st = ensure_workspace(c, B);
  if (st != PES_OK) return st;
  const LoglikeWork ws{c->wtab,  c->wtab32, c->wkep,     c->wkep32, c->ntiles,
                       c->perm,  c->gstart, c->counters, c->partial};
  return run_loglike(c, theta, B, logl, ws, (hipStream_t)stream);
}

// The log-likelihood workspace of B walkers carved out of one buffer (each
// part 256-byte aligned); returns the bytes it takes.  base may be null to
// size it only.
static int64_t carve_loglike_work(char* base, int64_t B, int ntmax, int n_kep, bool f32, LoglikeWork* ws) {
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) / 256 * 256;
    return p;
  };
  char* wtab = take(sizeof(double) * B * W_STRIDE);
  char* wtab32 = take(sizeof(float) * B * W_STRIDE);
  char* wkep = n_kep > 0 ? take(sizeof(double) * B * n_kep * KW_STRIDE) : nullptr;
  char* wkep32 = n_kep > 0 && f32 ? take(sizeof(float) * B * n_kep * KW_STRIDE) : nullptr;
  char* ntiles = take(sizeof(int) * B);
  char* perm = take(sizeof(int) * B);
  char* gstart = take(sizeof(int) * (B + 3));
  char* counters = take(sizeof(int) * 4);
  char* partial = take(sizeof(double) * 2 * B * (int64_t)ntmax);
  if (ws)
    *ws = LoglikeWork{(double*)wtab, (float*)wtab32, (double*)wkep,   (float*)wkep32,  (int*)ntiles,
                      (int*)perm,    (int*)gstart,   (int*)counters,  (double*)partial};
  return off;
}

int pes_loglike_noalloc(pes_ctx* c, const double* theta, int64_t B, double* logl, void* stream) {
  if (!c || B < 0 || (B > 0 && (!theta || !logl)) || B > (int64_t(1) << 24)) return PES_EINVAL;
  if (!c->has_data) return PES_ESTATE;
  if (B == 0) return PES_OK;
  int st = check_items(c, B);
  if (st != PES_OK) return st;
  if (!c->scratch) {
    snprintf(c->err, sizeof(c->err), "the device scratch array has no address on device %d", c->device);
    return PES_EHIP;
  }
  const int n_kep = c->kep ? c->cfg.n_det : 0;
  const int64_t need = carve_loglike_work(nullptr, B, c->ntmax, n_kep, c->f32, nullptr);
  if (need > kScratchBytes) {
    snprintf(c->err, sizeof(c->err), "%lld walkers x %d tiles need %lld bytes of scratch; it holds %lld",
             (long long)B, c->ntmax, (long long)need, (long long)kScratchBytes);
    return PES_ESHAPE;
  }
  LoglikeWork ws;
  carve_loglike_work((char*)c->scratch, B, c->ntmax, n_kep, c->f32, &ws);
  return run_loglike(c, theta, B, logl, ws, (hipStream_t)stream);
}

static JacArgs jac_args(const pes_ctx* c, int64_t B, int tile) {
  JacArgs A;
  A.N = c->N;
  A.B = (int)B;
  A.n_modes = c->cfg.n_modes;
  A.plan = c->plan;
  A.n_det = c->cfg.n_det;
  A.tile = tile;
  A.f0 = c->cfg.f0;
  A.df = c->cfg.df;
  A.dt = c->dt;
  A.theta = nullptr;
  A.kep = A.wkep = A.wkept = nullptr;
  return A;
}

// Kepler contexts: the walkers' projected orbit series and their sky-angle
// derivatives for the tangent kernels.
static int kepler_jac_setup(pes_ctx* c, const double* theta, int64_t B, bool tangents, JacArgs& A,
                            hipStream_t s) {
  if (!c->kep) return PES_OK;
  PES_HIP(c, launch_kepler_proj(theta, B, c->kep_tab, setup_args(c), c->wkep, s));
  if (tangents) PES_HIP(c, launch_kepler_proj_tan(theta, B, c->kep_tab, setup_args(c), c->wkept, s));
  A.kep = c->kep_tab;
  A.wkep = c->wkep;
  A.wkept = tangents ? c->wkept : nullptr;
  return PES_OK;
}

// The reverse sweep contracts the sky derivatives through the identity
// Delta_0 = L (n_0 + 2 n_1) / 3, Delta_1 = -L (2 n_0 + n_1) / 3 of a
// constellation whose spacecraft offsets sum to zero (both orbit models of
// fill_geometry are such triangles); this checks it for a detector.
static bool centred_triangle(const DetParams& p) {
  for (int cc = 0; cc < 3; ++cc)
    for (int i = 0; i < 5; ++i)
      if (std::fabs(p.G[0][cc][i] + p.G[1][cc][i] + p.G[2][cc][i]) > 1e-12 * p.L) return false;
  return true;
}

int pes_grad(pes_ctx* c, const double* theta, int64_t B, double* logl, double* grad, void* stream) {
  if (!c || B < 0 || B > kMaxDerivBatch || (B > 0 && (!theta || !grad))) return PES_EINVAL;
  if (!c->has_data) return PES_ESTATE;
  if (B == 0) return PES_OK;
  const bool adjoint = c->grad_method == PES_GRAD_ADJOINT;
  if (adjoint && !c->kep)   // the first-order sky contraction needs the centred triangle
    for (int d = 0; d < c->cfg.n_det; ++d)
      if (!centred_triangle(c->dt.p[d])) {
        snprintf(c->err, sizeof(c->err), "detector %d: spacecraft offsets do not sum to zero", d);
        return PES_EINVAL;
      }
  int st = ensure_jac(c, B);
  if (st != PES_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  PES_HIP(c, launch_setup_tan(theta, B, c->wtab, c->wtan, c->ntiles, setup_args(c), s));
  JacArgs A = jac_args(c, B, kGradTile);
  A.theta = theta;
  st = kepler_jac_setup(c, theta, B, !adjoint, A, s);
  if (st != PES_OK) return st;
  PES_HIP(c, launch_grad(c->bins, c->tabs, c->wtab, c->wtan, c->jpart, c->dd, A, c->long_sinc, adjoint, logl,
                         grad, s));
  return PES_OK;
}

int pes_set_precision(pes_ctx* c, int bits) {
  if (!c || (bits != 32 && bits != 64)) return PES_EINVAL;
  c->f32 = bits == 32;
  return PES_OK;
}

int pes_set_schedule(pes_ctx* c, int schedule) {
  if (!c || (schedule != PES_SCHED_QUEUE && schedule != PES_SCHED_GRID)) return PES_EINVAL;
  c->schedule = schedule;
  return PES_OK;
}

int pes_set_grad_method(pes_ctx* c, int method) {
  if (!c || (method != PES_GRAD_ADJOINT && method != PES_GRAD_FORWARD)) return PES_EINVAL;
  c->grad_method = method;
  return PES_OK;
}

int pes_fisher(pes_ctx* c, const double* theta, int64_t B, double* F, void* stream) {
  if (!c || B < 0 || B > kMaxDerivBatch || (B > 0 && (!theta || !F))) return PES_EINVAL;
  if (B == 0) return PES_OK;
  int st = ensure_jac(c, B);
  if (st != PES_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  PES_HIP(c, launch_setup_tan(theta, B, c->wtab, c->wtan, c->ntiles, setup_args(c), s));
  JacArgs A = jac_args(c, B, kFisherTile);
  st = kepler_jac_setup(c, theta, B, true, A, s);
  if (st != PES_OK) return st;
  PES_HIP(c, launch_fisher(c->bins, c->tabs, c->wtab, c->wtan, c->jpart, A, c->long_sinc, F, s));
  return PES_OK;
}

}  // extern "C"

struct pes_sampler {
  pes_ctx* ctx = nullptr;
  int64_t B = 0, H0 = 0, H1 = 0;   // walkers, half sizes
  uint64_t seed = 0;
  int64_t chain_len = 0;
  PriorArgs prior;
  double width[kNParams];
  double gamma = 0.0;
  double *theta = nullptr, *logl = nullptr, *logp = nullptr;
  double *prop = nullptr, *prop_logl = nullptr, *qratio = nullptr, *chain = nullptr;
  int64_t* accepts = nullptr;
  uint64_t* step = nullptr;   // [2]: current step, next step
  // learned proposal (mixture with DE)
  pes_flow* flow = nullptr;
  double p_flow = 0.0;
  double *zbuf = nullptr, *fprop = nullptr, *lq_prop = nullptr, *lq_cur = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // what the captured graph's kernels point into: the context's workspace and
  // the flow's, at the generations current at capture
  uint64_t cap_ws_gen = 0, cap_flow_gen = 0;
  pes_flow* cap_flow = nullptr;
};

namespace {

DeArgs de_args(const pes_sampler* s, int half) {
  DeArgs a;
  memset(&a, 0, sizeof(a));
  a.upd0 = half ? s->H0 : 0;
  a.n_upd = half ? s->H1 : s->H0;
  a.ref0 = half ? 0 : s->H0;
  a.n_ref = half ? s->H0 : s->H1;
  a.half = half;
  a.gamma = s->gamma;
  a.seed = s->seed;
  for (int k = 0; k < kNParams; ++k) a.width[k] = s->width[k];
  a.prior = s->prior;
  return a;
}

// Proposals for one half into s->prop / s->qratio: DE, then (with a flow)
// the per-walker mixture with the flow's independence proposal.
int sampler_propose(pes_sampler* s, const DeArgs& a, bool use_flow, double* prop, double* qratio,
                    hipStream_t st) {
  PES_HIP(s->ctx, launch_de_propose(s->theta, prop, qratio, s->step, a, st));
  if (!use_flow) return PES_OK;
  PES_HIP(s->ctx, launch_flow_latent(s->zbuf, s->step, a, st));
  int rc = flow_inverse(s->flow, s->zbuf, a.n_upd, s->fprop, nullptr, st);
  if (rc == PES_OK) rc = flow_forward(s->flow, s->fprop, a.n_upd, nullptr, s->lq_prop, st);
  if (rc == PES_OK) rc = flow_forward(s->flow, s->theta + 11 * a.upd0, a.n_upd, nullptr, s->lq_cur, st);
  if (rc != PES_OK) {
    snprintf(s->ctx->err, sizeof(s->ctx->err), "flow proposal: %s", pes_flow_last_error(s->flow));
    return rc;
  }
  PES_HIP(s->ctx, launch_flow_mix(s->fprop, s->lq_prop, s->lq_cur, prop, qratio, s->step, a, s->p_flow, st));
  return PES_OK;
}

int sampler_one_step(pes_sampler* s, hipStream_t st) {
  for (int half = 0; half < 2; ++half) {
    const DeArgs a = de_args(s, half);
    int rc = sampler_propose(s, a, s->flow != nullptr, s->prop, s->qratio, st);
    if (rc != PES_OK) return rc;
    rc = pes_loglike(s->ctx, s->prop, a.n_upd, s->prop_logl, st);
    if (rc != PES_OK) return rc;
    PES_HIP(s->ctx, launch_accept(s->theta, s->logl, s->logp, s->prop, s->prop_logl, s->qratio, s->accepts,
                                  s->step, a, st));
  }
  PES_HIP(s->ctx, launch_end_step(s->theta, s->step, s->chain, s->chain_len, s->B, st));
  return PES_OK;
}

void sampler_free(pes_sampler* s) {
  if (s->exec) (void)hipGraphExecDestroy(s->exec);
  if (s->graph) (void)hipGraphDestroy(s->graph);
  (void)hipFree(s->theta);
  (void)hipFree(s->logl);
  (void)hipFree(s->logp);
  (void)hipFree(s->prop);
  (void)hipFree(s->prop_logl);
  (void)hipFree(s->qratio);
  (void)hipFree(s->chain);
  (void)hipFree(s->accepts);
  (void)hipFree(s->step);
  (void)hipFree(s->zbuf);
  (void)hipFree(s->fprop);
  (void)hipFree(s->lq_prop);
  (void)hipFree(s->lq_cur);
}

}  // namespace

extern "C" {

int pes_philox(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n, uint32_t* out,
               void* stream) {
  if (n < 0 || (n > 0 && !out)) return PES_EINVAL;
  if (n == 0) return PES_OK;
  return launch_philox(key, c0, c1, c2, c3, n, out, (hipStream_t)stream) == hipSuccess ? PES_OK : PES_EHIP;
}

int pes_sampler_create(pes_ctx* ctx, const pes_prior* prior, int64_t n_walkers, uint64_t seed,
                       int64_t chain_len, pes_sampler** out) {
  if (!ctx || !prior || !out || n_walkers < 4 || n_walkers > (int64_t(1) << 24) || chain_len < 0) return PES_EINVAL;
  *out = nullptr;
  int n_free = 0;
  for (int k = 0; k < kNParams; ++k) {
    const int kind = prior->kind[k];
    if (kind < PES_PRIOR_UNIFORM || kind > PES_PRIOR_FIXED) return PES_EINVAL;
    if (kind != PES_PRIOR_FIXED && !(prior->hi[k] > prior->lo[k])) return PES_EINVAL;
    if (kind == PES_PRIOR_LOGUNIFORM && !(prior->lo[k] > 0)) return PES_EINVAL;
    if (kind != PES_PRIOR_FIXED) ++n_free;
  }
  if (n_free == 0) return PES_EINVAL;
  if (!ctx->has_data) return PES_ESTATE;
  pes_sampler* s = new (std::nothrow) pes_sampler();
  if (!s) return PES_ENOMEM;
  s->ctx = ctx;
  s->B = n_walkers;
  s->H0 = n_walkers / 2;
  s->H1 = n_walkers - s->H0;
  s->seed = seed;
  s->chain_len = chain_len;
  for (int k = 0; k < kNParams; ++k) {
    s->prior.kind[k] = prior->kind[k];
    s->prior.lo[k] = prior->lo[k];
    s->prior.hi[k] = prior->hi[k];
    s->width[k] = prior->kind[k] == PES_PRIOR_FIXED ? 0.0 : prior->hi[k] - prior->lo[k];
  }
  s->gamma = 2.38 / sqrt(2.0 * n_free);
  const int64_t B = n_walkers, H = s->H1;
  if (hipMalloc(&s->theta, sizeof(double) * B * 11) != hipSuccess ||
      hipMalloc(&s->logl, sizeof(double) * B) != hipSuccess ||
      hipMalloc(&s->logp, sizeof(double) * B) != hipSuccess ||
      hipMalloc(&s->prop, sizeof(double) * H * 11) != hipSuccess ||
      hipMalloc(&s->prop_logl, sizeof(double) * H) != hipSuccess ||
      hipMalloc(&s->qratio, sizeof(double) * H) != hipSuccess ||
      hipMalloc(&s->accepts, sizeof(int64_t) * B) != hipSuccess ||
      hipMalloc(&s->step, sizeof(uint64_t) * 2) != hipSuccess ||
      (chain_len > 0 && hipMalloc(&s->chain, sizeof(double) * chain_len * B * 11) != hipSuccess)) {
    sampler_free(s);
    delete s;
    return PES_ENOMEM;
  }
  const int rc = ensure_workspace(ctx, std::max(B, H));
  if (rc != PES_OK) {
    sampler_free(s);
    delete s;
    return rc;
  }
  *out = s;
  return PES_OK;
}

int pes_sampler_destroy(pes_sampler* s) {
  if (!s) return PES_EINVAL;
  (void)hipDeviceSynchronize();
  sampler_free(s);
  delete s;
  return PES_OK;
}

int pes_sampler_set_state(pes_sampler* s, const double* theta, void* stream) {
  if (!s || !theta) return PES_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  PES_HIP(s->ctx, hipMemcpyAsync(s->theta, theta, sizeof(double) * s->B * 11, hipMemcpyDeviceToDevice, st));
  const int rc = pes_loglike(s->ctx, s->theta, s->B, s->logl, st);
  if (rc != PES_OK) return rc;
  PES_HIP(s->ctx, launch_init_state(s->theta, s->logp, s->B, s->prior, st));
  PES_HIP(s->ctx, hipStreamSynchronize(st));
  const uint64_t zero2[2] = {0, 0};
  PES_HIP(s->ctx, hipMemcpy(s->step, zero2, sizeof(zero2), hipMemcpyHostToDevice));
  int64_t* z = new (std::nothrow) int64_t[s->B]();
  if (!z) return PES_ENOMEM;
  const hipError_t e = hipMemcpy(s->accepts, z, sizeof(int64_t) * s->B, hipMemcpyHostToDevice);
  delete[] z;
  PES_HIP(s->ctx, e);
  return PES_OK;
}

int pes_sampler_set_step(pes_sampler* s, uint64_t steps) {
  if (!s) return PES_EINVAL;
  PES_HIP(s->ctx, hipDeviceSynchronize());
  const uint64_t v[2] = {steps, steps};
  PES_HIP(s->ctx, hipMemcpy(s->step, v, sizeof(v), hipMemcpyHostToDevice));
  return PES_OK;
}

int pes_sampler_step(pes_sampler* s, int64_t n_steps, void* stream) {
  if (!s || n_steps < 0) return PES_EINVAL;
  for (int64_t n = 0; n < n_steps; ++n) {
    const int rc = sampler_one_step(s, (hipStream_t)stream);
    if (rc != PES_OK) return rc;
  }
  return PES_OK;
}

int pes_sampler_capture(pes_sampler* s, void* stream) {
  if (!s) return PES_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (!st) return PES_EINVAL;   // capture needs a non-default stream
  if (s->exec) {
    (void)hipGraphExecDestroy(s->exec);
    s->exec = nullptr;
  }
  if (s->graph) {
    (void)hipGraphDestroy(s->graph);
    s->graph = nullptr;
  }
  const bool timing = s->ctx->timing;
  s->ctx->timing = false;
  PES_HIP(s->ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  const int rc = sampler_one_step(s, st);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  s->ctx->timing = timing;
  if (rc != PES_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  PES_HIP(s->ctx, e);
  s->graph = g;
  PES_HIP(s->ctx, hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0));
  s->cap_ws_gen = s->ctx->ws_gen;
  s->cap_flow = s->flow;
  s->cap_flow_gen = s->flow ? flow_generation(s->flow) : 0;
  return PES_OK;
}

int pes_sampler_launch(pes_sampler* s, int64_t n_steps, void* stream) {
  if (!s || n_steps < 0) return PES_EINVAL;
  if (!s->exec) return PES_ESTATE;
  // the graph holds raw pointers into workspaces that a larger call since the
  // capture may have reallocated; replaying it then would touch freed memory
  if (s->ctx->ws_gen != s->cap_ws_gen || s->flow != s->cap_flow ||
      (s->flow && flow_generation(s->flow) != s->cap_flow_gen)) {
    snprintf(s->ctx->err, sizeof(s->ctx->err),
             "workspace reallocated or flow changed since the capture: capture the step again");
    return PES_ESTATE;
  }
  for (int64_t n = 0; n < n_steps; ++n) PES_HIP(s->ctx, hipGraphLaunch(s->exec, (hipStream_t)stream));
  return PES_OK;
}

int pes_sampler_state(pes_sampler* s, double* theta, double* logl, int64_t* accepts, uint64_t* steps,
                      void* stream) {
  if (!s) return PES_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (theta) PES_HIP(s->ctx, hipMemcpyAsync(theta, s->theta, sizeof(double) * s->B * 11, hipMemcpyDeviceToDevice, st));
  if (logl) PES_HIP(s->ctx, hipMemcpyAsync(logl, s->logl, sizeof(double) * s->B, hipMemcpyDeviceToDevice, st));
  if (accepts)
    PES_HIP(s->ctx, hipMemcpyAsync(accepts, s->accepts, sizeof(int64_t) * s->B, hipMemcpyDeviceToDevice, st));
  PES_HIP(s->ctx, hipStreamSynchronize(st));
  if (steps) PES_HIP(s->ctx, hipMemcpy(steps, s->step, sizeof(uint64_t), hipMemcpyDeviceToHost));
  return PES_OK;
}

int pes_sampler_chain(pes_sampler* s, const double** chain) {
  if (!s || !chain) return PES_EINVAL;
  *chain = s->chain;
  return PES_OK;
}

int pes_sampler_read_chain(pes_sampler* s, double* out, int64_t* n_states, void* stream) {
  if (!s || !out || !n_states) return PES_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  PES_HIP(s->ctx, hipStreamSynchronize(st));
  uint64_t step = 0;
  PES_HIP(s->ctx, hipMemcpy(&step, s->step, sizeof(uint64_t), hipMemcpyDeviceToHost));
  const int64_t L = s->chain_len;
  const int64_t n = std::min<int64_t>((int64_t)step, L);
  *n_states = n;
  if (n == 0) return PES_OK;
  const size_t row = sizeof(double) * s->B * 11;
  if ((int64_t)step <= L) {
    PES_HIP(s->ctx, hipMemcpyAsync(out, s->chain, row * n, hipMemcpyDeviceToDevice, st));
  } else {   // ring: the oldest state sits at step % L
    const int64_t o = (int64_t)(step % (uint64_t)L);
    PES_HIP(s->ctx, hipMemcpyAsync(out, s->chain + o * s->B * 11, row * (L - o), hipMemcpyDeviceToDevice, st));
    if (o > 0)
      PES_HIP(s->ctx, hipMemcpyAsync(out + (L - o) * s->B * 11, s->chain, row * o, hipMemcpyDeviceToDevice, st));
  }
  PES_HIP(s->ctx, hipStreamSynchronize(st));
  return PES_OK;
}

int pes_propose(pes_sampler* s, int kind, int half, double* theta_prop, double* log_qratio, void* stream) {
  if (!s || !theta_prop || !log_qratio || (half != 0 && half != 1) ||
      (kind != PES_PROPOSE_DE && kind != PES_PROPOSE_FLOW))
    return PES_EINVAL;
  if (kind == PES_PROPOSE_FLOW && !s->flow) return PES_ESTATE;
  return sampler_propose(s, de_args(s, half), kind == PES_PROPOSE_FLOW, theta_prop, log_qratio,
                         (hipStream_t)stream);
}

int pes_sampler_set_flow(pes_sampler* s, pes_flow* f, double p_flow) {
  if (!s || (f && !(p_flow >= 0.0 && p_flow <= 1.0))) return PES_EINVAL;
  if (!f) {
    s->flow = nullptr;
    s->p_flow = 0.0;
    return PES_OK;
  }
  for (int k = 0; k < kNParams; ++k)
    if (s->prior.kind[k] == PES_PRIOR_FIXED) return PES_EINVAL;
  const int64_t H = s->H1;
  if (!s->zbuf) {
    if (hipMalloc(&s->zbuf, sizeof(double) * H * 11) != hipSuccess ||
        hipMalloc(&s->fprop, sizeof(double) * H * 11) != hipSuccess ||
        hipMalloc(&s->lq_prop, sizeof(double) * H) != hipSuccess ||
        hipMalloc(&s->lq_cur, sizeof(double) * H) != hipSuccess)
      return PES_ENOMEM;
  }
  const int rc = flow_reserve(f, H);
  if (rc != PES_OK) return rc;
  s->flow = f;
  s->p_flow = p_flow;
  return PES_OK;
}

}  // extern "C"
