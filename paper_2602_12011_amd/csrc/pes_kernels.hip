// Kernels of libpes (gfx950): per-bin tables, data folding, per-walker
// setup, the (walker group, bin tile) work plan, the persistent log-likelihood
// kernel, the deterministic per-walker reduction and the response kernel.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "../../include/pes.h"
#include "pes_eval.hpp"
#include "pes_eval32.hpp"
#include "pes_launch.hpp"

namespace pes {

// ---------------------------------------------------------------- constants
// G M_sun / c^3 [s]; 1 Gpc / c [s]; Schwarzschild ISCO M f = 6^{-3/2} / pi.
constexpr double kMsunS = 4.925490947641267e-6;
constexpr double kGpcS = 3.085677581491367e25 / 299792458.0;
constexpr double kMfIsco = 0.068041381743977169 / kPi;
constexpr double kEulerGamma = 0.57721566490153286061;

// ---------------------------------------------------------------- bin tables
// Per bin: f, f^{1/3}, f^{-1/3}, f^{-7/6}, ln f.  Per detector: z, the common
// channel factor G, the weights of the analytic PSD with the TDI factor
// cancelled analytically, W_A = w_A |G|^2 / 2 = df a^2 / Q_A and
// W_T = w_T |G|^2 / 3 = df a^2 / (3 Q_T), and the raw w_c = 4 df / S_c.
// The PSD: S_A = S_E = 8 sin^2 x Q_A, S_T = 16 sin^2 x Q_T (TDI 1.5, x = 2 pi f L),
// times 4 sin^2 2x for TDI 2.0, with Q_A = (2 + cos x) S_oms + 2 (3 + 2 cos x +
// cos 2x) S_acc and Q_T = 2 sin^2(x/2) (S_oms + 4 sin^2(x/2) S_acc).
__global__ void bin_tables_kernel(double* __restrict__ bins, double* __restrict__ tabs,
                                  int64_t N, double f0, double df, int n_det, DetTable dt) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const double f = fma((double)k, df, f0);
  bins[B_F * N + k] = f;
  const double f13 = cbrt(f);
  bins[B_F13 * N + k] = f13;
  bins[B_FM13 * N + k] = 1.0 / f13;
  bins[B_FM76 * N + k] = 1.0 / (f * sqrt(f13));   // f^{-7/6} = 1 / (f f^{1/6})
  bins[B_LNF * N + k] = log(f);
  for (int d = 0; d < n_det; ++d) {
    const DetParams& p = dt.p[d];
    double* t = tabs + (int64_t)d * T_NFIELDS * N;
    const double a = kPi * f * p.L;   // pi f L
    const double x = 2.0 * a;
    double sx, cx, s2x, c2x, sh, ch;
    sincos(x, &sx, &cx);
    sincos(2.0 * x, &s2x, &c2x);
    sincos(0.5 * x, &sh, &ch);
    const double twopif = 2.0 * kPi * f;
    const double r1 = 2e-3 / f, r2 = 4e-4 / f, r3 = f / 8e-3;
    const double c = 299792458.0;
    const double Soms = p.oms2 * (1.0 + r1 * r1 * r1 * r1) * (twopif / c) * (twopif / c);
    const double Sacc = p.acc2 * (1.0 + r2 * r2) * (1.0 + r3 * r3 * r3 * r3) /
                        ((twopif * c) * (twopif * c));
    const double QA = (2.0 + cx) * Soms + 2.0 * (3.0 + 2.0 * cx + c2x) * Sacc;
    const double QT = 2.0 * sh * sh * (Soms + 4.0 * sh * sh * Sacc);
    double SA = 8.0 * sx * sx * QA, ST = 16.0 * sx * sx * QT;
    double Gr, Gi;
    double ph;  // G = |G| e^{-i ph}
    double gmag;
    if (p.tdi_gen == 20) {
      SA *= 4.0 * s2x * s2x;
      ST *= 4.0 * s2x * s2x;
      // G = (1 - z^2)(1 - z^4)(-i a) e^{-i a} = 4 i a sin x sin 2x e^{-3.5 i x}
      gmag = 4.0 * a * sx * s2x;
      ph = 3.5 * x - 0.5 * kPi;   // i = e^{+i pi/2}
    } else {
      // G = (1 - z^2)(-i a) e^{-i a} = 2 a sin x e^{-1.5 i x}
      gmag = 2.0 * a * sx;
      ph = 1.5 * x;
    }
    double sph, cph;
    sincos(ph, &sph, &cph);
    Gr = gmag * cph;
    Gi = -gmag * sph;
    double zs, zc;
    sincos(x, &zs, &zc);
    t[T_ZR * N + k] = zc;
    t[T_ZI * N + k] = -zs;
    const bool okA = SA != 0.0, okT = ST != 0.0;
    t[T_WA * N + k] = okA ? df * a * a / QA : 0.0;
    t[T_WT * N + k] = okT ? df * a * a / (3.0 * QT) : 0.0;
    t[T_WAE * N + k] = okA ? 4.0 * df / SA : 0.0;
    t[T_WTT * N + k] = okT ? 4.0 * df / ST : 0.0;
    t[T_A * N + k] = a;
    t[T_GR * N + k] = Gr;
    t[T_GI * N + k] = Gi;
    t[T_DAR * N + k] = 0.0;
    t[T_DAI * N + k] = 0.0;
    t[T_DER * N + k] = 0.0;
    t[T_DEI * N + k] = 0.0;
    t[T_DTR * N + k] = 0.0;
    t[T_DTI * N + k] = 0.0;
  }
}

// ---------------------------------------------------------------- data
// D_c = w_c n_c conj(G) d_c with n = (1/sqrt2, 1/sqrt6, 1/sqrt3), and per-block
// partial sums of <d|d> = sum_c w_c |d_c|^2 (fixed-order reduction).
__global__ void set_data_kernel(const double* __restrict__ d, double* __restrict__ tabs,
                                double* __restrict__ dd_part, int64_t N, int n_det) {
  __shared__ double red[256 / 64];
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double acc = 0.0;
  if (k < N) {
    for (int det = 0; det < n_det; ++det) {
      double* t = tabs + (int64_t)det * T_NFIELDS * N;
      const double Gr = t[T_GR * N + k], Gi = t[T_GI * N + k];
      const double wA = t[T_WAE * N + k], wT = t[T_WTT * N + k];
      const double nrm[3] = {0.70710678118654752440, 0.40824829046386301637,
                             0.57735026918962576451};
      const int fr[3] = {T_DAR, T_DER, T_DTR};
      for (int c = 0; c < 3; ++c) {
        const double w = (c == 2) ? wT : wA;
        const double dr = d[2 * ((det * 3 + c) * N + k)];
        const double di = d[2 * ((det * 3 + c) * N + k) + 1];
        // conj(G) d
        const double cr = Gr * dr + Gi * di, ci = Gr * di - Gi * dr;
        t[fr[c] * N + k] = w * nrm[c] * cr;
        t[(fr[c] + 1) * N + k] = w * nrm[c] * ci;
        acc += w * (dr * dr + di * di);
      }
    }
  }
  acc = wave_sum(acc);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    dd_part[blockIdx.x] = s;
  }
}

// Fixed-order sum of the block partials (one block).
__global__ void sum_kernel(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double red[1024 / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += part[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    out[0] = s;
  }
}

// ---------------------------------------------------------------- walker setup
// theta -> per-walker constant table (TaylorF2 stand-in, leading-order mode
// amplitudes, -2Y_lm closed forms, sky basis, orbit projection coefficients).
// Written once over a scalar type T: double for the values, Dual<11> for their
// derivatives with respect to theta.
template <class T>
__device__ void ylm_pair(int l, int m, const T& iota, T& yp, T& ym) {
  // -2Y_{l,+m}(iota, 0) and -2Y_{l,-m}(iota, 0)
  const T C = cos(0.5 * iota), S = sin(0.5 * iota), c = cos(iota);
  const T C2 = C * C, S2 = S * S, C4 = C2 * C2, S4 = S2 * S2;
  if (l == 2 && m == 2) {
    yp = sqrt(5.0 / (64.0 * kPi)) * ((1.0 + c) * (1.0 + c));
    ym = sqrt(5.0 / (64.0 * kPi)) * ((1.0 - c) * (1.0 - c));
  } else if (l == 2 && m == 1) {
    yp = sqrt(5.0 / (16.0 * kPi)) * (sin(iota) * (1.0 + c));
    ym = sqrt(5.0 / (16.0 * kPi)) * (sin(iota) * (1.0 - c));
  } else if (l == 3 && m == 3) {
    yp = -sqrt(21.0 / (2.0 * kPi)) * (C4 * C * S);
    ym = sqrt(21.0 / (2.0 * kPi)) * (C * S4 * S);
  } else if (l == 3 && m == 2) {
    yp = sqrt(7.0 / (4.0 * kPi)) * (C4 * (3.0 * c - 2.0));
    ym = sqrt(7.0 / (4.0 * kPi)) * (S4 * (3.0 * c + 2.0));
  } else {  // (4, 4)
    yp = 3.0 * sqrt(7.0 / kPi) * (C4 * C2 * S2);
    ym = 3.0 * sqrt(7.0 / kPi) * (C2 * S4 * S2);
  }
}

__device__ bool theta_valid(const double* th) {
  bool ok = true;
  for (int i = 0; i < 11; ++i) ok = ok && isfinite(th[i]);
  return ok && th[0] > 0.0 && th[1] > 0.0 && th[1] <= 1.0 && fabs(th[2]) < 1.0 &&
         fabs(th[3]) < 1.0 && th[4] > 0.0;
}

// Output of the setup: plain values, or value and one tangent per entry.
struct ValOut {
  double* w;
  __device__ void operator()(int i, double x) const { w[i] = x; }
};
struct TanOut {
  double* w;    // values, written by the k == 0 thread
  double* t;    // tangents [W_STRIDE][kNParams]
  int k;
  __device__ void operator()(int i, const Dual<1>& x) const {
    if (k == 0) w[i] = x.v;
    t[i * kNParams + k] = x.d[0];
  }
};

// arg of the harmonic factor of mode (l, m) in quarter turns (pi/2 each).
__host__ __device__ inline int argu_quarters(int l, int m) {
  if ((l == 2 && m == 1) || (l == 3 && m == 3)) return -1;
  if ((l == 3 && m == 2) || (l == 4 && m == 4)) return 2;
  return 0;
}

// Sky basis: source direction (lam, beta), k = -nhat, polarization axes p, q
// rotated by psi.
template <class T>
__device__ void sky_basis(const T& lam, const T& beta, const T& psi, T kv[3], T pv[3], T qv[3]) {
  const T cl = cos(lam), sl = sin(lam), cb = cos(beta), sb = sin(beta);
  const T cps = cos(psi), sps = sin(psi);
  kv[0] = -(cb * cl);
  kv[1] = -(cb * sl);
  kv[2] = -sb;
  const T uu[3] = {-sl, cl, T(0.0)};
  const T vv[3] = {-(sb * cl), -(sb * sl), cb};
  for (int i = 0; i < 3; ++i) {
    pv[i] = cps * uu[i] + sps * vv[i];
    qv[i] = sps * (-1.0 * uu[i]) + cps * vv[i];
  }
}

// Writes the W_STRIDE entries of a physical theta's table through `put`;
// returns the highest mode cutoff [Hz].
template <class T, class Out>
__device__ double setup_walker(const T* th, const SetupArgs& sa, const Out& put, int part = -1) {
  // part < 0: the whole table.  Otherwise one share of it, so that several
  // threads build one walker's table together: part 0 the header and the
  // unused blocks, part 1 + j mode j, part 1 + n_modes + d detector d.
  const bool all = part < 0;
  if (all) {
    for (int i = 0; i < W_STRIDE; ++i) put(i, T(0.0));
  } else if (part == 0) {
    for (int i = 0; i < W_MODE0; ++i) put(i, T(0.0));
    for (int i = W_MODE0 + sa.n_modes * W_MODE_STRIDE; i < W_DET0; ++i) put(i, T(0.0));
    for (int i = W_DET0 + sa.n_det * W_DET_STRIDE; i < W_ROT0; ++i) put(i, T(0.0));
    for (int i = W_ROT0 + sa.n_modes * R_STRIDE; i < W_STRIDE; ++i) put(i, T(0.0));
  }
  const T M = th[0] * kMsunS;
  const T q = th[1];
  const T eta = q / ((1.0 + q) * (1.0 + q));
  const T delta = (1.0 - q) / (1.0 + q);
  const T chi1 = th[2], chi2 = th[3];
  const T chis = 0.5 * (chi1 + chi2), chia = 0.5 * (chi1 - chi2);
  const T DL = th[4] * kGpcS;
  const T iota = th[5], phic = th[6], lam = th[7], beta = th[8], psi = th[9], tc = th[10];
  // TaylorF2 coefficients psi_k (+ ln v parts) -- 3.5PN, aligned spins
  const double p0 = 1.0;
  const T p2 = 3715.0 / 756.0 + 55.0 / 9.0 * eta;
  const T p3 = -16.0 * kPi + (113.0 / 3.0 - 76.0 / 3.0 * eta) * chis + 113.0 / 3.0 * (delta * chia);
  const T p4 = 15293365.0 / 508032.0 + 27145.0 / 504.0 * eta + 3085.0 / 72.0 * (eta * eta) -
               10.0 * (79.0 / 8.0) * (eta * chi1 * chi2);
  const T p5 = kPi * (38645.0 / 756.0 - 65.0 / 9.0 * eta);
  const T p5l = 3.0 * p5;
  const T p6 = (11583231236531.0 / 4694215680.0 - 640.0 / 3.0 * kPi * kPi -
                6848.0 / 21.0 * kEulerGamma - 6848.0 / 21.0 * log(4.0)) +
               (-15737765635.0 / 3048192.0 + 2255.0 / 12.0 * kPi * kPi) * eta +
               76055.0 / 1728.0 * (eta * eta) - 127825.0 / 1296.0 * (eta * eta * eta);
  const double p6l = -6848.0 / 21.0;
  const T p7 = kPi * (77096675.0 / 254016.0 + 378515.0 / 1512.0 * eta - 74045.0 / 756.0 * (eta * eta));
  if (all || part == 0) {
    put(W_VALID, T(1.0));
    put(W_TC, tc);
  }
  double fmx = 0.0;
  for (int j = 0; j < sa.n_modes; ++j) {
    const int l = sa.modes[j].l, m = sa.modes[j].m;
    const int M0 = W_MODE0 + j * W_MODE_STRIDE;
    const double mm = (double)m;
    const T fcut = (0.5 * mm * kMfIsco) / M;
    fmx = fmx > val(fcut) ? fmx : val(fcut);
    if (!(all || part == 1 + j)) continue;
    const T cm = cbrt(M * (kTwoPi / mm));
    put(M0 + M_CM, cm);
    put(M0 + M_CMI, 1.0 / cm);
    put(M0 + M_LNCM, log(cm));
    // phase in cycles: (m/2) * 3/(128 eta) * sum_k psi_k v^{k-5} / (2 pi)
    const T pref = (0.5 * mm * 3.0 / 128.0 / kTwoPi) / eta;
    // constant phase: -(m/2) phi_c - pi/4 - arg(unit_lm), in cycles
    const double argu = 0.5 * kPi * (double)argu_quarters(l, m);
    put(M0 + M_C0, pref * p5 + (-0.5 * mm / kTwoPi) * phic + (-0.25 * kPi - argu) / kTwoPi);
    put(M0 + M_A0, pref * p0);
    put(M0 + M_A2, pref * p2);
    put(M0 + M_A3, pref * p3);
    put(M0 + M_A4, pref * p4);
    put(M0 + M_B5, pref * p5l);
    put(M0 + M_A6, pref * p6);
    put(M0 + M_B6, pref * p6l);
    put(M0 + M_A7, pref * p7);
    // t_f - t_c = M/(256 eta) sum_k [(k-5) psi_k + psi_k^{ln}] v^{k-8}, mode-scaled v
    const T tpref = M / (256.0 * eta);
    put(M0 + M_T0, tpref * (-5.0 * p0));
    put(M0 + M_T2, tpref * (-3.0 * p2));
    put(M0 + M_T3, tpref * (-2.0 * p3));
    put(M0 + M_T4, tpref * (-1.0 * p4));
    put(M0 + M_T5, tpref * p5l);
    put(M0 + M_T6, tpref * (p6 + p6l));
    put(M0 + M_T6L, tpref * p6l);
    put(M0 + M_T7, tpref * (2.0 * p7));
    // amplitude sqrt(2/m) pi sqrt(2 eta/3) M^2 v^{-7/2} |H_lm(v)| / D_L, v^{-7/2} = cm^{-7/2} f^{-7/6}
    const T apref = (sqrt(2.0 / mm) * kPi) * sqrt(eta * (2.0 / 3.0)) * (M * M) / DL /
                    (cm * cm * cm * sqrt(cm));
    T h0 = T(0.0), h1 = T(0.0), h2 = T(0.0);
    if (l == 2 && m == 2) h0 = T(1.0);
    if (l == 2 && m == 1) h1 = delta / 3.0;
    if (l == 3 && m == 3) h1 = 0.75 * sqrt(15.0 / 14.0) * delta;
    if (l == 3 && m == 2) h2 = sqrt(5.0 / 7.0) / 3.0 * (1.0 - 3.0 * eta);
    if (l == 4 && m == 4) h2 = 8.0 / 9.0 * sqrt(5.0 / 7.0) * (1.0 - 3.0 * eta);
    put(M0 + M_AM0, apref * h0);
    put(M0 + M_AM1, apref * h1);
    put(M0 + M_AM2, apref * h2);
    T yp, ym;
    ylm_pair(l, m, iota, yp, ym);
    const double sgn = (l & 1) ? -1.0 : 1.0;
    const T kp = 0.5 * (ym + sgn * yp), kc = ym - sgn * yp;   // K_+, 2 K_x
    put(M0 + M_KP, kp);
    put(M0 + M_KC, kc);
    // the same factors on the phase of the first mode with this m:
    // rot = e^{i (arg_j - arg_lead)} = i^q exactly
    int lead = j;
    for (int i = j - 1; i >= 0; --i)
      if (sa.modes[i].m == m) lead = i;
    const int q = (((argu_quarters(l, m) - argu_quarters(sa.modes[lead].l, m)) % 4) + 4) % 4;
    const double rr = q == 0 ? 1.0 : (q == 2 ? -1.0 : 0.0), ri = q == 1 ? 1.0 : (q == 3 ? -1.0 : 0.0);
    const int R0 = W_ROT0 + R_STRIDE * j;
    put(R0 + R_KPR, kp * rr);
    put(R0 + R_KPI, kp * ri);
    put(R0 + R_KCR, kc * rr);
    put(R0 + R_KCI, kc * ri);
    put(M0 + M_FCI, 1.0 / fcut);
  }
  if (all || part == 0) put(W_FMAX, T(fmx));
  if (!(all || part > sa.n_modes)) return fmx;
  T kv[3], pv[3], qv[3];
  sky_basis(lam, beta, psi, kv, pv, qv);
  for (int d = 0; d < sa.n_det; ++d) {
    if (!(all || part == 1 + sa.n_modes + d)) continue;
    const DetParams& P = sa.dt.p[d];
    const int D0 = W_DET0 + d * W_DET_STRIDE;
    put(D0 + D_AO, tc * P.inv_year + P.phase0_cyc);
    put(D0 + D_PO, tc * P.inv_ptq);
    for (int t = 0; t < 2; ++t) {
      const int s1 = (t + 1) % 3, s2 = (t + 2) % 3;
      for (int i = 0; i < 5; ++i) {
        T kn = T(0.0), np = T(0.0), nq = T(0.0), kd = T(0.0);
        for (int c = 0; c < 3; ++c) {
          const double n = (P.G[s2][c][i] - P.G[s1][c][i]) / P.L;
          kn = kn + kv[c] * n;
          np = np + pv[c] * n;
          nq = nq + qv[c] * n;
          kd = kd + kv[c] * P.G[t][c][i];
        }
        put(D0 + D_KN + 5 * t + i, kn);
        put(D0 + D_NP + 5 * t + i, np);
        put(D0 + D_NQ + 5 * t + i, nq);
        put(D0 + D_KD + 5 * t + i, kd);
      }
    }
    put(D0 + D_KR, P.AUc * kv[0]);
    put(D0 + D_KR + 1, P.AUc * kv[1]);
  }
  return fmx;
}

__device__ int active_tiles(double fmx, const SetupArgs& sa, int tile) {
  if (sa.full_tiles) return (int)((sa.N + tile - 1) / tile);
  // active bins: f_k < fmax (upper bound; the kernels test each mode exactly)
  double nb = ceil((fmx - sa.f0) / sa.df) + 1.0;
  nb = fmin(fmax(nb, 0.0), (double)sa.N);
  const int64_t nact = (int64_t)nb;
  return (int)((nact + tile - 1) / tile);
}

// One thread per (walker, share of its table), 1 + n_modes + n_det shares:
// blockIdx.y is the share, so a wavefront runs one share for 64 walkers and
// the shares of one walker run side by side in different wavefronts.
__global__ void setup_kernel(const double* __restrict__ theta, int64_t B, double* __restrict__ wtab,
                             int* __restrict__ ntiles, SetupArgs sa) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int part = blockIdx.y;
  const double* th = theta + 11 * b;
  double* w = wtab + b * W_STRIDE;
  if (!theta_valid(th)) {
    if (part == 0) {
      for (int i = 0; i < W_STRIDE; ++i) w[i] = 0.0;
      ntiles[b] = 0;
    }
    return;
  }
  const double fmx = setup_walker<double>(th, sa, ValOut{w}, part);
  if (part == 0) ntiles[b] = active_tiles(fmx, sa, sa.tile);
}

// Exact Kepler orbits: each walker's projections of the detectors' orbit
// series onto its sky basis, one thread per (walker, detector).  Rows of a
// geocentric detector, and of an unphysical walker, are left zero (the
// evaluation never reads them).
__global__ void kepler_proj_kernel(const double* __restrict__ theta, int64_t B, const double* __restrict__ kep,
                                   SetupArgs sa, double* __restrict__ wkep) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * sa.n_det) return;
  const int64_t b = i / sa.n_det;
  const int d = (int)(i - b * sa.n_det);
  double* __restrict__ out = wkep + i * KW_STRIDE;
  const double* th = theta + b * 11;
  if (sa.dt.p[d].kind == 2 || !theta_valid(th)) {
    for (int j = 0; j < KW_STRIDE; ++j) out[j] = 0.0;
    return;
  }
  double kv[3], pv[3], qv[3];
  sky_basis(th[7], th[8], th[9], kv, pv, qv);
  const double* __restrict__ v = kep + d * KV_STRIDE;
  for (int j = 0; j < kKepT; ++j) {
    double c[15] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int x = 0; x < 3; ++x) {
      const double d0 = v[KV_D0 + x * kKepT + j], d1 = v[KV_D1 + x * kKepT + j];
      const double x0 = v[KV_X0 + x * kKepT + j], x1 = v[KV_X1 + x * kKepT + j], xc = v[KV_C + x * kKepT + j];
      c[0] = fma(kv[x], d0, c[0]);
      c[1] = fma(kv[x], d1, c[1]);
      c[2] = fma(pv[x], d0, c[2]);
      c[3] = fma(pv[x], d1, c[3]);
      c[4] = fma(qv[x], d0, c[4]);
      c[5] = fma(qv[x], d1, c[5]);
      c[6] = fma(kv[x], x0, c[6]);
      c[7] = fma(kv[x], x1, c[7]);
      c[8] = fma(kv[x], xc, c[8]);
      c[9] = fma(pv[x], x0, c[9]);
      c[10] = fma(pv[x], x1, c[10]);
      c[11] = fma(qv[x], x0, c[11]);
      c[12] = fma(qv[x], x1, c[12]);
      c[13] = fma(pv[x], xc, c[13]);
      c[14] = fma(qv[x], xc, c[14]);
    }
    for (int f = 0; f < 15; ++f) out[f * kKepT + j] = c[f];
  }
  for (int j = 15 * kKepT; j < KW_STRIDE; ++j) out[j] = 0.0;
}

// Derivatives of the projected series in the sky angles: the series projected
// on the derivatives of the sky basis, one thread per (walker, detector, angle
// s = lambda, beta, psi).  wkept[b][d][s][KW_STRIDE]; zero rows as above.
__global__ void kepler_proj_tan_kernel(const double* __restrict__ theta, int64_t B, const double* __restrict__ kep,
                                       SetupArgs sa, double* __restrict__ wkept) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * sa.n_det * 3) return;
  const int64_t b = i / (sa.n_det * 3);
  const int r = (int)(i - b * sa.n_det * 3);
  const int d = r / 3, sk = r - 3 * d;
  double* __restrict__ out = wkept + i * KW_STRIDE;
  const double* th = theta + b * 11;
  if (sa.dt.p[d].kind == 2 || !theta_valid(th)) {
    for (int j = 0; j < KW_STRIDE; ++j) out[j] = 0.0;
    return;
  }
  Dual<1> ang[3];
  for (int q = 0; q < 3; ++q) {
    ang[q] = Dual<1>(th[7 + q]);
    ang[q].d[0] = q == sk ? 1.0 : 0.0;
  }
  Dual<1> kd[3], pd[3], qd[3];
  sky_basis(ang[0], ang[1], ang[2], kd, pd, qd);
  double kv[3], pv[3], qv[3];
  for (int x = 0; x < 3; ++x) {
    kv[x] = kd[x].d[0];
    pv[x] = pd[x].d[0];
    qv[x] = qd[x].d[0];
  }
  const double* __restrict__ v = kep + d * KV_STRIDE;
  for (int j = 0; j < kKepT; ++j) {
    double c[15] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int x = 0; x < 3; ++x) {
      const double d0 = v[KV_D0 + x * kKepT + j], d1 = v[KV_D1 + x * kKepT + j];
      const double x0 = v[KV_X0 + x * kKepT + j], x1 = v[KV_X1 + x * kKepT + j], xc = v[KV_C + x * kKepT + j];
      c[0] = fma(kv[x], d0, c[0]);
      c[1] = fma(kv[x], d1, c[1]);
      c[2] = fma(pv[x], d0, c[2]);
      c[3] = fma(pv[x], d1, c[3]);
      c[4] = fma(qv[x], d0, c[4]);
      c[5] = fma(qv[x], d1, c[5]);
      c[6] = fma(kv[x], x0, c[6]);
      c[7] = fma(kv[x], x1, c[7]);
      c[8] = fma(kv[x], xc, c[8]);
      c[9] = fma(pv[x], x0, c[9]);
      c[10] = fma(pv[x], x1, c[10]);
      c[11] = fma(qv[x], x0, c[11]);
      c[12] = fma(qv[x], x1, c[12]);
      c[13] = fma(pv[x], xc, c[13]);
      c[14] = fma(qv[x], xc, c[14]);
    }
    for (int f = 0; f < 15; ++f) out[f * kKepT + j] = c[f];
  }
  for (int j = 15 * kKepT; j < KW_STRIDE; ++j) out[j] = 0.0;
}

// Values and theta-derivatives of the walker table, wtan[b][i][k] = d w_i / d theta_k:
// one thread per (walker, direction k) carrying a single tangent.
__global__ void setup_tan_kernel(const double* __restrict__ theta, int64_t B, double* __restrict__ wtab,
                                 double* __restrict__ wtan, int* __restrict__ ntiles, SetupArgs sa) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= B * kNParams) return;
  const int64_t b = g / kNParams;
  const int k = (int)(g - b * kNParams);
  const double* th = theta + 11 * b;
  double* w = wtab + b * W_STRIDE;
  double* wt = wtan + b * W_STRIDE * kNParams;
  if (!theta_valid(th)) {
    for (int i = 0; i < W_STRIDE; ++i) {
      if (k == 0) w[i] = 0.0;
      wt[i * kNParams + k] = 0.0;
    }
    if (k == 0) ntiles[b] = 0;
    return;
  }
  Dual<1> thd[kNParams];
  for (int i = 0; i < kNParams; ++i) {
    thd[i] = Dual<1>(th[i]);
    thd[i].d[0] = (i == k) ? 1.0 : 0.0;
  }
  const double fmx = setup_walker<Dual<1>>(thd, sa, TanOut{w, wt, k});
  if (k == 0) ntiles[b] = active_tiles(fmx, sa, sa.tile);
}

// ---------------------------------------------------------------- work plan
// One block: counting sort of the walkers by active tile count (descending,
// keys quantized to at most kPlanKeys buckets), walker groups of `wg`
// consecutive sorted walkers, each group's tile count (its maximum), their
// exclusive prefix sum (group-major work items), and the queue counters.
constexpr int kPlanKeys = 8192;

// Exclusive scan, in place, of n ints in global memory by one 1024-thread
// block (each thread owns a contiguous chunk); returns the total to every thread.
__device__ int block_exclusive_scan(int* __restrict__ a, int n, int* wsum) {
  const int per = (n + 1023) / 1024;
  const int base = threadIdx.x * per;
  int local = 0;
  for (int i = 0; i < per; ++i)
    if (base + i < n) local += a[base + i];
  int incl = local;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    const int o = __shfl_up(incl, off, 64);
    if (lane >= off) incl += o;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int i = 0; i < 1024 / 64; ++i) {
      const int t = wsum[i];
      wsum[i] = run;
      run += t;
    }
    wsum[16] = run;
  }
  __syncthreads();
  int run = incl - local + wsum[wv];
  for (int i = 0; i < per; ++i)
    if (base + i < n) {
      const int h = a[base + i];
      a[base + i] = run;
      run += h;
    }
  const int total = wsum[16];
  __syncthreads();
  return total;
}

__global__ void __launch_bounds__(1024) plan_kernel(const int* __restrict__ ntiles, int B, int wg,
                                                    int ntmax, int sorted, int* __restrict__ perm,
                                                    int* __restrict__ gstart, int* __restrict__ counters) {
  __shared__ int hist[kPlanKeys];
  __shared__ int wsum[17];
  if (sorted) {  // counting sort by descending tile count
    int shift = 0;
    while ((ntmax >> shift) >= kPlanKeys) ++shift;
    const int nkeys = (ntmax >> shift) + 1;   // tile counts 0 .. ntmax
    for (int i = threadIdx.x; i < nkeys; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
      const int key = nkeys - 1 - (ntiles[b] >> shift);   // descending tile counts
      atomicAdd(&hist[key], 1);
    }
    __syncthreads();
    {  // exclusive scan of the histogram in LDS (a contiguous chunk per thread)
      const int per = (nkeys + 1023) / 1024;
      const int base = threadIdx.x * per;
      int local = 0;
      for (int i = 0; i < per; ++i)
        if (base + i < nkeys) local += hist[base + i];
      int incl = local;
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
      for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
      }
      if (lane == 63) wsum[wv] = incl;
      __syncthreads();
      if (threadIdx.x == 0) {
        int run = 0;
        for (int i = 0; i < 1024 / 64; ++i) {
          const int t = wsum[i];
          wsum[i] = run;
          run += t;
        }
      }
      __syncthreads();
      int run = incl - local + wsum[wv];
      for (int i = 0; i < per; ++i) {
        if (base + i >= nkeys) break;
        const int h = hist[base + i];
        hist[base + i] = run;
        run += h;
      }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < B; b += blockDim.x) {
      const int key = nkeys - 1 - (ntiles[b] >> shift);
      const int pos = atomicAdd(&hist[key], 1);
      perm[pos] = b;
    }
  } else {  // batch order
    for (int b = threadIdx.x; b < B; b += blockDim.x) perm[b] = b;
  }
  __syncthreads();
  // each group's tile count (the maximum over its walkers), then the
  // exclusive prefix over groups: work item i belongs to the group g with
  // gstart[g] <= i < gstart[g + 1], tile i - gstart[g]
  const int ng = (B + wg - 1) / wg;
  for (int g = threadIdx.x; g < ng; g += blockDim.x) {
    int mx = 0;
    for (int s = 0; s < wg; ++s) {
      const int idx = g * wg + s;
      if (idx < B) {
        const int nt = ntiles[perm[idx]];
        mx = nt > mx ? nt : mx;
      }
    }
    gstart[g] = mx;
  }
  __syncthreads();
  const int total = block_exclusive_scan(gstart, ng, wsum);
  if (threadIdx.x == 0) {
    gstart[ng] = total;
    counters[0] = 0;      // ticket
    counters[1] = total;  // number of work items
  }
}

// ---------------------------------------------------------------- log-likelihood
// Persistent kernel: each block takes (group, tile) items from an atomic
// ticket.  Lanes own bins; the walkers of the group are processed in turn,
// each lane evaluating its bins, then a wavefront reduction and one LDS slot
// per (walker, wave).  partial[w][tile] = (<d|h>, <h|h>) of that tile.
template <int BPL, bool LS, bool F32, bool KEP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
    loglike_kernel(const double* __restrict__ bins, const double* __restrict__ tabs,
                   const double* __restrict__ wtab, const int* __restrict__ ntiles,
                   const int* __restrict__ perm, const int* __restrict__ gstart,
                   int* __restrict__ counters, double* __restrict__ partial, LoglikeArgs A) {
  __shared__ double acc[kMaxGroup][4][2];
  __shared__ int s_item[2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t N = A.N;
  const int tile = 256 * BPL;
  while (true) {
    if (threadIdx.x == 0) {
      const int it = A.grid_mode ? (int)blockIdx.x : atomicAdd(&counters[0], 1);
      int g = -1;
      if (it < counters[1]) {
        // group-major: largest g with gstart[g] <= it
        int lo = 0, hi = A.n_groups;   // gstart[lo] <= it < gstart[hi]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (gstart[mid] <= it) lo = mid; else hi = mid;
        }
        g = lo;
      }
      s_item[0] = it;
      s_item[1] = g;
    }
    __syncthreads();
    const int it = s_item[0];
    const int g = __builtin_amdgcn_readfirstlane(s_item[1]);
    if (g < 0) break;
    const int t = __builtin_amdgcn_readfirstlane(it - gstart[g]);
    const int64_t k0 = (int64_t)t * tile;
    for (int det = 0; det < A.n_det; ++det) {
      const double* __restrict__ tb = tabs + (int64_t)det * T_NFIELDS * N;
      BinRegs br[BPL];
      double zr[BPL], zi[BPL], dar[BPL], dai[BPL], der[BPL], dei[BPL], dtr[BPL], dti[BPL], wa[BPL],
          wtt[BPL], aa[BPL];
      bool in[BPL];
#pragma unroll
      for (int q = 0; q < BPL; ++q) {
        const int64_t k = k0 + q * 256 + threadIdx.x;
        in[q] = k < N;
        const int64_t kk = in[q] ? k : N - 1;
        br[q].f = bins[B_F * N + kk];
        br[q].f13 = bins[B_F13 * N + kk];
        br[q].fm13 = bins[B_FM13 * N + kk];
        br[q].fm76 = bins[B_FM76 * N + kk];
        br[q].lnf = bins[B_LNF * N + kk];
        zr[q] = tb[T_ZR * N + kk];
        zi[q] = tb[T_ZI * N + kk];
        dar[q] = tb[T_DAR * N + kk];
        dai[q] = tb[T_DAI * N + kk];
        der[q] = tb[T_DER * N + kk];
        dei[q] = tb[T_DEI * N + kk];
        dtr[q] = tb[T_DTR * N + kk];
        dti[q] = tb[T_DTI * N + kk];
        wa[q] = in[q] ? tb[T_WA * N + kk] : 0.0;
        wtt[q] = in[q] ? tb[T_WT * N + kk] : 0.0;
        aa[q] = tb[T_A * N + kk];
        if (!in[q]) { dar[q] = dai[q] = der[q] = dei[q] = dtr[q] = dti[q] = 0.0; }
      }
      const DetParams& P = A.dt.p[det];
      // fit class of each of this wave's bin sets (wave-uniform)
      int cls[BPL];
#pragma unroll
      for (int q = 0; q < BPL; ++q) cls[q] = __builtin_amdgcn_readfirstlane(fit_class(2.0 * wave_max(aa[q])));
      for (int s = 0; s < A.wg; ++s) {
        const int idx = g * A.wg + s;
        if (idx >= A.B) break;
        const int w = __builtin_amdgcn_readfirstlane(perm[idx]);
        if (t >= ntiles[w]) continue;
        const double* __restrict__ wt = wtab + (int64_t)w * W_STRIDE;
        double dh = 0.0, hh = 0.0;
#pragma unroll
        for (int q = 0; q < BPL; ++q) {
          Chan c;
          if constexpr (F32) {
            const float* __restrict__ ws = A.wtab32 + (int64_t)w * W_STRIDE;
            ChanT<float> cf;
            if (P.kind == 2) {
              cf = eval_channels_f32_cls<true, LS>(cls[q], wt, ws, det, A.plan, P.inv_year, P.inv_ptq, br[q],
                                                   (float)aa[q], (float)zr[q], (float)zi[q]);
            } else if constexpr (KEP) {
              const float* __restrict__ kw = A.wkep32 + ((int64_t)w * A.n_det + det) * KW_STRIDE;
              const float* __restrict__ kinv = A.kep32 + det * KV_STRIDE + KV_INVL;
              cf = eval_channels_f32_cls<false, LS, true>(cls[q], wt, ws, det, A.plan, P.inv_year, P.inv_ptq,
                                                          br[q], (float)aa[q], (float)zr[q], (float)zi[q], kw, kinv);
            } else {
              cf = eval_channels_f32_cls<false, LS>(cls[q], wt, ws, det, A.plan, P.inv_year, P.inv_ptq, br[q],
                                                    (float)aa[q], (float)zr[q], (float)zi[q]);
            }
            c = Chan{cf.ar, cf.ai, cf.er, cf.ei, cf.tr, cf.ti};
          } else if (P.kind == 2) {
            c = eval_channels_cls<true, LS>(cls[q], wt, det, A.plan, P.inv_year, P.inv_ptq, br[q], aa[q], zr[q],
                                            zi[q]);
          } else if constexpr (KEP) {
            const double* __restrict__ kw = A.wkep + ((int64_t)w * A.n_det + det) * KW_STRIDE;
            const double* __restrict__ kinv = A.kep + det * KV_STRIDE + KV_INVL;
            c = eval_channels_cls<false, LS, true>(cls[q], wt, det, A.plan, P.inv_year, P.inv_ptq, br[q], aa[q],
                                                   zr[q], zi[q], kw, kinv);
          } else {
            c = eval_channels_cls<false, LS>(cls[q], wt, det, A.plan, P.inv_year, P.inv_ptq, br[q], aa[q], zr[q],
                                             zi[q]);
          }
          dh = fma(dar[q], c.ar, dh);
          dh = fma(dai[q], c.ai, dh);
          dh = fma(der[q], c.er, dh);
          dh = fma(dei[q], c.ei, dh);
          dh = fma(dtr[q], c.tr, dh);
          dh = fma(dti[q], c.ti, dh);
          const double a2 = fma(c.ar, c.ar, c.ai * c.ai) + (1.0 / 3.0) * fma(c.er, c.er, c.ei * c.ei);
          const double t2 = fma(c.tr, c.tr, c.ti * c.ti);
          hh = fma(wa[q], a2, fma(wtt[q], t2, hh));
        }
        dh = wave_sum_dpp(dh);
        hh = wave_sum_dpp(hh);
        if (lane == 0) {
          if (det == 0) {
            acc[s][wv][0] = dh;
            acc[s][wv][1] = hh;
          } else {
            acc[s][wv][0] += dh;
            acc[s][wv][1] += hh;
          }
        }
      }
    }
    __syncthreads();
    if (threadIdx.x < A.wg) {
      const int s = threadIdx.x;
      const int idx = g * A.wg + s;
      if (idx < A.B) {
        const int w = perm[idx];
        if (t < ntiles[w]) {
          const double dh = (acc[s][0][0] + acc[s][1][0]) + (acc[s][2][0] + acc[s][3][0]);
          const double hh = (acc[s][0][1] + acc[s][1][1]) + (acc[s][2][1] + acc[s][3][1]);
          // tile-major: partial[t][w] (coalesced for the per-walker reduction)
          double* p = partial + ((int64_t)t * A.B + w) * 2;
          p[0] = dh;
          p[1] = hh;
        }
      }
    }
    __syncthreads();
    if (A.grid_mode) break;
  }
}

// log L = <d|h> - <h|h>/2 - <d|d>/2.  partial is tile-major, [tile][walker][2].
// A block takes kFinW walkers; its kFinP thread rows each sum the tiles
// t = row, row + kFinP, ... of every walker (neighbouring threads read
// neighbouring walkers), then the row sums are combined in a fixed order, so
// the result does not depend on the launch or on the batch order.
constexpr int kFinW = 32, kFinP = 32;
__global__ void __launch_bounds__(kFinW * kFinP)
    finalize_kernel(const double* __restrict__ partial, const int* __restrict__ ntiles,
                    const double* __restrict__ wtab, const double* __restrict__ dd, int64_t B,
                    double* __restrict__ logl) {
  __shared__ double sh[kFinP][kFinW][2];
  const int wl = threadIdx.x % kFinW, row = threadIdx.x / kFinW;
  const int64_t b = (int64_t)blockIdx.x * kFinW + wl;
  double dh = 0.0, hh = 0.0;
  if (b < B) {
    const int nt = ntiles[b];
    for (int t = row; t < nt; t += kFinP) {
      const double* p = partial + ((int64_t)t * B + b) * 2;
      dh += p[0];
      hh += p[1];
    }
  }
  sh[row][wl][0] = dh;
  sh[row][wl][1] = hh;
  __syncthreads();
  for (int h = kFinP / 2; h > 0; h >>= 1) {   // pairwise tree over the rows
    if (row < h) {
      sh[row][wl][0] += sh[row + h][wl][0];
      sh[row][wl][1] += sh[row + h][wl][1];
    }
    __syncthreads();
  }
  if (row == 0 && b < B)
    logl[b] = wtab[b * W_STRIDE + W_VALID] == 0.0 ? -INFINITY
                                                  : (sh[0][wl][0] - 0.5 * sh[0][wl][1]) - 0.5 * dd[0];
}

// ---------------------------------------------------------------- response
// out[b][det][c][k] = n_c G(f_k) C''_c for one walker per blockIdx.y.
template <bool LS, bool F32, bool KEP>
__global__ void response_kernel(ResponseArgs A) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = blockIdx.y;
  if (k >= A.N) return;
  const double* __restrict__ wt = A.wtab + b * W_STRIDE;
  const int64_t N = A.N;
  const bool valid = wt[W_VALID] != 0.0;
  BinRegs br;
  br.f = A.bins[B_F * N + k];
  br.f13 = A.bins[B_F13 * N + k];
  br.fm13 = A.bins[B_FM13 * N + k];
  br.fm76 = A.bins[B_FM76 * N + k];
  br.lnf = A.bins[B_LNF * N + k];
  for (int det = 0; det < A.n_det; ++det) {
    const double* __restrict__ tb = A.tabs + (int64_t)det * T_NFIELDS * N;
    const DetParams& P = A.dt.p[det];
    Chan c = {0, 0, 0, 0, 0, 0};
    if (valid) {
      if constexpr (F32) {
        const float* __restrict__ ws = A.wtab32 + b * W_STRIDE;
        const float a = (float)tb[T_A * N + k], zr = (float)tb[T_ZR * N + k], zi = (float)tb[T_ZI * N + k];
        ChanT<float> cf;
        if (P.kind == 2) {
          cf = eval_channels_f32<true, LS, 1>(wt, ws, det, A.plan, P.inv_year, P.inv_ptq, br, a, zr, zi);
        } else if constexpr (KEP) {
          const float* __restrict__ kw = A.wkep32 + (b * A.n_det + det) * KW_STRIDE;
          const float* __restrict__ kinv = A.kep32 + det * KV_STRIDE + KV_INVL;
          cf = eval_channels_f32<false, LS, 1, true>(wt, ws, det, A.plan, P.inv_year, P.inv_ptq, br, a, zr, zi, kw,
                                                     kinv);
        } else {
          cf = eval_channels_f32<false, LS, 1>(wt, ws, det, A.plan, P.inv_year, P.inv_ptq, br, a, zr, zi);
        }
        c = Chan{cf.ar, cf.ai, cf.er, cf.ei, cf.tr, cf.ti};
      } else if (P.kind == 2) {
        c = eval_channels<true, LS>(wt, det, A.plan, P.inv_year, P.inv_ptq, br, tb[T_A * N + k], tb[T_ZR * N + k],
                                    tb[T_ZI * N + k]);
      } else if constexpr (KEP) {
        const double* __restrict__ kw = A.wkep + (b * A.n_det + det) * KW_STRIDE;
        const double* __restrict__ kinv = A.kep + det * KV_STRIDE + KV_INVL;
        c = eval_channels<false, LS, 1, true>(wt, det, A.plan, P.inv_year, P.inv_ptq, br, tb[T_A * N + k],
                                              tb[T_ZR * N + k], tb[T_ZI * N + k], kw, kinv);
      } else {
        c = eval_channels<false, LS>(wt, det, A.plan, P.inv_year, P.inv_ptq, br, tb[T_A * N + k], tb[T_ZR * N + k],
                                     tb[T_ZI * N + k]);
      }
    }
    const double Gr = tb[T_GR * N + k], Gi = tb[T_GI * N + k];
    const double nrm[3] = {0.70710678118654752440, 0.40824829046386301637, 0.57735026918962576451};
    const double cr[3] = {c.ar, c.er, c.tr}, ci[3] = {c.ai, c.ei, c.ti};
    for (int ch = 0; ch < 3; ++ch) {
      double* o = A.out + 2 * (((b * A.n_det + det) * 3 + ch) * N + k);
      o[0] = valid ? nrm[ch] * (Gr * cr[ch] - Gi * ci[ch]) : NAN;
      o[1] = valid ? nrm[ch] * (Gr * ci[ch] + Gi * cr[ch]) : NAN;
    }
  }
}

// FP32 copy of the walker tables (or of the orbit series) for the
// single-precision kernels.
__global__ void table32_kernel(const double* __restrict__ wtab, int64_t n, float* __restrict__ wtab32) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) wtab32[i] = (float)wtab[i];
}

// ---------------------------------------------------------------- stage probes
// The evaluation of the response with hooks that write its stages out, one
// thread per (walker, bin), every mode its own unit; KEP: heliocentric
// detectors on exact Kepler ellipses.  Test entry point only.
struct ProbeWriter {
  int stage, det, n_modes, n_det;
  int64_t b, k, N;
  double* out;
  __device__ void mode(int j, double amp, double phase, double tau) const {
    if (stage != PES_PROBE_MODE || det != 0) return;
    double* o = out + ((b * n_modes + j) * N + k) * 3;
    o[0] = amp;
    o[1] = phase - floor(phase);
    o[2] = tau;
  }
  __device__ void geom(int j, const double* kn, const double* np, const double* nq, const double* kd,
                       double kR) const {
    if (stage != PES_PROBE_GEOM) return;
    double* o = out + (((b * n_det + det) * n_modes + j) * N + k) * 12;
    for (int t = 0; t < 3; ++t) {
      o[t] = kn[t];
      o[3 + t] = np[t] * np[t] - nq[t] * nq[t];
      o[6 + t] = np[t] * nq[t];
    }
    o[9] = kd[0];
    o[10] = kd[1];
    o[11] = kR;
  }
  __device__ void links(const double* y) const {
    if (stage != PES_PROBE_LINKS) return;
    double* o = out + ((b * n_det + det) * N + k) * 12;
    for (int i = 0; i < 12; ++i) o[i] = y[i];
  }
};

template <bool LS, bool KEP>
__global__ void probe_kernel(ResponseArgs A, int64_t B, int stage) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t N = A.N;
  if (g >= B * N) return;
  const int64_t b = g / N, k = g - b * N;
  const double* __restrict__ wt = A.wtab + b * W_STRIDE;
  ModePlan plan;
  plan.n_units = A.n_modes;
  plan.n_pairs = 0;
  for (int j = 0; j < kMaxModes; ++j) {
    plan.lead[j] = j;
    plan.member[j] = -1;
  }
  // stages beyond a mode's cutoff are not evaluated: amplitude 0, NaN elsewhere
  if (stage == PES_PROBE_MODE)
    for (int j = 0; j < A.n_modes; ++j) {
      double* o = A.out + ((b * A.n_modes + j) * N + k) * 3;
      o[0] = 0.0;
      o[1] = NAN;
      o[2] = NAN;
    }
  if (stage == PES_PROBE_GEOM)
    for (int i = 0; i < A.n_det * A.n_modes * 12; ++i) {
      const int det = i / (A.n_modes * 12), j = (i / 12) % A.n_modes, r = i % 12;
      A.out[(((b * A.n_det + det) * A.n_modes + j) * N + k) * 12 + r] = NAN;
    }
  if (wt[W_VALID] == 0.0) return;
  BinRegs br;
  br.f = A.bins[B_F * N + k];
  br.f13 = A.bins[B_F13 * N + k];
  br.fm13 = A.bins[B_FM13 * N + k];
  br.fm76 = A.bins[B_FM76 * N + k];
  br.lnf = A.bins[B_LNF * N + k];
  for (int det = 0; det < A.n_det; ++det) {
    const double* tb = A.tabs + (int64_t)det * T_NFIELDS * N;
    const DetParams& P = A.dt.p[det];
    const ProbeWriter pw{stage, det, A.n_modes, A.n_det, b, k, N, A.out};
    if (P.kind == 2)
      eval_channels_t<true, LS, 1, double, ValTab, ProbeWriter>(ValTab{wt}, det, plan, P.inv_year, P.inv_ptq, br,
                                                               tb[T_A * N + k], tb[T_ZR * N + k],
                                                               tb[T_ZI * N + k], pw);
    else if constexpr (KEP)
      eval_channels_t<false, LS, 1, double, ValTab, ProbeWriter, true>(
          ValTab{wt}, det, plan, P.inv_year, P.inv_ptq, br, tb[T_A * N + k], tb[T_ZR * N + k], tb[T_ZI * N + k],
          pw, A.wkep + (b * A.n_det + det) * KW_STRIDE, A.kep + det * KV_STRIDE + KV_INVL);
    else
      eval_channels_t<false, LS, 1, double, ValTab, ProbeWriter>(ValTab{wt}, det, plan, P.inv_year, P.inv_ptq, br,
                                                                tb[T_A * N + k], tb[T_ZR * N + k],
                                                                tb[T_ZI * N + k], pw);
  }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_bin_tables(double* bins, double* tabs, int64_t N, double f0, double df, int n_det,
                             const DetTable& dt, hipStream_t s) {
  const int bs = 256;
  hipLaunchKernelGGL(bin_tables_kernel, dim3((unsigned)((N + bs - 1) / bs)), dim3(bs), 0, s, bins, tabs,
                     N, f0, df, n_det, dt);
  return hipGetLastError();
}

hipError_t launch_set_data(const double* d, double* tabs, double* dd_part, double* dd, int64_t N,
                           int n_det, hipStream_t s) {
  const int bs = 256;
  const int nb = (int)((N + bs - 1) / bs);
  hipLaunchKernelGGL(set_data_kernel, dim3(nb), dim3(bs), 0, s, d, tabs, dd_part, N, n_det);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(1024), 0, s, dd_part, nb, dd);
  return hipGetLastError();
}

hipError_t launch_setup_tan(const double* theta, int64_t B, double* wtab, double* wtan, int* ntiles,
                            const SetupArgs& sa, hipStream_t s) {
  const int bs = 64;
  hipLaunchKernelGGL(setup_tan_kernel, dim3((unsigned)((B * kNParams + bs - 1) / bs)), dim3(bs), 0, s, theta,
                     B, wtab, wtan, ntiles, sa);
  return hipGetLastError();
}

hipError_t launch_setup(const double* theta, int64_t B, double* wtab, int* ntiles, const SetupArgs& sa,
                        hipStream_t s) {
  const int bs = 64;
  hipLaunchKernelGGL(setup_kernel, dim3((unsigned)((B + bs - 1) / bs), 1 + sa.n_modes + sa.n_det), dim3(bs), 0, s,
                     theta, B, wtab, ntiles, sa);
  return hipGetLastError();
}

hipError_t launch_plan(const int* ntiles, int B, int wg, int ntmax, bool sorted, int* perm, int* gstart,
                       int* counters, hipStream_t s) {
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(1024), 0, s, ntiles, B, wg, ntmax, sorted ? 1 : 0, perm, gstart,
                     counters);
  return hipGetLastError();
}

template <int BPL, bool LS, bool F32, bool KEP>
static void launch_ll(const LoglikeArgs& a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((loglike_kernel<BPL, LS, F32, KEP>), dim3(grid), dim3(256), 0, s, a.bins, a.tabs, a.wtab,
                     a.ntiles, a.perm, a.gstart, a.counters, a.partial, a);
}

template <bool F32, bool KEP>
static void launch_ll_f(const LoglikeArgs& a, int bpl, bool long_sinc, int grid, hipStream_t s) {
  if (bpl == 2)
    long_sinc ? launch_ll<2, true, F32, KEP>(a, grid, s) : launch_ll<2, false, F32, KEP>(a, grid, s);
  else
    long_sinc ? launch_ll<1, true, F32, KEP>(a, grid, s) : launch_ll<1, false, F32, KEP>(a, grid, s);
}

// Variants: FP64 or FP32, each on the first-order orbit or on exact Kepler orbits.
hipError_t launch_loglike(const LoglikeArgs& a, int bpl, bool long_sinc, bool f32, bool kep, int grid,
                          hipStream_t s) {
  if (f32 && !a.wtab32) return hipErrorInvalidValue;       // the FP32 kernels read the FP32 walker tables
  if (kep && (!a.wkep || !a.kep)) return hipErrorInvalidValue;   // and the Kepler ones the orbit series
  if (kep && f32 && (!a.wkep32 || !a.kep32)) return hipErrorInvalidValue;   // in FP32 their FP32 copies
  if (f32)
    kep ? launch_ll_f<true, true>(a, bpl, long_sinc, grid, s) : launch_ll_f<true, false>(a, bpl, long_sinc, grid, s);
  else if (kep)
    launch_ll_f<false, true>(a, bpl, long_sinc, grid, s);
  else
    launch_ll_f<false, false>(a, bpl, long_sinc, grid, s);
  return hipGetLastError();
}

hipError_t launch_kepler_proj(const double* theta, int64_t B, const double* kep, const SetupArgs& sa,
                              double* wkep, hipStream_t s) {
  if (!kep || !wkep) return hipErrorInvalidValue;
  const int64_t n = B * sa.n_det;
  hipLaunchKernelGGL(kepler_proj_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, theta, B, kep, sa, wkep);
  return hipGetLastError();
}

hipError_t launch_kepler_proj_tan(const double* theta, int64_t B, const double* kep, const SetupArgs& sa,
                                  double* wkept, hipStream_t s) {
  if (!kep || !wkept) return hipErrorInvalidValue;
  const int64_t n = B * sa.n_det * 3;
  hipLaunchKernelGGL(kepler_proj_tan_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, theta, B, kep, sa,
                     wkept);
  return hipGetLastError();
}

hipError_t launch_copy_f32(const double* src, int64_t n, float* dst, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (!src || !dst) return hipErrorInvalidValue;
  hipLaunchKernelGGL(table32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, n, dst);
  return hipGetLastError();
}

hipError_t launch_table32(const double* wtab, int64_t B, float* wtab32, hipStream_t s) {
  return launch_copy_f32(wtab, B * W_STRIDE, wtab32, s);
}

hipError_t launch_finalize(const double* partial, const int* ntiles, const double* wtab, const double* dd,
                           int64_t B, double* logl, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)((B + kFinW - 1) / kFinW)), dim3(kFinW * kFinP), 0, s, partial,
                     ntiles, wtab, dd, B, logl);
  return hipGetLastError();
}

template <bool LS, bool KEP>
static void launch_pr(const ResponseArgs& a, int64_t B, int stage, dim3 grid, hipStream_t s) {
  hipLaunchKernelGGL((probe_kernel<LS, KEP>), grid, dim3(64), 0, s, a, B, stage);
}

hipError_t launch_probe(const ResponseArgs& a, int64_t B, bool long_sinc, bool kep, int stage, hipStream_t s) {
  if (kep && (!a.wkep || !a.kep)) return hipErrorInvalidValue;
  const int64_t n = B * a.N;
  const dim3 grid((unsigned)((n + 63) / 64));
  if (kep)
    long_sinc ? launch_pr<true, true>(a, B, stage, grid, s) : launch_pr<false, true>(a, B, stage, grid, s);
  else
    long_sinc ? launch_pr<true, false>(a, B, stage, grid, s) : launch_pr<false, false>(a, B, stage, grid, s);
  return hipGetLastError();
}

template <bool LS, bool F32, bool KEP>
static void launch_resp(const ResponseArgs& a, dim3 grid, int bs, hipStream_t s) {
  hipLaunchKernelGGL((response_kernel<LS, F32, KEP>), grid, dim3(bs), 0, s, a);
}

hipError_t launch_response(const ResponseArgs& a, int64_t B, bool long_sinc, bool f32, bool kep, hipStream_t s) {
  if (f32 && !a.wtab32) return hipErrorInvalidValue;   // the FP32 kernel reads the FP32 walker tables
  if (kep && (!a.wkep || !a.kep)) return hipErrorInvalidValue;
  if (kep && f32 && (!a.wkep32 || !a.kep32)) return hipErrorInvalidValue;
  const int bs = 256;
  const dim3 grid((unsigned)((a.N + bs - 1) / bs), (unsigned)B);
  if (f32 && kep)
    long_sinc ? launch_resp<true, true, true>(a, grid, bs, s) : launch_resp<false, true, true>(a, grid, bs, s);
  else if (f32)
    long_sinc ? launch_resp<true, true, false>(a, grid, bs, s) : launch_resp<false, true, false>(a, grid, bs, s);
  else if (kep)
    long_sinc ? launch_resp<true, false, true>(a, grid, bs, s) : launch_resp<false, false, true>(a, grid, bs, s);
  else
    long_sinc ? launch_resp<true, false, false>(a, grid, bs, s) : launch_resp<false, false, false>(a, grid, bs, s);
  return hipGetLastError();
}

template <bool F32, bool KEP>
static int blocks_per_cu(int bpl, bool long_sinc) {
  int nb = 0;
  hipError_t e;
  if (bpl == 2)
    e = long_sinc ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, loglike_kernel<2, true, F32, KEP>, 256, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, loglike_kernel<2, false, F32, KEP>, 256, 0);
  else
    e = long_sinc ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, loglike_kernel<1, true, F32, KEP>, 256, 0)
                  : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, loglike_kernel<1, false, F32, KEP>, 256, 0);
  return e == hipSuccess ? nb : 1;
}

int loglike_blocks_per_cu(int bpl, bool long_sinc, bool f32, bool kep) {
  if (f32) return kep ? blocks_per_cu<true, true>(bpl, long_sinc) : blocks_per_cu<true, false>(bpl, long_sinc);
  return kep ? blocks_per_cu<false, true>(bpl, long_sinc) : blocks_per_cu<false, false>(bpl, long_sinc);
}

}  // namespace pes
