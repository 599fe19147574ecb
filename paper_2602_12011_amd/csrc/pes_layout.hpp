// Memory layout shared by the host runtime and the kernels of libpes.
#pragma once
#include <stdint.h>

namespace pes {

constexpr int kMaxModes = 5;
constexpr int kMaxDet = 3;
constexpr int kNParams = 11;

// ---- per-walker constant table (doubles), built by the setup kernel.
// Every quantity the per-(walker, bin) evaluation needs that depends only on
// theta is precomputed here, so the hot loop reads it through the scalar
// cache (the walker index is uniform across a wavefront).
enum : int {
  W_VALID = 0,   // 1.0 for a physical sample, 0.0 otherwise
  W_TC = 1,      // t_c [s]
  W_FMAX = 2,    // highest mode cutoff [Hz]
  W_MODE0 = 4,
  W_MODE_STRIDE = 26,
  W_DET0 = W_MODE0 + kMaxModes * W_MODE_STRIDE,  // 134
  W_DET_STRIDE = 44,
  W_ROT0 = W_DET0 + kMaxDet * W_DET_STRIDE,      // 266
  W_STRIDE = 288  // >= W_ROT0 + kMaxModes * 4 (286), multiple of 8
};

// Modes that share m share v, t_f, the orbit, the projections, the arm phases
// and the sinc values; their phases differ by the constant C0_j - C0_lead, a
// whole number of quarter cycles (the constant phase of each mode is
// -(m/2) phi_c - pi/4 - arg of its harmonic factor, a multiple of pi/2).  For
// mode j, with rot_j = e^{-2 pi i (C0_j - C0_lead)} exactly in {1, i, -1, -i}
// and lead the first mode of the context with the same m:
//   W_ROT0 + 4 j + (0, 1, 2, 3) = (KP Re rot, KP Im rot, KC Re rot, KC Im rot).
enum : int { R_KPR = 0, R_KPI, R_KCR, R_KCI, R_STRIDE };

// Evaluation units of a context.  The first n_pairs units pair a mode (lead)
// with the next mode of the same m (member), added as a complex amplitude on
// the lead's phase factor; the remaining units hold one mode each.
struct ModePlan {
  int n_units, n_pairs;
  int lead[kMaxModes];
  int member[kMaxModes];
};

// Per mode: v = CM f^{1/3}, 1/v = CMI f^{-1/3}, ln v = LNCM + ln(f)/3.
// Phase in cycles (without the f t_c term):
//   C0 + A0 w^5 + A2 w^3 + A3 w^2 + A4 w + B5 ln v + v (A6 + B6 ln v + A7 v),  w = 1/v
// t_f - t_c [s]:
//   T0 w^8 + T2 w^6 + T3 w^5 + T4 w^4 + T5 w^3 + (T6 + T6L ln v) w^2 + T7 w
// Amplitude: f^{-7/6} (AM0 + AM1 v + AM2 v^2) x taper(f * FCI); polarization
// h_+ = KP amp e^{-i phase}, h_x = i (KC / 2) amp e^{-i phase} (KC holds 2 K_x).
enum : int {
  M_CM = 0, M_CMI, M_LNCM, M_C0, M_A0, M_A2, M_A3, M_A4, M_B5, M_A6, M_B6, M_A7,
  M_T0, M_T2, M_T3, M_T4, M_T5, M_T6, M_T6L, M_T7, M_AM0, M_AM1, M_AM2, M_KP, M_KC, M_FCI
};

// Per detector.  Orbit phases in cycles: alpha = AO + (t_f - t_c)/yr (guiding
// centre), and for the geocentric orbit phi = PO + (t_f - t_c)/P.  Each
// projection below is linear in u = (a, b, cos alpha, sin alpha, 1), where
// (a, b) = (cos 2 alpha, sin 2 alpha) for heliocentric and (cos phi, sin phi)
// for geocentric orbits: 5 coefficients each.
//   KN[t]: k . n_t for arms t = 0, 1 (n_t = (x_{t+2} - x_{t+1})/L; n_2 = -n_0 - n_1)
//   NP[t], NQ[t]: p . n_t, q . n_t (polarization axes)
//   KD[s]: k . (x_s - centre) [light-s] for spacecraft s = 0, 1 (s = 2: minus the sum)
//   KR: k . centre = KR0 cos alpha + KR1 sin alpha [light-s]
enum : int {
  D_AO = 0, D_PO = 1, D_KN = 2, D_NP = 12, D_NQ = 22, D_KD = 32, D_KR = 42
};

// ---- exact Keplerian heliocentric orbits (detector option).  Every
// orbit-dependent vector is a periodic function of the revolution phase alpha,
// kept as a Fourier series to harmonic kKepH (the Kepler ellipses' series
// converge roughly as e^k; e ~ 5e-3; the inverse arm lengths, truncated here,
// keep a relative 4e-11, the separations 3e-14 s): term 0 the constant,
// 2k - 1 the cos(k alpha) and 2k the sin(k alpha) coefficient.
constexpr int kKepH = 6;
constexpr int kKepT = 2 * kKepH + 1;   // 13 terms
// Per detector (host-computed, walker-independent), light-seconds: the arm
// vectors Delta_0 = x_2 - x_1, Delta_1 = x_0 - x_2, the offsets x_0 - c,
// x_1 - c from the centroid c, and c, each [3 components][kKepT]; then the
// inverse arm lengths 1/|Delta_t| (Delta_2 = x_1 - x_0) [3][kKepT].
enum : int {
  KV_D0 = 0, KV_D1 = 3 * kKepT, KV_X0 = 6 * kKepT, KV_X1 = 9 * kKepT, KV_C = 12 * kKepT,
  KV_INVL = 15 * kKepT, KV_STRIDE = 240   // >= 18 kKepT (234)
};
// Per walker and detector (setup): the series of the projections
//   k.Delta_0, k.Delta_1, p.Delta_0, p.Delta_1, q.Delta_0, q.Delta_1,
//   k.(x_0 - c), k.(x_1 - c), k.c   (9 x kKepT, what the response evaluates),
//   p.(x_0 - c), p.(x_1 - c), q.(x_0 - c), q.(x_1 - c), p.c, q.c
//   (6 x kKepT, the reverse sweep's sky contraction)
enum : int {
  KW_KD0 = 0, KW_KD1 = kKepT, KW_PD0 = 2 * kKepT, KW_PD1 = 3 * kKepT, KW_QD0 = 4 * kKepT,
  KW_QD1 = 5 * kKepT, KW_KX0 = 6 * kKepT, KW_KX1 = 7 * kKepT, KW_KC = 8 * kKepT,
  KW_PX0 = 9 * kKepT, KW_PX1 = 10 * kKepT, KW_QX0 = 11 * kKepT, KW_QX1 = 12 * kKepT, KW_PC = 13 * kKepT,
  KW_QC = 14 * kKepT, KW_STRIDE = 200   // >= 15 kKepT (195)
};

// ---- per-bin tables (structure of arrays, n_bins doubles per field).
enum : int { B_F = 0, B_F13, B_FM13, B_FM76, B_LNF, B_NFIELDS };
// Per detector and bin: delay factor z = e^{-2 pi i f L}; the TDI- and
// response-factor-folded, noise-weighted data D_c = w_c n_c conj(G) d_c;
// the weights W_A (W_E = W_A / 3) and W_T of |combination|^2; a = pi f L;
// the common factor G = F_TDI(z) (-i pi f L) e^{-i pi f L} of every channel;
// the raw weights w_c = 4 df / S_c.
enum : int {
  T_ZR = 0, T_ZI, T_DAR, T_DAI, T_DER, T_DEI, T_DTR, T_DTI, T_WA, T_WT, T_A,
  T_GR, T_GI, T_WAE, T_WTT, T_NFIELDS
};

struct DetParams {
  int kind;          // 0 LISA, 1 Taiji: heliocentric; 2 TianQin: geocentric
  int tdi_gen;       // 15 or 20
  double L;          // arm [s]
  double inv_year;   // 1/yr [1/s]
  double inv_ptq;    // 1/P for the geocentric orbit
  double phase0_cyc; // revolution phase of the centre [cycles]
  // geometry: spacecraft offsets from the centre, Delta_s = sum_i G[s][c][i] u_i
  double G[3][3][5];
  double AUc;        // AU / c [s]
  double oms2, acc2; // ASD^2
};

struct ModeSpec {
  int l, m;
};

}  // namespace pes
