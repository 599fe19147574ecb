// Reverse-mode (adjoint) gradient of the per-bin log-likelihood term,
// written by hand (Sec. 2.3 differentiates the response in reverse mode).
//
// For one (walker, bin, detector) the term is
//   l = sum_c D_c C_c - 1/2 sum_c W_c C_c^2
// over the six real channel components C = (A'', E'', T'') of the folded
// tables, so dl/dC_c = D_c - W_c C_c (the weighted residual).  That seed goes
// back through A/E/T and the TDI combinations to the six complex links
// (adj_links), then, for every active mode, through the link transfer
// functions, the projections, the orbit at t_f, amplitude, phase and t_f to
// the entries of the walker table (adj_unit).  Each mode entry's adjoint is
// contracted at once with its theta-derivatives (the tangent table of the
// setup), so only a few accumulators live across bins.  The sky angles enter
// only through the unit vectors k, p, q, whose projections onto the arms are
// the detector entries; their adjoints collapse into three sums per lane
// (adj_unit), contracted with the derivatives of the sky basis once per block.
// The forward values of a unit are recomputed from the table, nothing is
// stored per bin.
#pragma once
#include "pes_eval.hpp"
#include "pes_launch.hpp"

namespace pes {

// A value the compiler must treat as unknown (an empty asm that claims to
// modify it): recomputations from it are not merged with earlier ones.
__device__ __forceinline__ double opaque(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

// g[J...] += cbar * d(entry)/d(theta_J) for the parameters J the entry depends
// on (the setup makes every other derivative exactly zero).  tan_row holds
// those derivatives in the order of J (the compact tangent layout below).
template <int... J>
struct Deps {
  __device__ __forceinline__ static void add(double* g, double cbar, const double* tan_row) {
    int i = 0;
    ((g[J] = fma(cbar, tan_row[i++], g[J])), ...);
  }
};
// theta = (M, q, chi1, chi2, D_L, iota, phi_c, lambda, beta, psi, t_c)
using DepM = Deps<0>;
using DepIota = Deps<5>;
using DepSky = Deps<7, 8>;
using DepTc = Deps<10>;

// Compact tangent layout: per table entry only the derivatives with respect
// to the parameters in its mask (bit k: theta_k), in increasing k; entries
// ordered t_c, then modes 0..4 (26 fields each), then detectors 0..2 (44
// fields each), then the rotated polarization factors of modes 0..4 (4 each,
// iota only).  The masks are the parameter lists the reverse sweep uses.
constexpr unsigned kBitM = 1u << 0, kBitQ = 1u << 1, kBitChi = (1u << 2) | (1u << 3), kBitD = 1u << 4,
                   kBitIota = 1u << 5, kBitPhi = 1u << 6, kBitSky = (1u << 7) | (1u << 8), kBitPsi = 1u << 9,
                   kBitTc = 1u << 10;
__host__ __device__ constexpr unsigned mode_mask(int f) {
  switch (f) {
    case M_CM: case M_CMI: case M_LNCM: case M_FCI: return kBitM;
    case M_C0: return kBitQ | kBitPhi;
    case M_A3: case M_A4: return kBitQ | kBitChi;
    case M_A0: case M_A2: case M_B5: case M_A6: case M_B6: case M_A7: return kBitQ;
    case M_T3: case M_T4: return kBitM | kBitQ | kBitChi;
    case M_T0: case M_T2: case M_T5: case M_T6: case M_T6L: case M_T7: return kBitM | kBitQ;
    case M_AM0: case M_AM1: case M_AM2: return kBitM | kBitQ | kBitD;
    default: return kBitIota;   // M_KP, M_KC
  }
}
__host__ __device__ constexpr unsigned det_mask(int f) {
  return f < D_KN ? kBitTc : (f >= D_NP && f < D_KD) ? (kBitSky | kBitPsi) : kBitSky;
}
// Slot offsets of the fields within a mode / detector block, evaluated at
// compile time (tm/td below index them with constants).
struct TanLayout {
  int mode[W_MODE_STRIDE + 1];
  int det[W_DET_STRIDE + 1];
  constexpr TanLayout() : mode(), det() {
    for (int f = 0; f < W_MODE_STRIDE; ++f) mode[f + 1] = mode[f] + __builtin_popcount(mode_mask(f));
    for (int f = 0; f < W_DET_STRIDE; ++f) det[f + 1] = det[f] + __builtin_popcount(det_mask(f));
  }
};
constexpr TanLayout kTanLayout{};
constexpr int kModeSlots = kTanLayout.mode[W_MODE_STRIDE];   // 49
constexpr int kDetSlots = kTanLayout.det[W_DET_STRIDE];      // 106
constexpr int kTanMode0 = 1;
constexpr int kTanDet0 = kTanMode0 + kMaxModes * kModeSlots;
constexpr int kTanRot0 = kTanDet0 + kMaxDet * kDetSlots;
constexpr int kTanSlots = kTanRot0 + kMaxModes * R_STRIDE;
static_assert(kModeSlots == 49 && kDetSlots == 106, "compact tangent layout");
static_assert(kTanSlots == kTanCompactSlots, "compact tangent table size");
template <int F> struct ModeOff { static constexpr int value = kTanLayout.mode[F]; };
template <int F> struct DetOff { static constexpr int value = kTanLayout.det[F]; };

// Copies the full tangent table [W_STRIDE][11] of one walker into the compact
// layout, entries split over the n threads of a block.
__device__ inline void compact_tangents(const double* __restrict__ full, double* __restrict__ out, int tid,
                                        int n) {
  for (int e = tid; e < 1 + kMaxModes * W_MODE_STRIDE + kMaxDet * W_DET_STRIDE + kMaxModes * R_STRIDE; e += n) {
    int entry, slot;
    unsigned mask;
    if (e == 0) {
      entry = W_TC;
      slot = 0;
      mask = kBitTc;
    } else if (e < 1 + kMaxModes * W_MODE_STRIDE) {
      const int j = (e - 1) / W_MODE_STRIDE, f = (e - 1) % W_MODE_STRIDE;
      entry = W_MODE0 + j * W_MODE_STRIDE + f;
      mask = mode_mask(f);
      slot = kTanMode0 + j * kModeSlots;
      for (int q = 0; q < f; ++q) slot += __builtin_popcount(mode_mask(q));
    } else if (e >= 1 + kMaxModes * W_MODE_STRIDE + kMaxDet * W_DET_STRIDE) {
      const int r = e - 1 - kMaxModes * W_MODE_STRIDE - kMaxDet * W_DET_STRIDE;
      entry = W_ROT0 + r;
      mask = kBitIota;
      slot = kTanRot0 + r;
    } else {
      const int r = e - 1 - kMaxModes * W_MODE_STRIDE;
      const int d = r / W_DET_STRIDE, f = r % W_DET_STRIDE;
      entry = W_DET0 + d * W_DET_STRIDE + f;
      mask = det_mask(f);
      slot = kTanDet0 + d * kDetSlots;
      for (int q = 0; q < f; ++q) slot += __builtin_popcount(det_mask(q));
    }
    for (int k = 0; k < kNParams; ++k)
      if (mask & (1u << k)) out[slot++] = full[entry * kNParams + k];
  }
}

// Link adjoints yb[arm][Fr, Fi, Br, Bi] from the channel values c and the
// per-bin data D and weights (wA, wT).  Arm 0 carries y32 (F) / y23 (B),
// arm 1 y13 / y31, arm 2 y21 / y12 (as in eval_channels_t).
__device__ __forceinline__ void adj_links(const Chan& c, const double (&D)[6], double wA, double wT,
                                          double zr, double zi, double (&yb)[3][4]) {
  const double Ar = fma(-wA, c.ar, D[0]), Ai = fma(-wA, c.ai, D[1]);
  const double wE = wA * (1.0 / 3.0);
  const double Er = fma(-wE, c.er, D[2]), Ei = fma(-wE, c.ei, D[3]);
  const double Tr = fma(-wT, c.tr, D[4]), Ti = fma(-wT, c.ti, D[5]);
  // A'' = Z - X, E'' = X - 2Y + Z, T'' = X + Y + Z
  const double Xr = (Er - Ar) + Tr, Xi = (Ei - Ai) + Ti;
  const double Yr = fma(-2.0, Er, Tr), Yi = fma(-2.0, Ei, Ti);
  const double Zr = (Ar + Er) + Tr, Zi = (Ai + Ei) + Ti;
  // u = conj(z) * (adjoint of a z-multiplied difference)
  const double uXr = fma(zr, Xr, zi * Xi), uXi = fma(zr, Xi, -(zi * Xr));
  const double uYr = fma(zr, Yr, zi * Yi), uYi = fma(zr, Yi, -(zi * Yr));
  const double uZr = fma(zr, Zr, zi * Zi), uZi = fma(zr, Zi, -(zi * Zr));
  // X = y13 - y12 + z (y31 - y21); Y = y21 - y23 + z (y12 - y32);
  // Z = y32 - y31 + z (y23 - y13)
  yb[0][0] = Zr - uYr;  yb[0][1] = Zi - uYi;   // y32
  yb[0][2] = uZr - Yr;  yb[0][3] = uZi - Yi;   // y23
  yb[1][0] = Xr - uZr;  yb[1][1] = Xi - uZi;   // y13
  yb[1][2] = uXr - Zr;  yb[1][3] = uXi - Zi;   // y31
  yb[2][0] = Yr - uXr;  yb[2][1] = Yi - uXi;   // y21
  yb[2][2] = uYr - Xr;  yb[2][3] = uYi - Xi;   // y12
}

// Adjoint of one arm's contribution y_F += sinc(a(1-kn)) G, y_B += sinc(a(1+kn)) G
// with G = W e, W = pp (aP E) + i pc (2 aC E), pp = np^2 - nq^2, pc = np nq.
// Accumulates the adjoints of aP E and 2 aC E and returns those of the arm's
// e = (c, s), kn, np, nq.
template <bool LS>
__device__ __forceinline__ void adj_arm(const double* yb, double a, double pEr, double pEi, double cEr,
                                        double cEi, double c, double s, double np, double nq, double kn,
                                        double& pEbr, double& pEbi, double& cEbr, double& cEbi, double& cb,
                                        double& sb, double& knb, double& npb, double& nqb) {
  const double pp = fma(np, np, -(nq * nq)), pc = np * nq;
  const double Wr = fma(pp, pEr, -(pc * cEi)), Wi = fma(pp, pEi, pc * cEr);
  const double Gr = fma(Wr, c, -(Wi * s)), Gi = fma(Wr, s, Wi * c);
  const double bf = fma(-a, kn, a), bb = fma(a, kn, a);
  double sf, dsf, sbk, dsb;
  if (LS) {
    horner_d<1>(kSincLong, bf * bf, sf, dsf);
    horner_d<1>(kSincLong, bb * bb, sbk, dsb);
  } else {
    horner_d<1>(kSincShort, bf * bf, sf, dsf);
    horner_d<1>(kSincShort, bb * bb, sbk, dsb);
  }
  const double sfb = fma(yb[0], Gr, yb[1] * Gi), sbb = fma(yb[2], Gr, yb[3] * Gi);
  const double Gbr = fma(sf, yb[0], sbk * yb[2]), Gbi = fma(sf, yb[1], sbk * yb[3]);
  // d sinc(b)/db = 2 b P'(b^2)
  knb = 2.0 * a * fma(sbb * bb, dsb, -(sfb * bf * dsf));
  // G = W e
  const double Wbr = fma(Gbr, c, Gbi * s), Wbi = fma(Gbi, c, -(Gbr * s));
  cb = fma(Gbr, Wr, Gbi * Wi);
  sb = fma(Gbi, Wr, -(Gbr * Wi));
  // W = pp (pEr, pEi) + pc (-cEi, cEr)
  const double ppb = fma(Wbr, pEr, Wbi * pEi), pcb = fma(Wbi, cEr, -(Wbr * cEi));
  pEbr = fma(Wbr, pp, pEbr);
  pEbi = fma(Wbi, pp, pEbi);
  cEbr = fma(Wbi, pc, cEbr);
  cEbi = fma(-Wbr, pc, cEbi);
  npb = fma(2.0 * np, ppb, nq * pcb);
  nqb = fma(-2.0 * nq, ppb, np * pcb);
}

// Harmonics cos k alpha, sin k alpha (k = 0..kKepH) of the orbit phase from
// its cosine and sine (Chebyshev recurrence, as the response evaluates them).
__device__ __forceinline__ void kep_harmonics(double ca, double sa, double (&hc)[kKepH + 1],
                                              double (&hs)[kKepH + 1]) {
  hc[0] = 1.0;
  hs[0] = 0.0;
  hc[1] = ca;
  hs[1] = sa;
  const double c2a = 2.0 * ca;
#pragma unroll
  for (int k = 2; k <= kKepH; ++k) {
    hc[k] = fma(c2a, hc[k - 1], -hc[k - 2]);
    hs[k] = fma(c2a, hs[k - 1], -hs[k - 2]);
  }
}
__device__ __forceinline__ double kep_series(const double* __restrict__ cg, const double (&hc)[kKepH + 1],
                                             const double (&hs)[kKepH + 1]) {
  cdouble* c = as_const(cg);
  double r = c[0];
#pragma unroll
  for (int k = 1; k <= kKepH; ++k) r = fma(c[2 * k - 1], hc[k], fma(c[2 * k], hs[k], r));
  return r;
}

// Adjoint of the unit of mode j (and, when PAIR, of mode jm riding on it, as
// in eval_channels_t) of (walker, bin, detector) given the link adjoints yb
// (12 values: arm-major Fr, Fi, Br, Bi); accumulates d l / d theta into
// g[0..10] and the three sky sums into g[11..13] (see the sky part below).
// wt: the walker's table; tn: its tangents in the compact layout; ftc = f t_c
// mod 1; L3 = L / 3 of the detector.  KEP: a heliocentric detector on exact
// Kepler ellipses, kw its projected orbit series for this walker, kinv its
// inverse-arm-length series (the geometry as the response evaluates it).
template <bool GEO, bool LS, bool PAIR, bool KEP = false>
__device__ __forceinline__ void adj_unit(const double* __restrict__ wt, const double* __restrict__ tn, int det,
                                         int j, int jm, double inv_year, double inv_ptq, double L3,
                                         const BinRegs& b, double a, double ftc, const double* yb, double* g,
                                         const double* __restrict__ kw = nullptr,
                                         const double* __restrict__ kinv = nullptr) {
  int M0 = W_MODE0 + opaque_u(j) * W_MODE_STRIDE;
  int D0 = W_DET0 + opaque_u(det) * W_DET_STRIDE;
  int N0 = W_MODE0 + opaque_u(jm) * W_MODE_STRIDE, R0 = W_ROT0 + R_STRIDE * opaque_u(jm);
#define wm(i) wt[M0 + (i)]
#define wd(i) wt[D0 + (i)]
#define wn(i) wt[N0 + (i)]
#define wr(i) wt[R0 + (i)]
#define tm(i) (tn + kTanMode0 + j * kModeSlots + ModeOff<(i)>::value)
#define tnm(i) (tn + kTanMode0 + jm * kModeSlots + ModeOff<(i)>::value)
#define tr(i) (tn + kTanRot0 + R_STRIDE * jm + (i))
#define td(i) (tn + kTanDet0 + det * kDetSlots + DetOff<(i)>::value)
  const double x = b.f * wm(M_FCI);
  if (!(x < 1.0)) return;
  // ---- forward values (the same arithmetic as eval_channels_t).  The
  // waveform's intermediate powers are not kept through the geometry part:
  // they are recomputed for the waveform reverse below, which keeps the live
  // register set of this function small.
  double phase, tau, amp0, amn0 = 0.0;
  {
    const double v = wm(M_CM) * b.f13;
    const double w = wm(M_CMI) * b.fm13;
    const double lnv = b.lnf * (1.0 / 3.0) + wm(M_LNCM);
    const double w2 = w * w, w3 = w2 * w, w4 = w2 * w2, w5 = w4 * w, w6 = w4 * w2, w8 = w4 * w4;
    const double v2 = v * v, lv = lnv * v, lw2 = lnv * w2;
    double ph = wm(M_A4) * w;
    ph = fma(wm(M_A3), w2, ph);
    ph = fma(wm(M_A2), w3, ph);
    ph = fma(wm(M_A0), w5, ph);
    ph = fma(wm(M_B5), lnv, ph);
    ph = fma(wm(M_A6), v, ph);
    ph = fma(wm(M_B6), lv, ph);
    ph = fma(wm(M_A7), v2, ph);
    phase = ftc + (ph + wm(M_C0));
    tau = wm(M_T7) * w;
    tau = fma(wm(M_T6), w2, tau);
    tau = fma(wm(M_T6L), lw2, tau);
    tau = fma(wm(M_T5), w3, tau);
    tau = fma(wm(M_T4), w4, tau);
    tau = fma(wm(M_T3), w5, tau);
    tau = fma(wm(M_T2), w6, tau);
    tau = fma(wm(M_T0), w8, tau);
    amp0 = (fma(wm(M_AM2), v2, wm(M_AM1) * v) + wm(M_AM0)) * b.fm76;
    if (PAIR) amn0 = (fma(wn(M_AM2), v2, wn(M_AM1) * v) + wn(M_AM0)) * b.fm76;
  }
  double tap = 1.0, dtap = 0.0;   // taper and its derivative in x
  if (x > 0.9) {
    const double u = (x - 0.9) * 10.0;
    tap = fma(-(u * u * u), fma(u, fma(6.0, u, -15.0), 10.0), 1.0);
    const double um = u - 1.0;
    dtap = -300.0 * (u * u) * (um * um);
  }
  const double amp = amp0 * tap;
  double aP = amp * wm(M_KP), aC2 = amp * wm(M_KC);   // the table holds 2 K_x
  double aPi = 0.0, aCi = 0.0, amn = 0.0;
  if (PAIR) {
    amn = amn0 * tap;
    aP = fma(amn, wr(R_KPR), aP);
    aPi = amn * wr(R_KPI);
    aC2 = fma(amn, wr(R_KCR), aC2);
    aCi = amn * wr(R_KCI);
  }
  double sa, ca, ua = 0.0, ub = 0.0;
  sincos_cycles(tau * inv_year + wd(D_AO), sa, ca);
  double kn0, kn1, kn2, np0, np1, np2, nq0, nq1, nq2, kd0, kd1, kR;
  double KD0 = 0.0, KD1 = 0.0, PD0 = 0.0, PD1 = 0.0, QD0 = 0.0, QD1 = 0.0, iL0 = 0.0, iL1 = 0.0, iL2 = 0.0;
  if constexpr (KEP) {
    // separations Delta_t projected and over their lengths; offsets from the
    // centroid and the centroid projected on k
    double hc[kKepH + 1], hs[kKepH + 1];
    kep_harmonics(ca, sa, hc, hs);
    iL0 = kep_series(kinv, hc, hs);
    iL1 = kep_series(kinv + kKepT, hc, hs);
    iL2 = kep_series(kinv + 2 * kKepT, hc, hs);
    KD0 = kep_series(kw + KW_KD0, hc, hs);
    KD1 = kep_series(kw + KW_KD1, hc, hs);
    PD0 = kep_series(kw + KW_PD0, hc, hs);
    PD1 = kep_series(kw + KW_PD1, hc, hs);
    QD0 = kep_series(kw + KW_QD0, hc, hs);
    QD1 = kep_series(kw + KW_QD1, hc, hs);
    kn0 = KD0 * iL0;
    kn1 = KD1 * iL1;
    kn2 = -(KD0 + KD1) * iL2;
    np0 = PD0 * iL0;
    np1 = PD1 * iL1;
    np2 = -(PD0 + PD1) * iL2;
    nq0 = QD0 * iL0;
    nq1 = QD1 * iL1;
    nq2 = -(QD0 + QD1) * iL2;
    kd0 = kep_series(kw + KW_KX0, hc, hs);
    kd1 = kep_series(kw + KW_KX1, hc, hs);
    kR = kep_series(kw + KW_KC, hc, hs);
  } else {
    if (GEO) {
      sincos_cycles(tau * inv_ptq + wd(D_PO), ub, ua);
    } else {
      ua = fma(-2.0 * sa, sa, 1.0);
      ub = 2.0 * sa * ca;
    }
#define PES_LIN(off) (fma(wd((off) + 3), sa, fma(wd((off) + 2), ca, fma(wd((off) + 1), ub, wd((off)) * ua))) + wd((off) + 4))
    kn0 = PES_LIN(D_KN);
    kn1 = PES_LIN(D_KN + 5);
    np0 = PES_LIN(D_NP);
    np1 = PES_LIN(D_NP + 5);
    nq0 = PES_LIN(D_NQ);
    nq1 = PES_LIN(D_NQ + 5);
    kd0 = PES_LIN(D_KD);
    kd1 = PES_LIN(D_KD + 5);
#undef PES_LIN
    kn2 = -(kn0 + kn1);
    np2 = -(np0 + np1);
    nq2 = -(nq0 + nq1);
    kR = fma(wd(D_KR), ca, wd(D_KR + 1) * sa);
  }
  double sp, cp;
  sincos_cycles(fma(b.f, kR, phase), sp, cp);
  double pEr, pEi, cEr, cEi;
  if (PAIR) {
    pEr = fma(aP, cp, aPi * sp);
    pEi = fma(aPi, cp, -(aP * sp));
    cEr = fma(aC2, cp, aCi * sp);
    cEi = fma(aCi, cp, -(aC2 * sp));
  } else {
    pEr = aP * cp;
    pEi = -(aP * sp);
    cEr = aC2 * cp;
    cEi = -(aC2 * sp);
  }
  double s0, c0, s1, c1;
  const double pi_f = kPi * b.f;
  if (LS) {
    sincos_cycles(0.5 * b.f * kd0, s0, c0);
    sincos_cycles(0.5 * b.f * kd1, s1, c1);
  } else {
    sincos_small(pi_f * kd0, s0, c0);
    sincos_small(pi_f * kd1, s1, c1);
  }
  const double c2 = fma(c0, c1, -(s0 * s1)), s2 = -fma(s0, c1, c0 * s1);

  // table entries are loaded again below (see opaque_u)
  det = opaque_u(det);
  j = opaque_u(j);
  jm = opaque_u(jm);
  M0 = W_MODE0 + j * W_MODE_STRIDE;
  N0 = W_MODE0 + jm * W_MODE_STRIDE;
  R0 = W_ROT0 + R_STRIDE * jm;
  D0 = W_DET0 + det * W_DET_STRIDE;
  // ---- reverse: arms
  double pEbr = 0.0, pEbi = 0.0, cEbr = 0.0, cEbi = 0.0;
  double cb0, sb0, knb0, npb0, nqb0, cb1, sb1, knb1, npb1, nqb1, cb2, sb2, knb2, npb2, nqb2;
  adj_arm<LS>(yb, a, pEr, pEi, cEr, cEi, c0, s0, np0, nq0, kn0, pEbr, pEbi, cEbr, cEbi, cb0, sb0, knb0, npb0, nqb0);
  adj_arm<LS>(yb + 4, a, pEr, pEi, cEr, cEi, c1, s1, np1, nq1, kn1, pEbr, pEbi, cEbr, cEbi, cb1, sb1, knb1, npb1, nqb1);
  adj_arm<LS>(yb + 8, a, pEr, pEi, cEr, cEi, c2, s2, np2, nq2, kn2, pEbr, pEbi, cEbr, cEbi, cb2, sb2, knb2, npb2, nqb2);
  // (aP + i aPi) E, (2 aC + i aCi) E with E = (cp, -sp)
  const double aPb = fma(pEbr, cp, -(pEbi * sp));
  const double aCb = fma(cEbr, cp, -(cEbi * sp));
  double cpb = fma(pEbr, aP, cEbr * aC2);
  double spb = -fma(pEbi, aP, cEbi * aC2);
  double aPib = 0.0, aCib = 0.0;
  if (PAIR) {
    aPib = fma(pEbr, sp, pEbi * cp);
    aCib = fma(cEbr, sp, cEbi * cp);
    cpb = fma(pEbi, aPi, fma(cEbi, aCi, cpb));
    spb = fma(pEbr, aPi, fma(cEbr, aCi, spb));
  }
  // the third arm follows from the other two (its phase always; its
  // projections on the rigid triangle)
  if (!KEP) {
    knb0 -= knb2;
    knb1 -= knb2;
    npb0 -= npb2;
    npb1 -= npb2;
    nqb0 -= nqb2;
    nqb1 -= nqb2;
  }
  cb0 = fma(cb2, c1, fma(-sb2, s1, cb0));
  sb0 = fma(-cb2, s1, fma(-sb2, c1, sb0));
  cb1 = fma(cb2, c0, fma(-sb2, s0, cb1));
  sb1 = fma(-cb2, s0, fma(-sb2, c0, sb1));
  // arm phases pi f kd_t (radians)
  const double kdb0 = pi_f * fma(sb0, c0, -(cb0 * s0));
  const double kdb1 = pi_f * fma(sb1, c1, -(cb1 * s1));
  // common phase (cycles): (sp, cp) = (sin, cos)(2 pi Phi), Phi = f kR + phase
  const double Phib = kTwoPi * fma(spb, cp, -(cpb * sp));
  const double kRb = b.f * Phib;
  double taub = 0.0, alphab;
  if constexpr (KEP) {
    // ---- exact Kepler orbits: adjoints of the twelve series values
    const double KDb0 = fma(knb0, iL0, -(knb2 * iL2)), KDb1 = fma(knb1, iL1, -(knb2 * iL2));
    const double PDb0 = fma(npb0, iL0, -(npb2 * iL2)), PDb1 = fma(npb1, iL1, -(npb2 * iL2));
    const double QDb0 = fma(nqb0, iL0, -(nqb2 * iL2)), QDb1 = fma(nqb1, iL1, -(nqb2 * iL2));
    const double iLb0 = fma(knb0, KD0, fma(npb0, PD0, nqb0 * QD0));
    const double iLb1 = fma(knb1, KD1, fma(npb1, PD1, nqb1 * QD1));
    const double iLb2 = -fma(knb2, KD0 + KD1, fma(npb2, PD0 + PD1, nqb2 * (QD0 + QD1)));
    double hc[kKepH + 1], hs[kKepH + 1];
    kep_harmonics(ca, sa, hc, hs);
    // sky part: every projected vector V (Delta_t, x_t - c, c) is
    // (k.V) k + (p.V) p + (q.V) q, so with the triad identities of the
    // first-order branch below the sky adjoints reduce to the same three sums
    const double PX0 = kep_series(kw + KW_PX0, hc, hs), PX1 = kep_series(kw + KW_PX1, hc, hs);
    const double QX0 = kep_series(kw + KW_QX0, hc, hs), QX1 = kep_series(kw + KW_QX1, hc, hs);
    const double PC = kep_series(kw + KW_PC, hc, hs), QC = kep_series(kw + KW_QC, hc, hs);
    g[kNParams] = fma(KDb0, PD0, fma(-PDb0, KD0, fma(KDb1, PD1, fma(-PDb1, KD1,
                  fma(kdb0, PX0, fma(kdb1, PX1, fma(kRb, PC, g[kNParams])))))));
    g[kNParams + 1] = fma(KDb0, QD0, fma(-QDb0, KD0, fma(KDb1, QD1, fma(-QDb1, KD1,
                      fma(kdb0, QX0, fma(kdb1, QX1, fma(kRb, QC, g[kNParams + 1])))))));
    g[kNParams + 2] = fma(PDb0, QD0, fma(-QDb0, PD0, fma(PDb1, QD1, fma(-QDb1, PD1, g[kNParams + 2]))));
    // time part: d/d alpha of the series, c_{2k-1} cos k alpha + c_{2k} sin k alpha
    // -> k (c_{2k} cos k alpha - c_{2k-1} sin k alpha), summed with the adjoints
    // d/d alpha of one series at this alpha
    auto dser = [&](const double* __restrict__ cg) __attribute__((always_inline)) {
      cdouble* c = as_const(cg);
      double r = c[2] * hc[1] - c[1] * hs[1];
#pragma unroll
      for (int k = 2; k <= kKepH; ++k) r = fma((double)k, fma(c[2 * k], hc[k], -(c[2 * k - 1] * hs[k])), r);
      return r;
    };
    double dal = iLb0 * dser(kinv);
    dal = fma(iLb1, dser(kinv + kKepT), dal);
    dal = fma(iLb2, dser(kinv + 2 * kKepT), dal);
    dal = fma(KDb0, dser(kw + KW_KD0), dal);
    dal = fma(KDb1, dser(kw + KW_KD1), dal);
    dal = fma(PDb0, dser(kw + KW_PD0), dal);
    dal = fma(PDb1, dser(kw + KW_PD1), dal);
    dal = fma(QDb0, dser(kw + KW_QD0), dal);
    dal = fma(QDb1, dser(kw + KW_QD1), dal);
    dal = fma(kdb0, dser(kw + KW_KX0), dal);
    dal = fma(kdb1, dser(kw + KW_KX1), dal);
    dal = fma(kRb, dser(kw + KW_KC), dal);
    alphab = kTwoPi * dal;   // per cycle of the orbit phase
  } else {
  // ---- projections: P = c0 ua + c1 ub + c2 ca + c3 sa + c4
  double uab = 0.0, ubb = 0.0, cab = kRb * wd(D_KR), sab = kRb * wd(D_KR + 1);
  DepSky::add(g, kRb * ca, td(D_KR));
  DepSky::add(g, kRb * sa, td(D_KR + 1));
#define PES_LIN_ADJ(off, pb)                   \
  {                                            \
    uab = fma(pb, wd((off)), uab);             \
    ubb = fma(pb, wd((off) + 1), ubb);         \
    cab = fma(pb, wd((off) + 2), cab);         \
    sab = fma(pb, wd((off) + 3), sab);         \
  }
  PES_LIN_ADJ(D_KN, knb0)
  PES_LIN_ADJ(D_KN + 5, knb1)
  PES_LIN_ADJ(D_NP, npb0)
  PES_LIN_ADJ(D_NP + 5, npb1)
  PES_LIN_ADJ(D_NQ, nqb0)
  PES_LIN_ADJ(D_NQ + 5, nqb1)
  PES_LIN_ADJ(D_KD, kdb0)
  PES_LIN_ADJ(D_KD + 5, kdb1)
  // ---- sky part.  The projections are kn_t = k.n_t, np_t = p.n_t,
  // nq_t = q.n_t, kd_t = k.Delta_t of the unit vectors k, p, q onto the arm
  // directions n_t and spacecraft offsets Delta_t at t_f, whose coefficients
  // alone depend on (lambda, beta, psi).  So d l / d theta_J gets
  //   K.dk_J + P.dp_J + Q.dq_J,  K = sum_t knb_t n_t + kdb_t Delta_t,
  //   P = sum_t npb_t n_t,  Q = sum_t nqb_t n_t.
  // The offsets of a centred triangle are Delta_0 = L (n_0 + 2 n_1) / 3 and
  // Delta_1 = -L (2 n_0 + n_1) / 3, so K = sum_t kap_t n_t.  Writing
  // n_t = kn_t k + np_t p + nq_t q in the orthonormal triad and using
  // k.dk = p.dp = q.dq = 0, k.dp = -p.dk, k.dq = -q.dk, p.dq = -q.dp:
  //   d l / d theta_J += (p.dk_J) S_a + (q.dk_J) S_b + (q.dp_J) S_c,
  //   S_a = sum_t kap_t np_t - npb_t kn_t,  S_b = sum_t kap_t nq_t - nqb_t kn_t,
  //   S_c = sum_t npb_t nq_t - nqb_t np_t,
  // three sums per lane, contracted once per block by the kernel.
  {
    const double kap0 = fma(L3, fma(-2.0, kdb1, kdb0), knb0);
    const double kap1 = fma(L3, fma(2.0, kdb0, -kdb1), knb1);
    g[kNParams] = fma(kap0, np0, fma(-npb0, kn0, fma(kap1, np1, fma(-npb1, kn1, g[kNParams]))));
    g[kNParams + 1] = fma(kap0, nq0, fma(-nqb0, kn0, fma(kap1, nq1, fma(-nqb1, kn1, g[kNParams + 1]))));
    g[kNParams + 2] = fma(npb0, nq0, fma(-nqb0, np0, fma(npb1, nq1, fma(-nqb1, np1, g[kNParams + 2]))));
  }
#undef PES_LIN_ADJ
  // ---- orbit at t_f
  if (GEO) {
    const double betab = kTwoPi * fma(ubb, ua, -(uab * ub));
    taub = betab * inv_ptq;
    DepTc::add(g, betab, td(D_PO));
  } else {
    sab = fma(-4.0 * sa, uab, fma(2.0 * ca, ubb, sab));
    cab = fma(2.0 * sa, ubb, cab);
  }
  alphab = kTwoPi * fma(sab, ca, -(cab * sa));
  }
  taub = fma(alphab, inv_year, taub);
  DepTc::add(g, alphab, td(D_AO));
  // ---- amplitude, polarization, taper
  DepIota::add(g, aPb * amp, tm(M_KP));
  DepIota::add(g, aCb * amp, tm(M_KC));
  const double ampb = fma(aPb, wm(M_KP), aCb * wm(M_KC));   // aCb: adjoint of 2 aC
  double xb = ampb * amp0 * dtap;
  const double qa = ampb * tap * b.fm76;
  double qn = 0.0;
  if (PAIR) {
    DepIota::add(g, aPb * amn, tr(R_KPR));
    DepIota::add(g, aPib * amn, tr(R_KPI));
    DepIota::add(g, aCb * amn, tr(R_KCR));
    DepIota::add(g, aCib * amn, tr(R_KCI));
    const double amnb = fma(aPb, wr(R_KPR), fma(aPib, wr(R_KPI), fma(aCb, wr(R_KCR), aCib * wr(R_KCI))));
    xb = fma(amnb * amn0, dtap, xb);
    qn = amnb * tap * b.fm76;
  }
  DepM::add(g, xb * b.f, tm(M_FCI));
  // recompute the waveform powers (from opaque copies of the bin values, so
  // the forward ones are not kept alive)
  const double v = wm(M_CM) * opaque(b.f13);
  const double w = wm(M_CMI) * opaque(b.fm13);
  const double lnv = opaque(b.lnf) * (1.0 / 3.0) + wm(M_LNCM);
  const double w2 = w * w, w3 = w2 * w, w4 = w2 * w2, w5 = w4 * w, w6 = w4 * w2, w8 = w4 * w4;
  const double v2 = v * v, lv = lnv * v, lw2 = lnv * w2;
  // The contractions below group each parameter's terms first (sum over the
  // entries of basis value x tangent) and scale by the common adjoint once.
  // amplitude: A = AM0 + AM1 v + AM2 v^2 on (M, q, D_L)
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int J = r == 2 ? 4 : r;
    double d = fma(v2, tm(M_AM2)[r], fma(v, tm(M_AM1)[r], tm(M_AM0)[r]));
    if (PAIR) d = fma(qn, fma(v2, tnm(M_AM2)[r], fma(v, tnm(M_AM1)[r], tnm(M_AM0)[r])), qa * d);
    else d = qa * d;
    g[J] += d;
  }
  double vb = qa * fma(2.0 * wm(M_AM2), v, wm(M_AM1));
  if (PAIR) vb = fma(qn, fma(2.0 * wn(M_AM2), v, wn(M_AM1)), vb);
  // ---- t_f - t_c
  // t_f series on (M, q) for every entry, (chi1, chi2) for T4 and T3
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    double d = w * tm(M_T7)[r];
    d = fma(w2, tm(M_T6)[r], d);
    d = fma(lw2, tm(M_T6L)[r], d);
    d = fma(w3, tm(M_T5)[r], d);
    d = fma(w4, tm(M_T4)[r], d);
    d = fma(w5, tm(M_T3)[r], d);
    d = fma(w6, tm(M_T2)[r], d);
    d = fma(w8, tm(M_T0)[r], d);
    g[r] = fma(taub, d, g[r]);
  }
#pragma unroll
  for (int r = 2; r < 4; ++r) g[r] = fma(taub, fma(w4, tm(M_T4)[r], w5 * tm(M_T3)[r]), g[r]);
  // d tau / d w
  double dtw = 8.0 * wm(M_T0) * w;
  dtw = fma(dtw, w, 6.0 * wm(M_T2));
  dtw = fma(dtw, w, 5.0 * wm(M_T3));
  dtw = fma(dtw, w, 4.0 * wm(M_T4));
  dtw = fma(dtw, w, 3.0 * wm(M_T5));
  dtw = fma(dtw, w, 2.0 * fma(wm(M_T6L), lnv, wm(M_T6)));
  dtw = fma(dtw, w, wm(M_T7));
  double wb = taub * dtw;
  double lnvb = taub * wm(M_T6L) * w2;
  // ---- phase
  const double phb = Phib;
  DepTc::add(g, phb * b.f, tn);
  {   // phase series on q for every entry, (chi1, chi2) for A3 and A4, phi_c for C0
    double d = fma(w5, tm(M_A0)[0], tm(M_C0)[0]);
    d = fma(w3, tm(M_A2)[0], d);
    d = fma(w2, tm(M_A3)[0], d);
    d = fma(w, tm(M_A4)[0], d);
    d = fma(lnv, tm(M_B5)[0], d);
    d = fma(v, tm(M_A6)[0], d);
    d = fma(lv, tm(M_B6)[0], d);
    d = fma(v2, tm(M_A7)[0], d);
    g[1] = fma(phb, d, g[1]);
#pragma unroll
    for (int r = 1; r < 3; ++r) g[r + 1] = fma(phb, fma(w2, tm(M_A3)[r], w * tm(M_A4)[r]), g[r + 1]);
    g[6] = fma(phb, tm(M_C0)[1], g[6]);
  }
  const double dpw = fma(fma(5.0 * wm(M_A0), w2, 3.0 * wm(M_A2)), w2, fma(2.0 * wm(M_A3), w, wm(M_A4)));
  wb = fma(phb, dpw, wb);
  lnvb = fma(phb, fma(wm(M_B6), v, wm(M_B5)), lnvb);
  vb = fma(phb, fma(2.0 * wm(M_A7), v, fma(wm(M_B6), lnv, wm(M_A6))), vb);
  // ---- v = CM f^{1/3}, w = CMI f^{-1/3}, ln v = LNCM + ln(f)/3
  DepM::add(g, vb * b.f13, tm(M_CM));
  DepM::add(g, wb * b.fm13, tm(M_CMI));
  DepM::add(g, lnvb, tm(M_LNCM));
#undef wm
#undef wd
#undef wn
#undef wr
#undef tm
#undef tnm
#undef tr
#undef td
}

}  // namespace pes
