// Single-precision variant of the per-(walker, bin, detector) evaluation
// (the FP32 side of the paper's FP32/FP64 comparison, Sec. 3.1 and Fig.
// fig_cost).  The quantities that need more than 24 bits stay in FP64: the
// mode's SPA phase (up to ~1e6 cycles) and t_f (up to ~3e7 s) from the same
// series as the FP64 evaluation, f t_c, the cutoff test, and the exact
// removal of whole cycles before every sine and cosine.  Everything after
// that -- amplitude and taper, the orbit at t_f, the projections (of the
// first-order triangle or the series of the exact Kepler ellipses), the
// Roemer delay, the polarization factors, the six links with their transfer
// functions and the TDI combinations -- runs in FP32 with FP32 fits, on FP32
// copies of the walker table and of the orbit series.  The channels are returned in FP32; the
// caller forms the noise-weighted inner products in FP64.
#pragma once
#include "pes_eval.hpp"

namespace pes {

template <int CLS>
__device__ __forceinline__ void sincos_small_fit_f(float x, float& s, float& c) {
  if constexpr (CLS == 0) {
    const float t = x * x;
    s = x * horner(kSinSmallC0F, t);
    c = horner(kCosSmallC0F, t);
  } else {
    sincos_small_f(x, s, c);
  }
}
template <bool LONG, int CLS>
__device__ __forceinline__ float sinc_fit_f(float b) {
  if constexpr (CLS == 0) {
    return horner(kSincC0F, b * b);
  } else {
    return sinc_f<LONG>(b);
  }
}

// wt: the walker's FP64 table (phase, t_f, cutoff, t_c); ws: its FP32 copy
// (everything else).  b: the bin's FP64 powers; a = pi f L, (zr, zi) =
// e^{-2 pi i f L} in FP32.  KEP: a heliocentric detector on exact Kepler
// ellipses, with FP32 copies of the walker's projected orbit series for this
// detector (kw, [KW_STRIDE]) and of the detector's inverse-arm-length series
// (kinv, [3][kKepT]).
template <bool GEO, bool LONG_SINC, int CLS, bool KEP = false>
__device__ __forceinline__ ChanT<float> eval_channels_f32(const double* __restrict__ wt,
                                                          const float* __restrict__ ws, int det,
                                                          const ModePlan& plan, double inv_year, double inv_ptq,
                                                          const BinRegs& b, float a, float zr, float zi,
                                                          const float* __restrict__ kw = nullptr,
                                                          const float* __restrict__ kinv = nullptr) {
  float yFr0 = 0.0f, yFi0 = 0.0f, yBr0 = 0.0f, yBi0 = 0.0f;
  float yFr1 = 0.0f, yFi1 = 0.0f, yBr1 = 0.0f, yBi1 = 0.0f;
  float yFr2 = 0.0f, yFi2 = 0.0f, yBr2 = 0.0f, yBi2 = 0.0f;
  const double ftc = frac_prod(b.f, wt[W_TC]);
  const float ff = (float)b.f;
  const float fm76 = (float)b.fm76;
  const float half_f = 0.5f * ff;
  const float pi_f = 3.14159265358979f * ff;
  const int D0 = W_DET0 + det * W_DET_STRIDE;

  auto unit = [&](int j, int jm, auto pair) __attribute__((always_inline)) {
    constexpr bool PAIR = decltype(pair)::value;
    const int M0 = W_MODE0 + j * W_MODE_STRIDE;
#define wm(i) wt[M0 + (i)]
#define sm(i) ws[M0 + (i)]
#define sd(i) ws[D0 + (i)]
    const double x = b.f * wm(M_FCI);
    if (!(x < 1.0)) return;  // beyond this mode's cutoff
    // FP64: the SPA phase (cycles) and t_f - t_c (eq. eq_tf)
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
    const double phase = ftc + (ph + wm(M_C0));
    double tau = wm(M_T7) * w;
    tau = fma(wm(M_T6), w2, tau);
    tau = fma(wm(M_T6L), lw2, tau);
    tau = fma(wm(M_T5), w3, tau);
    tau = fma(wm(M_T4), w4, tau);
    tau = fma(wm(M_T3), w5, tau);
    tau = fma(wm(M_T2), w6, tau);
    tau = fma(wm(M_T0), w8, tau);
    // FP32 from here: amplitude with the C^2 cutoff taper
    const float vf = (float)v;
    float scale = fm76;
    if (x > 0.9) {
      const float t = ((float)x - 0.9f) * 10.0f;
      scale *= fmaf(-(t * t * t), fmaf(t, fmaf(6.0f, t, -15.0f), 10.0f), 1.0f);
    }
    float amp = sm(M_AM1) * vf;
    amp = fmaf(sm(M_AM2), vf * vf, amp) + sm(M_AM0);
    amp *= scale;
    float aP = amp * sm(M_KP);
    float aC2 = amp * sm(M_KC);
    float aPi = 0.0f, aCi = 0.0f;
    if (PAIR) {
      const int N0 = W_MODE0 + jm * W_MODE_STRIDE, R0 = W_ROT0 + R_STRIDE * jm;
      float am = ws[N0 + M_AM1] * vf;
      am = fmaf(ws[N0 + M_AM2], vf * vf, am) + ws[N0 + M_AM0];
      am *= scale;
      aP = fmaf(am, ws[R0 + R_KPR], aP);
      aPi = am * ws[R0 + R_KPI];
      aC2 = fmaf(am, ws[R0 + R_KCR], aC2);
      aCi = am * ws[R0 + R_KCI];
    }
    // spacecraft geometry at t_f: the orbit phases reduced in FP64
    float sa, ca;
    sincos_cycles_f(fma(tau, inv_year, wt[D0 + D_AO]), sa, ca);
    float kn0, kn1, kn2, np0, np1, np2, nq0, nq1, nq2, kd0, kd1, kR;
    if constexpr (KEP) {
      // exact Kepler ellipses: the same series as the FP64 evaluation, in FP32
      // (harmonics cos k alpha, sin k alpha by the Chebyshev recurrence)
      float hc[kKepH + 1], hs[kKepH + 1];
      hc[0] = 1.0f;
      hs[0] = 0.0f;
      hc[1] = ca;
      hs[1] = sa;
      const float c2a = 2.0f * ca;
#pragma unroll
      for (int k = 2; k <= kKepH; ++k) {
        hc[k] = fmaf(c2a, hc[k - 1], -hc[k - 2]);
        hs[k] = fmaf(c2a, hs[k - 1], -hs[k - 2]);
      }
      auto series = [&](const float* __restrict__ c) __attribute__((always_inline)) {
        float r = c[0];
#pragma unroll
        for (int k = 1; k <= kKepH; ++k) r = fmaf(c[2 * k - 1], hc[k], fmaf(c[2 * k], hs[k], r));
        return r;
      };
      const float iL0 = series(kinv), iL1 = series(kinv + kKepT), iL2 = series(kinv + 2 * kKepT);
      const float KD0 = series(kw + KW_KD0), KD1 = series(kw + KW_KD1);
      const float PD0 = series(kw + KW_PD0), PD1 = series(kw + KW_PD1);
      const float QD0 = series(kw + KW_QD0), QD1 = series(kw + KW_QD1);
      kn0 = KD0 * iL0;
      kn1 = KD1 * iL1;
      kn2 = -(KD0 + KD1) * iL2;
      np0 = PD0 * iL0;
      np1 = PD1 * iL1;
      np2 = -(PD0 + PD1) * iL2;
      nq0 = QD0 * iL0;
      nq1 = QD1 * iL1;
      nq2 = -(QD0 + QD1) * iL2;
      kd0 = series(kw + KW_KX0);
      kd1 = series(kw + KW_KX1);
      kR = series(kw + KW_KC);
    } else {
      float ua, ub;
      if (GEO) {
        sincos_cycles_f(fma(tau, inv_ptq, wt[D0 + D_PO]), ub, ua);
      } else {
        ua = fmaf(-2.0f * sa, sa, 1.0f);
        ub = 2.0f * sa * ca;
      }
#define PES_LIN(off) (fmaf(sd((off) + 3), sa, fmaf(sd((off) + 2), ca, fmaf(sd((off) + 1), ub, sd((off)) * ua))) + sd((off) + 4))
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
      kR = fmaf(sd(D_KR), ca, sd(D_KR + 1) * sa);
    }
    // mode phase plus the Roemer delay, whole cycles removed in FP64
    float sp, cp;
    sincos_cycles_f(fma(b.f, (double)kR, phase), sp, cp);
    float pEr, pEi, cEr, cEi;
    if (PAIR) {
      pEr = fmaf(aP, cp, aPi * sp);
      pEi = fmaf(aPi, cp, -(aP * sp));
      cEr = fmaf(aC2, cp, aCi * sp);
      cEi = fmaf(aCi, cp, -(aC2 * sp));
    } else {
      pEr = aP * cp;
      pEi = -(aP * sp);
      cEr = aC2 * cp;
      cEi = -(aC2 * sp);
    }
    // per-arm phase e^{+i pi f k.Delta_t}
    float s0, c0, s1, c1;
    if (LONG_SINC && CLS == 1) {
      sincos_rev_f(half_f * kd0, s0, c0);   // |f k.Delta / 2| < 1/2 cycle on every grid the fits allow
      sincos_rev_f(half_f * kd1, s1, c1);
    } else {
      sincos_small_fit_f<CLS>(pi_f * kd0, s0, c0);
      sincos_small_fit_f<CLS>(pi_f * kd1, s1, c1);
    }
    const float c2 = fmaf(c0, c1, -(s0 * s1)), s2 = -fmaf(s0, c1, c0 * s1);
#define PES_ARM(er, ei, np, nq, kn, FR, FI, BR, BI)                      \
  {                                                                     \
    const float pp = fmaf(np, np, -(nq * nq)), pc = np * nq;            \
    const float Wr = fmaf(pp, pEr, -(pc * cEi)), Wi = fmaf(pp, pEi, pc * cEr); \
    const float Gr = fmaf(Wr, er, -(Wi * ei)), Gi = fmaf(Wr, ei, Wi * er); \
    const float sf = sinc_fit_f<LONG_SINC, CLS>(fmaf(-a, kn, a)), sb = sinc_fit_f<LONG_SINC, CLS>(fmaf(a, kn, a)); \
    FR = fmaf(sf, Gr, FR);                                              \
    FI = fmaf(sf, Gi, FI);                                              \
    BR = fmaf(sb, Gr, BR);                                              \
    BI = fmaf(sb, Gi, BI);                                              \
  }
    PES_ARM(c0, s0, np0, nq0, kn0, yFr0, yFi0, yBr0, yBi0)
    PES_ARM(c1, s1, np1, nq1, kn1, yFr1, yFi1, yBr1, yBi1)
    PES_ARM(c2, s2, np2, nq2, kn2, yFr2, yFi2, yBr2, yBi2)
#undef PES_ARM
#undef wm
#undef sm
#undef sd
  };
  for (int u = 0; u < plan.n_pairs; ++u) unit(plan.lead[u], plan.member[u], std::true_type{});
  for (int u = plan.n_pairs; u < plan.n_units; ++u) unit(plan.lead[u], -1, std::false_type{});
  // TDI X, Y, Z (the common factor G is in the tables) and A'', E'', T''
  const float xr1 = yBr1 - yFr2, xi1 = yBi1 - yFi2;
  const float Xr = yFr1 - yBr2 + (zr * xr1 - zi * xi1);
  const float Xi = yFi1 - yBi2 + (zr * xi1 + zi * xr1);
  const float yr1 = yBr2 - yFr0, yi1 = yBi2 - yFi0;
  const float Yr = yFr2 - yBr0 + (zr * yr1 - zi * yi1);
  const float Yi = yFi2 - yBi0 + (zr * yi1 + zi * yr1);
  const float zr1 = yBr0 - yFr1, zi1 = yBi0 - yFi1;
  const float Zr = yFr0 - yBr1 + (zr * zr1 - zi * zi1);
  const float Zi = yFi0 - yBi1 + (zr * zi1 + zi * zr1);
  ChanT<float> c;
  c.ar = Zr - Xr;
  c.ai = Zi - Xi;
  c.er = Xr - 2.0f * Yr + Zr;
  c.ei = Xi - 2.0f * Yi + Zi;
  c.tr = Xr + Yr + Zr;
  c.ti = Xi + Yi + Zi;
  return c;
}

template <bool GEO, bool LONG_SINC, bool KEP = false>
__device__ __forceinline__ ChanT<float> eval_channels_f32_cls(int cls, const double* __restrict__ wt,
                                                              const float* __restrict__ ws, int det,
                                                              const ModePlan& plan, double inv_year, double inv_ptq,
                                                              const BinRegs& b, float a, float zr, float zi,
                                                              const float* __restrict__ kw = nullptr,
                                                              const float* __restrict__ kinv = nullptr) {
  if (cls == 0)
    return eval_channels_f32<GEO, LONG_SINC, 0, KEP>(wt, ws, det, plan, inv_year, inv_ptq, b, a, zr, zi, kw, kinv);
  return eval_channels_f32<GEO, LONG_SINC, 1, KEP>(wt, ws, det, plan, inv_year, inv_ptq, b, a, zr, zi, kw, kinv);
}

}  // namespace pes
