// Per-(walker, bin, detector) evaluation of the response: every active mode's
// amplitude, phase and t_f (SPA, eq. eq_tf), the orbit at t_f, the six link
// transfer functions (eq. eq_fd_resp), summed over modes, then the TDI
// combinations X, Y, Z and the unnormalized channels A'' = Z - X,
// E'' = X - 2Y + Z, T'' = X + Y + Z (Sec. 2.1).  The per-bin common factor G
// and the channel normalizations are folded into the bin tables.
#pragma once
#include <type_traits>
#include "pes_dual.hpp"
#include "pes_layout.hpp"
#include "pes_math.hpp"

namespace pes {

// ---- walker-constant accessors: values only, or (value, tangent k)
struct ValTab {
  const double* __restrict__ w;
  __device__ __forceinline__ double operator()(int i) const { return w[i]; }
};
struct TanTab {
  const double* __restrict__ w;   // values [W_STRIDE]
  const double* __restrict__ t;   // tangents [W_STRIDE][kNParams]
  int k;                          // tangent direction
  __device__ __forceinline__ Dual<1> operator()(int i) const {
    Dual<1> r;
    r.v = w[i];
    r.d[0] = t[i * kNParams + k];
    return r;
  }
};

// Kepler orbit series coefficients are constant while a kernel runs and the
// same for every lane: read through the constant address space, they come in
// by scalar loads instead of occupying vector registers.  The derivative
// kernels read them so (KwScalar, KwLane); the log-likelihood and response
// kernels, whose scalar registers are the tighter ones, keep plain loads.
typedef const __attribute__((address_space(4))) double cdouble;
__device__ __forceinline__ cdouble* as_const(const double* p) { return (cdouble*)p; }
struct KwScalar {
  const double* __restrict__ p;
};

// The projected Kepler orbit series of a walker in the tangent kernels: the
// values (wavefront-uniform) and this lane's tangent row (zeros unless its
// direction is a sky angle).
struct KwLane {
  const double* __restrict__ v;
  const double* __restrict__ t;
};
__device__ __forceinline__ double kw_at(const double* __restrict__ kw, int i) { return kw[i]; }
__device__ __forceinline__ double kw_at(const KwScalar& kw, int i) { return as_const(kw.p)[i]; }
__device__ __forceinline__ Dual<1> kw_at(const KwLane& kw, int i) {
  Dual<1> r;
  r.v = as_const(kw.v)[i];
  r.d[0] = kw.t[i];
  return r;
}

// The same with a direction that may differ between lanes (the values stay
// wavefront-uniform, the tangents are per-lane loads).
struct TanTabLane {
  const double* __restrict__ w;
  const double* __restrict__ t;
  int k;
  __device__ __forceinline__ Dual<1> operator()(int i) const {
    Dual<1> r;
    r.v = w[i];
    r.d[0] = t[i * kNParams + k];
    return r;
  }
};

// ---- math on the tangent type (value by the double kernels, derivative by hand)
__device__ __forceinline__ void sincos_cycles(const Dual<1>& x, Dual<1>& s, Dual<1>& c) {
  sincos_cycles(x.v, s.v, c.v);
  s.d[0] = kTwoPi * c.v * x.d[0];
  c.d[0] = -kTwoPi * s.v * x.d[0];
}
__device__ __forceinline__ void sincos_small(const Dual<1>& x, Dual<1>& s, Dual<1>& c) {
  sincos_small(x.v, s.v, c.v);
  s.d[0] = c.v * x.d[0];
  c.d[0] = -s.v * x.d[0];
}
template <bool LONG>
__device__ __forceinline__ Dual<1> sinc(const Dual<1>& b) {
  const double t = b.v * b.v;
  double p, dp;
  if (LONG) horner_d<1>(kSincLong, t, p, dp);
  else horner_d<1>(kSincShort, t, p, dp);
  Dual<1> r;
  r.v = p;
  r.d[0] = 2.0 * b.v * dp * b.d[0];
  return r;
}
// f t_c modulo 1 (exact product split), with its derivative f dt_c.
__device__ __forceinline__ double frac_prod(double f, double tc) {
  double pt, et;
  two_prod(f, tc, pt, et);
  return (pt - rint(pt)) + et;
}
__device__ __forceinline__ Dual<1> frac_prod(double f, const Dual<1>& tc) {
  Dual<1> r;
  r.v = frac_prod(f, tc.v);
  r.d[0] = f * tc.d[0];
  return r;
}

// Fit classes of the log-likelihood kernel: a wavefront of bins whose link
// sinc arguments all stay at or below kClassBMax0 (class 0) evaluates the sinc
// and the arm phases with shorter fits of that range; class 1 is the full
// range (the short or long sinc fit of the context).  Every fit is at FP64
// rounding level on its range.
template <int CLS>
__device__ __forceinline__ void sincos_small_fit(double x, double& s, double& c) {
  if constexpr (CLS == 0) {
    const double t = x * x;
    s = x * horner(kSinSmallC0, t);
    c = horner(kCosSmallC0, t);
  } else {
    sincos_small(x, s, c);
  }
}
template <int CLS>
__device__ __forceinline__ void sincos_small_fit(const Dual<1>& x, Dual<1>& s, Dual<1>& c) {
  static_assert(CLS == 1, "tangent kernels use the full-range fits");
  sincos_small(x, s, c);
}
template <bool LONG, int CLS>
__device__ __forceinline__ double sinc_fit(double b) {
  if constexpr (CLS == 0) {
    return horner(kSincC0, b * b);
  } else {
    return sinc<LONG>(b);
  }
}
template <bool LONG, int CLS>
__device__ __forceinline__ Dual<1> sinc_fit(const Dual<1>& b) {
  static_assert(CLS == 1, "tangent kernels use the full-range fits");
  return sinc<LONG>(b);
}
// Class of a wavefront whose largest link sinc argument (2 pi f L at its
// highest frequency) is bmax.
__device__ __forceinline__ int fit_class(double bmax) { return bmax <= kClassBMax0 ? 0 : 1; }

struct BinRegs {
  double f, f13, fm13, fm76, lnf;
};

// A wave-uniform int the compiler must treat as unknown: table offsets built
// from it inside a loop are not hoisted out of it (the entries are loaded again
// from the scalar cache instead of held in scalar registers across the loop).
__device__ __forceinline__ int opaque_u(int x) {
  asm volatile("" : "+s"(x));
  return x;
}

struct Chan {
  double ar, ai, er, ei, tr, ti;
};

template <class S>
struct ChanT {
  S ar, ai, er, ei, tr, ti;
};

// Hooks into the stages of one evaluation, for the stage probes of the test
// suite; the hot path passes NoProbe, whose empty hooks compile to nothing.
struct NoProbe {
  template <class S>
  __device__ __forceinline__ void mode(int, const S&, const S&, const S&) const {}
  template <class S>
  __device__ __forceinline__ void geom(int, const S*, const S*, const S*, const S*, const S&) const {}
  template <class S>
  __device__ __forceinline__ void links(const S*) const {}
};

// Tab: accessor of this walker's constant table (wavefront-uniform); det: the
// detector block.  S = double (values) or Dual<1> (value and one tangent).
// GEO selects the geocentric orbit.  a = pi f L, (zr, zi) = e^{-2 pi i f L}.
// KEP: heliocentric detector on exact Kepler ellipses; kw: the walker's
// projected orbit series for this detector [KW_STRIDE] (a KwLane for S =
// Dual<1>), kinv: the
// detector's inverse-arm-length series [3][kKepT].
template <bool GEO, bool LONG_SINC, int CLS, class S, class Tab, class Probe = NoProbe, bool KEP = false,
          class KWA = const double*>
__device__ __forceinline__ ChanT<S> eval_channels_t(const Tab& T, int det, const ModePlan& plan,
                                                    double inv_year, double inv_ptq, const BinRegs& b,
                                                    double a, double zr, double zi,
                                                    const Probe& probe = Probe(),
                                                    KWA kw = KWA(),
                                                    const double* __restrict__ kinv = nullptr) {
  S yFr0 = 0.0, yFi0 = 0.0, yBr0 = 0.0, yBi0 = 0.0;
  S yFr1 = 0.0, yFi1 = 0.0, yBr1 = 0.0, yBi1 = 0.0;
  S yFr2 = 0.0, yFi2 = 0.0, yBr2 = 0.0, yBi2 = 0.0;
  // f t_c mod 1 to ~1e-16 absolute: exact product split, exact integer removal.
  const S ftc = frac_prod(b.f, T(W_TC));
  const double half_f = 0.5 * b.f;
  const double pi_f = kPi * b.f;

  // One evaluation unit: mode j and, when PAIR, the mode jm with the same m
  // added as a complex amplitude on j's phase factor.
  auto unit = [&](int j, int jm, auto pair) __attribute__((always_inline)) {
    constexpr bool PAIR = decltype(pair)::value;
    // Walker constants (wavefront-uniform, in scalar registers) enter as
    // multiplicands or plain addends, never as the addend of a fused
    // multiply-add, so no vector copy of a scalar operand is needed.
    const int M0 = W_MODE0 + j * W_MODE_STRIDE;
#define wm(i) T(M0 + (i))
#define wd(i) T(D0 + (i))
    const S x = b.f * wm(M_FCI);
    if (!(val(x) < 1.0)) return;  // beyond this mode's cutoff (diverges only in the cutoff tile)
    const S v = wm(M_CM) * b.f13;
    const S w = wm(M_CMI) * b.fm13;
    const S lnv = b.lnf * (1.0 / 3.0) + wm(M_LNCM);
    const S w2 = w * w, w3 = w2 * w, w4 = w2 * w2, w5 = w4 * w, w6 = w4 * w2, w8 = w4 * w4;
    const S v2 = v * v, lv = lnv * v, lw2 = lnv * w2;
    // SPA phase of the mode, in cycles
    S ph = wm(M_A4) * w;
    ph = fma(wm(M_A3), w2, ph);
    ph = fma(wm(M_A2), w3, ph);
    ph = fma(wm(M_A0), w5, ph);
    ph = fma(wm(M_B5), lnv, ph);
    ph = fma(wm(M_A6), v, ph);
    ph = fma(wm(M_B6), lv, ph);
    ph = fma(wm(M_A7), v2, ph);
    const S phase = ftc + (ph + wm(M_C0));
    // t_f - t_c from the same series (eq. eq_tf)
    S tau = wm(M_T7) * w;
    tau = fma(wm(M_T6), w2, tau);
    tau = fma(wm(M_T6L), lw2, tau);
    tau = fma(wm(M_T5), w3, tau);
    tau = fma(wm(M_T4), w4, tau);
    tau = fma(wm(M_T3), w5, tau);
    tau = fma(wm(M_T2), w6, tau);
    tau = fma(wm(M_T0), w8, tau);
    // amplitude with the C^2 cutoff taper (evaluated only where x > 0.9)
    S scale = b.fm76;
    if (val(x) > 0.9) {
      const S t = (x - 0.9) * 10.0;
      scale *= fma(-(t * t * t), fma(t, fma(6.0, t, -15.0), 10.0), 1.0);
    }
    S amp = wm(M_AM1) * v;
    amp = fma(wm(M_AM2), v2, amp) + wm(M_AM0);
    amp *= scale;
    probe.mode(j, amp, phase, tau);   // amplitude with taper, phase [cycles], t_f - t_c [s]
    S aP = amp * wm(M_KP);
    S aC2 = amp * wm(M_KC);   // the table holds 2 K_x
    // the paired mode: its amplitude on the rotated polarization factors
    S aPi = 0.0, aCi = 0.0;
    if (PAIR) {
      const int N0 = W_MODE0 + jm * W_MODE_STRIDE, R0 = W_ROT0 + R_STRIDE * jm;
      S am = T(N0 + M_AM1) * v;
      am = fma(T(N0 + M_AM2), v2, am) + T(N0 + M_AM0);
      am *= scale;
      aP = fma(am, T(R0 + R_KPR), aP);
      aPi = am * T(R0 + R_KPI);
      aC2 = fma(am, T(R0 + R_KCR), aC2);
      aCi = am * T(R0 + R_KCI);
    }
    // spacecraft geometry at t_f.  In the tangent kernels the detector entries
    // are loaded from here on (opaque_u), which keeps their scalar registers
    // free through the waveform part; the value kernels keep the default.
    const int D0 = W_DET0 + (std::is_same<S, double>::value ? det : opaque_u(det)) * W_DET_STRIDE;
    S sa, ca;
    sincos_cycles(tau * inv_year + wd(D_AO), sa, ca);
    S kn0, kn1, kn2, np0, np1, np2, nq0, nq1, nq2, kd0, kd1, kR;
    if constexpr (KEP) {
      // exact Kepler ellipses: every projection is a series in the harmonics
      // of alpha; the link directions are the separations over their lengths
      S hc[kKepH + 1], hs[kKepH + 1];
      hc[0] = 1.0;
      hs[0] = 0.0;
      hc[1] = ca;
      hs[1] = sa;
      const S c2a = 2.0 * ca;
#pragma unroll
      for (int k = 2; k <= kKepH; ++k) {
        hc[k] = fma(c2a, hc[k - 1], -hc[k - 2]);
        hs[k] = fma(c2a, hs[k - 1], -hs[k - 2]);
      }
      auto series = [&](const double* __restrict__ cg) __attribute__((always_inline)) {
        S r;
        if constexpr (std::is_same<KWA, const double*>::value) {
          const double* __restrict__ c = cg;
          r = c[0];
#pragma unroll
          for (int k = 1; k <= kKepH; ++k) r = fma(c[2 * k - 1], hc[k], fma(c[2 * k], hs[k], r));
          return r;
        }
        cdouble* c = as_const(cg);
        r = c[0];
#pragma unroll
        for (int k = 1; k <= kKepH; ++k) r = fma(c[2 * k - 1], hc[k], fma(c[2 * k], hs[k], r));
        return r;
      };
      // the same over the walker's series (coefficients with tangents in the tangent kernels)
      auto series_w = [&](int off) __attribute__((always_inline)) {
        S r = kw_at(kw, off);
#pragma unroll
        for (int k = 1; k <= kKepH; ++k)
          r = fma(kw_at(kw, off + 2 * k - 1), hc[k], fma(kw_at(kw, off + 2 * k), hs[k], r));
        return r;
      };
      const S iL0 = series(kinv), iL1 = series(kinv + kKepT), iL2 = series(kinv + 2 * kKepT);
      const S KD0 = series_w(KW_KD0), KD1 = series_w(KW_KD1);
      const S PD0 = series_w(KW_PD0), PD1 = series_w(KW_PD1);
      const S QD0 = series_w(KW_QD0), QD1 = series_w(KW_QD1);
      kn0 = KD0 * iL0;
      kn1 = KD1 * iL1;
      kn2 = -(KD0 + KD1) * iL2;
      np0 = PD0 * iL0;
      np1 = PD1 * iL1;
      np2 = -(PD0 + PD1) * iL2;
      nq0 = QD0 * iL0;
      nq1 = QD1 * iL1;
      nq2 = -(QD0 + QD1) * iL2;
      kd0 = series_w(KW_KX0);
      kd1 = series_w(KW_KX1);
      kR = series_w(KW_KC);
    } else {
      S ua, ub;
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
    {
      const S knv[3] = {kn0, kn1, kn2}, npv[3] = {np0, np1, np2}, nqv[3] = {nq0, nq1, nq2}, kdv[2] = {kd0, kd1};
      probe.geom(j, knv, npv, nqv, kdv, kR);
    }
    // mode phase plus the Roemer delay of the centre: E = e^{-2 pi i (phase + f k.R)}
    S sp, cp;
    sincos_cycles(fma(b.f, kR, phase), sp, cp);
    // polarization amplitudes times E = (cp, -sp): aP E and 2 aC E
    S pEr, pEi, cEr, cEi;
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
    // per-arm phase e^{+i pi f k.Delta_t} of the spacecraft opposite arm t
    S s0, c0, s1, c1;
    if (LONG_SINC && CLS == 1) {
      sincos_cycles(half_f * kd0, s0, c0);
      sincos_cycles(half_f * kd1, s1, c1);
    } else {  // |pi f k.Delta| <= pi f L / sqrt3 < 0.7 whenever the short sinc fit applies
      sincos_small_fit<CLS>(pi_f * kd0, s0, c0);
      sincos_small_fit<CLS>(pi_f * kd1, s1, c1);
    }
    const S c2 = fma(c0, c1, -(s0 * s1)), s2 = -fma(s0, c1, c0 * s1);

// One arm: W = E (aP (n.p)^2 - (n.q)^2) + i 2 aC (n.p)(n.q)), G = W e_arm,
// y_F += sinc(a (1 - k.n)) G, y_B += sinc(a (1 + k.n)) G.
#define PES_ARM(er, ei, np, nq, kn, FR, FI, BR, BI)                    \
  {                                                                   \
    const S pp = fma(np, np, -(nq * nq)), pc = np * nq;               \
    const S Wr = fma(pp, pEr, -(pc * cEi)), Wi = fma(pp, pEi, pc * cEr); \
    const S Gr = fma(Wr, er, -(Wi * ei)), Gi = fma(Wr, ei, Wi * er); \
    const S sf = sinc_fit<LONG_SINC, CLS>(fma(-a, kn, a)), sb = sinc_fit<LONG_SINC, CLS>(fma(a, kn, a)); \
    FR = fma(sf, Gr, FR);                                             \
    FI = fma(sf, Gi, FI);                                             \
    BR = fma(sb, Gr, BR);                                             \
    BI = fma(sb, Gi, BI);                                             \
  }
    PES_ARM(c0, s0, np0, nq0, kn0, yFr0, yFi0, yBr0, yBi0)
    PES_ARM(c1, s1, np1, nq1, kn1, yFr1, yFi1, yBr1, yBi1)
    PES_ARM(c2, s2, np2, nq2, kn2, yFr2, yFi2, yBr2, yBi2)
#undef PES_ARM
#undef wm
#undef wd
  };
  for (int u = 0; u < plan.n_pairs; ++u) unit(plan.lead[u], plan.member[u], std::true_type{});
  for (int u = plan.n_pairs; u < plan.n_units; ++u) unit(plan.lead[u], -1, std::false_type{});
  {
    const S yv[12] = {yFr0, yFi0, yBr0, yBi0, yFr1, yFi1, yBr1, yBi1, yFr2, yFi2, yBr2, yBi2};
    probe.links(yv);
  }
  // links: arm 0 carries y32 (F) / y23 (B), arm 1 y13 / y31, arm 2 y21 / y12.
  // X = y13 - y12 + z (y31 - y21), Y = y21 - y23 + z (y12 - y32),
  // Z = y32 - y31 + z (y23 - y13)   (the common factor G is in the tables)
  const S xr1 = yBr1 - yFr2, xi1 = yBi1 - yFi2;
  const S Xr = yFr1 - yBr2 + (zr * xr1 - zi * xi1);
  const S Xi = yFi1 - yBi2 + (zr * xi1 + zi * xr1);
  const S yr1 = yBr2 - yFr0, yi1 = yBi2 - yFi0;
  const S Yr = yFr2 - yBr0 + (zr * yr1 - zi * yi1);
  const S Yi = yFi2 - yBi0 + (zr * yi1 + zi * yr1);
  const S zr1 = yBr0 - yFr1, zi1 = yBi0 - yFi1;
  const S Zr = yFr0 - yBr1 + (zr * zr1 - zi * zi1);
  const S Zi = yFi0 - yBi1 + (zr * zi1 + zi * zr1);
  ChanT<S> c;
  c.ar = Zr - Xr;
  c.ai = Zi - Xi;
  c.er = Xr - 2.0 * Yr + Zr;
  c.ei = Xi - 2.0 * Yi + Zi;
  c.tr = Xr + Yr + Zr;
  c.ti = Xi + Yi + Zi;
  return c;
}

template <bool GEO, bool LONG_SINC, int CLS = 1, bool KEP = false, class KWA = const double*>
__device__ __forceinline__ Chan eval_channels(const double* __restrict__ wt, int det, const ModePlan& plan,
                                              double inv_year, double inv_ptq, const BinRegs& b,
                                              double a, double zr, double zi,
                                              KWA kw = KWA(),
                                              const double* __restrict__ kinv = nullptr) {
  const ChanT<double> c = eval_channels_t<GEO, LONG_SINC, CLS, double, ValTab, NoProbe, KEP, KWA>(
      ValTab{wt}, det, plan, inv_year, inv_ptq, b, a, zr, zi, NoProbe(), kw, kinv);
  return Chan{c.ar, c.ai, c.er, c.ei, c.tr, c.ti};
}

// eval_channels with the fit class chosen at run time (a wave-uniform branch).
template <bool GEO, bool LONG_SINC, bool KEP = false>
__device__ __forceinline__ Chan eval_channels_cls(int cls, const double* __restrict__ wt, int det,
                                                  const ModePlan& plan,
                                                  double inv_year, double inv_ptq, const BinRegs& b, double a,
                                                  double zr, double zi, const double* __restrict__ kw = nullptr,
                                                  const double* __restrict__ kinv = nullptr) {
  if (cls == 0)
    return eval_channels<GEO, LONG_SINC, 0, KEP>(wt, det, plan, inv_year, inv_ptq, b, a, zr, zi, kw, kinv);
  return eval_channels<GEO, LONG_SINC, 1, KEP>(wt, det, plan, inv_year, inv_ptq, b, a, zr, zi, kw, kinv);
}

}  // namespace pes
