// Per-(walker, bin, detector) evaluation of the response: every active mode's
// amplitude, phase and t_f (SPA, eq. eq_tf), the orbit at t_f, the six link
// transfer functions (eq. eq_fd_resp), summed over modes, then the TDI
// combinations X, Y, Z and the unnormalized channels A'' = Z - X,
// E'' = X - 2Y + Z, T'' = X + Y + Z (Sec. 2.1).  The per-bin common factor G
// and the channel normalizations are folded into the bin tables.
#pragma once
#include "pes_layout.hpp"
#include "pes_math.hpp"

namespace pes {

struct BinRegs {
  double f, f13, fm13, fm76, lnf;
};

struct Chan {
  double ar, ai, er, ei, tr, ti;
};

// wt: this walker's constant table (wavefront-uniform); wd: its detector block.
// GEO selects the geocentric orbit.  a = pi f L, (zr, zi) = e^{-2 pi i f L}.
template <bool GEO, bool LONG_SINC>
__device__ __forceinline__ Chan eval_channels(const double* __restrict__ wt,
                                              const double* __restrict__ wd, int n_modes,
                                              double inv_year, double inv_ptq, const BinRegs& b,
                                              double a, double zr, double zi) {
  double yFr0 = 0, yFi0 = 0, yBr0 = 0, yBi0 = 0;
  double yFr1 = 0, yFi1 = 0, yBr1 = 0, yBi1 = 0;
  double yFr2 = 0, yFi2 = 0, yBr2 = 0, yBi2 = 0;
  // f t_c mod 1 to ~1e-16 absolute: exact product split, exact integer removal.
  double pt, et;
  two_prod(b.f, wt[W_TC], pt, et);
  const double ftc = (pt - rint(pt)) + et;
  const double half_f = 0.5 * b.f;
  const double pi_f = kPi * b.f;

  for (int j = 0; j < n_modes; ++j) {
    // Walker constants (wavefront-uniform, in scalar registers) enter as
    // multiplicands or plain addends, never as the addend of a fused
    // multiply-add, so no vector copy of a scalar operand is needed.
    const double* __restrict__ wm = wt + W_MODE0 + j * W_MODE_STRIDE;
    const double x = b.f * wm[M_FCI];
    if (!(x < 1.0)) continue;  // beyond this mode's cutoff (diverges only in the cutoff tile)
    const double v = wm[M_CM] * b.f13;
    const double w = wm[M_CMI] * b.fm13;
    const double lnv = b.lnf * (1.0 / 3.0) + wm[M_LNCM];
    const double w2 = w * w, w3 = w2 * w, w4 = w2 * w2, w5 = w4 * w, w6 = w4 * w2, w8 = w4 * w4;
    const double v2 = v * v, lv = lnv * v, lw2 = lnv * w2;
    // SPA phase of the mode, in cycles
    double ph = wm[M_A4] * w;
    ph = fma(wm[M_A3], w2, ph);
    ph = fma(wm[M_A2], w3, ph);
    ph = fma(wm[M_A0], w5, ph);
    ph = fma(wm[M_B5], lnv, ph);
    ph = fma(wm[M_A6], v, ph);
    ph = fma(wm[M_B6], lv, ph);
    ph = fma(wm[M_A7], v2, ph);
    const double phase = ftc + (ph + wm[M_C0]);
    // t_f - t_c from the same series (eq. eq_tf)
    double tau = wm[M_T7] * w;
    tau = fma(wm[M_T6], w2, tau);
    tau = fma(wm[M_T6L], lw2, tau);
    tau = fma(wm[M_T5], w3, tau);
    tau = fma(wm[M_T4], w4, tau);
    tau = fma(wm[M_T3], w5, tau);
    tau = fma(wm[M_T2], w6, tau);
    tau = fma(wm[M_T0], w8, tau);
    // amplitude with the C^2 cutoff taper (evaluated only where x > 0.9)
    double amp = wm[M_AM1] * v;
    amp = fma(wm[M_AM2], v2, amp) + wm[M_AM0];
    amp *= b.fm76;
    if (x > 0.9) {
      const double u = (x - 0.9) * 10.0;
      amp *= fma(-u * u * u, fma(u, fma(6.0, u, -15.0), 10.0), 1.0);
    }
    const double aP = amp * wm[M_KP];
    const double aC = amp * wm[M_KC];
    // spacecraft geometry at t_f
    double sa, ca;
    sincos_cycles(tau * inv_year + wd[D_AO], sa, ca);
    double ua, ub;
    if (GEO) {
      sincos_cycles(tau * inv_ptq + wd[D_PO], ub, ua);
    } else {
      ua = fma(-2.0 * sa, sa, 1.0);
      ub = 2.0 * sa * ca;
    }
#define PES_LIN(off) (fma(wd[(off) + 3], sa, fma(wd[(off) + 2], ca, fma(wd[(off) + 1], ub, wd[(off)] * ua))) + wd[(off) + 4])
    const double kn0 = PES_LIN(D_KN), kn1 = PES_LIN(D_KN + 5);
    const double np0 = PES_LIN(D_NP), np1 = PES_LIN(D_NP + 5);
    const double nq0 = PES_LIN(D_NQ), nq1 = PES_LIN(D_NQ + 5);
    const double kd0 = PES_LIN(D_KD), kd1 = PES_LIN(D_KD + 5);
#undef PES_LIN
    const double kn2 = -(kn0 + kn1), np2 = -(np0 + np1), nq2 = -(nq0 + nq1);
    const double kR = fma(wd[D_KR], ca, wd[D_KR + 1] * sa);
    // mode phase plus the Roemer delay of the centre: E = e^{-2 pi i (phase + f k.R)}
    double sp, cp;
    sincos_cycles(fma(b.f, kR, phase), sp, cp);
    const double Er = cp, Ei = -sp;
    // per-arm phase e^{+i pi f k.Delta_t} of the spacecraft opposite arm t
    double s0, c0, s1, c1;
    if (LONG_SINC) {
      sincos_cycles(half_f * kd0, s0, c0);
      sincos_cycles(half_f * kd1, s1, c1);
    } else {  // |pi f k.Delta| <= pi f L / sqrt3 < 0.7 whenever the short sinc fit applies
      sincos_small(pi_f * kd0, s0, c0);
      sincos_small(pi_f * kd1, s1, c1);
    }
    const double c2 = fma(c0, c1, -s0 * s1), s2 = -fma(s0, c1, c0 * s1);

#define PES_ARM(er, ei, np, nq, kn, FR, FI, BR, BI)                    \
  {                                                                   \
    const double Qr = fma(Er, er, -Ei * ei), Qi = fma(Er, ei, Ei * er); \
    const double Pr = aP * fma(np, np, -nq * nq), Pi = aC * 2.0 * np * nq; \
    const double Gr = fma(Qr, Pr, -Qi * Pi), Gi = fma(Qr, Pi, Qi * Pr); \
    const double sf = sinc<LONG_SINC>(a * (1.0 - kn)), sb = sinc<LONG_SINC>(a * (1.0 + kn)); \
    FR = fma(sf, Gr, FR);                                             \
    FI = fma(sf, Gi, FI);                                             \
    BR = fma(sb, Gr, BR);                                             \
    BI = fma(sb, Gi, BI);                                             \
  }
    PES_ARM(c0, s0, np0, nq0, kn0, yFr0, yFi0, yBr0, yBi0)
    PES_ARM(c1, s1, np1, nq1, kn1, yFr1, yFi1, yBr1, yBi1)
    PES_ARM(c2, s2, np2, nq2, kn2, yFr2, yFi2, yBr2, yBi2)
#undef PES_ARM
  }
  // links: arm 0 carries y32 (F) / y23 (B), arm 1 y13 / y31, arm 2 y21 / y12.
  // X = y13 - y12 + z (y31 - y21), Y = y21 - y23 + z (y12 - y32),
  // Z = y32 - y31 + z (y23 - y13)   (the common factor G is in the tables)
  const double xr1 = yBr1 - yFr2, xi1 = yBi1 - yFi2;
  const double Xr = yFr1 - yBr2 + (zr * xr1 - zi * xi1);
  const double Xi = yFi1 - yBi2 + (zr * xi1 + zi * xr1);
  const double yr1 = yBr2 - yFr0, yi1 = yBi2 - yFi0;
  const double Yr = yFr2 - yBr0 + (zr * yr1 - zi * yi1);
  const double Yi = yFi2 - yBi0 + (zr * yi1 + zi * yr1);
  const double zr1 = yBr0 - yFr1, zi1 = yBi0 - yFi1;
  const double Zr = yFr0 - yBr1 + (zr * zr1 - zi * zi1);
  const double Zi = yFi0 - yBi1 + (zr * zi1 + zi * zr1);
  Chan c;
  c.ar = Zr - Xr;
  c.ai = Zi - Xi;
  c.er = Xr - 2.0 * Yr + Zr;
  c.ei = Xi - 2.0 * Yi + Zi;
  c.tr = Xr + Yr + Zr;
  c.ti = Xi + Yi + Zi;
  return c;
}

}  // namespace pes
