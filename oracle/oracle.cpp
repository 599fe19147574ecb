// TEST INFRASTRUCTURE ONLY -- the oracle.
//
// A plain, slow, obviously-correct CPU implementation of what the GPU path
// computes: for a parameter sample theta and every frequency bin, the
// per-(l,m) mode amplitude and phase, the time-frequency map t_f, the analytic
// spacecraft orbits at t_f, the six single-link transfer functions, TDI
// X/Y/Z -> A/E/T, and the noise-weighted Whittle log-likelihood.
//
// Everything is written out in the order and notation of arXiv:2602.12011:
//   Sec. 2.1  eq. (eq_tf) t_f, eq. (eq_fd_resp) link response, the FD TDI
//             combinations, the A/E/T channels;
//   Sec. 2.2  eq. (eq_ll_fd) likelihood, the joint likelihood over channels
//             and detectors, eq. (eq_inner_product), the Fisher matrix.
// Where the paper does not fix a model ingredient (waveform coefficients,
// orbit formulas, PSD shape) a stated stand-in is used; each function says so.
//
// No blocking, fusion or reordering beyond the definitions.  The scalar type is
// a template parameter: double (the default), long double (a rounding-floor
// reference) and Dual<11> (exact forward-mode derivatives for the gradient and
// the Fisher matrix).  The likelihood is the residual form summed over every
// bin, -1/2 sum 4 df |d - h|^2 / S.
//
// Parity unpinned (shared stated conventions, nothing in the paper to check
// them against): the literature values of the leading mode factors |H_lm| and
// their arguments, the constant part of psi_5 (a constant phase), the quintic
// shape of the taper between its C^2 joins, the PSD shaping functions, the
// TianQin plane orientation.  The phase coefficients, the SPA mode and
// polarization construction and the taper joins are pinned by the tests.

#include "oracle.h"

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace orc {

// ---------------------------------------------------------------- constants
// Physical constants (SI; the solar mass as G M_sun / c^3 in seconds).
constexpr long double kPi = 3.141592653589793238462643383279502884L;
constexpr long double kC = 299792458.0L;
constexpr long double kAU = 149597870700.0L;
constexpr long double kYear = 31557600.0L;                 // Julian year [s]
constexpr long double kMsunS = 4.925490947641267e-6L;      // G M_sun / c^3 [s]
constexpr long double kGpc = 3.085677581491367e25L;        // [m]
constexpr long double kEulerGamma = 0.5772156649015328606065120900824024L;
// Inspiral termination of the stand-in: the Schwarzschild ISCO, M f = 6^{-3/2}/pi.
constexpr long double kMfIsco = 0.06804138174397716939909063256727L / kPi;

// ---------------------------------------------------------------- dual numbers
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
};
template <int N> inline Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v + b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v - b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r;
}
template <int N> inline Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r(-a.v); for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r;
}
template <int N> inline Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v * b.v); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r;
}
template <int N> inline Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r(a.v / b.v);
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
template <int N> inline Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> inline Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> inline Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> inline Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> inline Dual<N> operator*(const Dual<N>& a, double b) {
  Dual<N> r(a.v * b); for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b; return r;
}
template <int N> inline Dual<N> operator*(double a, const Dual<N>& b) { return b * a; }
template <int N> inline Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> inline Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> inline Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }
template <int N> inline Dual<N> chain(const Dual<N>& a, double fv, double dfdv) {
  Dual<N> r(fv); for (int i = 0; i < N; ++i) r.d[i] = dfdv * a.d[i]; return r;
}
template <int N> inline Dual<N> sin(const Dual<N>& a) { return chain(a, std::sin(a.v), std::cos(a.v)); }
template <int N> inline Dual<N> cos(const Dual<N>& a) { return chain(a, std::cos(a.v), -std::sin(a.v)); }
template <int N> inline Dual<N> exp(const Dual<N>& a) { double e = std::exp(a.v); return chain(a, e, e); }
template <int N> inline Dual<N> log(const Dual<N>& a) { return chain(a, std::log(a.v), 1.0 / a.v); }
template <int N> inline Dual<N> sqrt(const Dual<N>& a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
template <int N> inline Dual<N> cbrt(const Dual<N>& a) {
  double c = std::cbrt(a.v); return chain(a, c, 1.0 / (3.0 * c * c));
}
template <int N> inline Dual<N> pow(const Dual<N>& a, double p) {
  return chain(a, std::pow(a.v, p), p * std::pow(a.v, p - 1.0));
}

inline double val(double x) { return x; }
inline long double val(long double x) { return x; }
template <int N> inline double val(const Dual<N>& x) { return x.v; }

// Conversion of a long double constant into the working scalar.
template <class T> inline T K(long double x) { return T(x); }
template <> inline double K<double>(long double x) { return (double)x; }
template <> inline Dual<11> K<Dual<11>>(long double x) { return Dual<11>((double)x); }

// ---------------------------------------------------------------- complex
template <class T>
struct Cx {
  T re, im;
  Cx() : re(K<T>(0)), im(K<T>(0)) {}
  Cx(T r, T i) : re(r), im(i) {}
};
template <class T> inline Cx<T> operator+(const Cx<T>& a, const Cx<T>& b) { return Cx<T>(a.re + b.re, a.im + b.im); }
template <class T> inline Cx<T> operator-(const Cx<T>& a, const Cx<T>& b) { return Cx<T>(a.re - b.re, a.im - b.im); }
template <class T> inline Cx<T> operator*(const Cx<T>& a, const Cx<T>& b) {
  return Cx<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <class T> inline Cx<T> operator*(const T& s, const Cx<T>& a) { return Cx<T>(s * a.re, s * a.im); }
template <class T> inline Cx<T> conj(const Cx<T>& a) { return Cx<T>(a.re, -a.im); }
template <class T> inline T norm2(const Cx<T>& a) { return a.re * a.re + a.im * a.im; }
// e^{i x}
template <class T> inline Cx<T> expi(const T& x) { using std::cos; using std::sin; return Cx<T>(cos(x), sin(x)); }

// ---------------------------------------------------------------- source
// Parameter order: [M_tot, q, chi1, chi2, D_L, iota, phi_c, lambda, beta, psi, t_c].
template <class T>
struct Source {
  bool valid;
  T M;            // total mass [s]
  T eta, delta;   // symmetric mass ratio, (m1 - m2)/M
  T DL;           // luminosity distance [s]
  T iota, phic, tc;
  T psi[8];       // PN phase coefficients psi_k (constant part)
  T psil[8];      // coefficient of ln v inside psi_k
  T k[3];         // propagation direction
  T ep[3][3], ec[3][3];  // polarization tensors e_+, e_x
};

// TaylorF2 stand-in for the mode phase (the paper uses PhenomXAS/XHM, whose
// coefficients it does not print): 3.5PN non-spinning phase, 1.5PN spin-orbit
// and 2PN spin-spin terms for aligned spins.
template <class T>
void pn_coefficients(Source<T>& s, const T& chi1, const T& chi2) {
  using std::log;
  const T eta = s.eta, delta = s.delta;
  const T chis = K<T>(0.5L) * (chi1 + chi2);
  const T chia = K<T>(0.5L) * (chi1 - chi2);
  const T pi = K<T>(kPi);
  for (int i = 0; i < 8; ++i) { s.psi[i] = K<T>(0); s.psil[i] = K<T>(0); }
  s.psi[0] = K<T>(1);
  s.psi[2] = K<T>(3715.0L / 756.0L) + K<T>(55.0L / 9.0L) * eta;
  s.psi[3] = K<T>(-16.0L) * pi + (K<T>(113.0L / 3.0L) - K<T>(76.0L / 3.0L) * eta) * chis +
             K<T>(113.0L / 3.0L) * delta * chia;
  s.psi[4] = K<T>(15293365.0L / 508032.0L) + K<T>(27145.0L / 504.0L) * eta +
             K<T>(3085.0L / 72.0L) * eta * eta - K<T>(10.0L * 79.0L / 8.0L) * eta * chi1 * chi2;
  const T c5 = pi * (K<T>(38645.0L / 756.0L) - K<T>(65.0L / 9.0L) * eta);
  s.psi[5] = c5;
  s.psil[5] = K<T>(3) * c5;
  s.psi[6] = K<T>(11583231236531.0L / 4694215680.0L) - K<T>(640.0L / 3.0L * kPi * kPi) -
             K<T>(6848.0L / 21.0L * kEulerGamma) - K<T>(6848.0L / 21.0L * logl(4.0L)) +
             (K<T>(-15737765635.0L / 3048192.0L) + K<T>(2255.0L / 12.0L * kPi * kPi)) * eta +
             K<T>(76055.0L / 1728.0L) * eta * eta - K<T>(127825.0L / 1296.0L) * eta * eta * eta;
  s.psil[6] = K<T>(-6848.0L / 21.0L);
  s.psi[7] = pi * (K<T>(77096675.0L / 254016.0L) + K<T>(378515.0L / 1512.0L) * eta -
                   K<T>(74045.0L / 756.0L) * eta * eta);
}

// Sky basis: source direction nhat(lambda, beta) in ecliptic coordinates,
// propagation k = -nhat, polarization axes p, q rotated by psi from the
// (lambda, beta) tangent vectors; e_+ = pp - qq, e_x = pq + qp.
template <class T>
void sky_basis(const T& lam, const T& beta, const T& psi, T k[3], T ep[3][3], T ec[3][3]) {
  using std::cos; using std::sin;
  const T cl = cos(lam), sl = sin(lam), cb = cos(beta), sb = sin(beta);
  const T cp = cos(psi), sp = sin(psi);
  const T nh[3] = {cb * cl, cb * sl, sb};
  const T u[3] = {-sl, cl, K<T>(0)};
  const T w[3] = {-sb * cl, -sb * sl, cb};
  T p[3], q[3];
  for (int i = 0; i < 3; ++i) {
    k[i] = -nh[i];
    p[i] = cp * u[i] + sp * w[i];
    q[i] = -sp * u[i] + cp * w[i];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      ep[i][j] = p[i] * p[j] - q[i] * q[j];
      ec[i][j] = p[i] * q[j] + q[i] * p[j];
    }
}

template <class T>
bool make_source(const T* th, Source<T>& s) {
  const double M = val(th[0]), q = val(th[1]), c1 = val(th[2]), c2 = val(th[3]), D = val(th[4]);
  bool ok = true;
  for (int i = 0; i < 11; ++i) ok = ok && std::isfinite((double)val(th[i]));
  ok = ok && M > 0 && q > 0 && q <= 1 && std::fabs(c1) < 1 && std::fabs(c2) < 1 && D > 0;
  s.valid = ok;
  if (!ok) return false;
  const T one = K<T>(1);
  s.M = th[0] * K<T>(kMsunS);
  s.eta = th[1] / ((one + th[1]) * (one + th[1]));
  s.delta = (one - th[1]) / (one + th[1]);
  s.DL = th[4] * K<T>(kGpc / kC);
  s.iota = th[5];
  s.phic = th[6];
  s.tc = th[10];
  pn_coefficients(s, th[2], th[3]);
  sky_basis(th[7], th[8], th[9], s.k, s.ep, s.ec);
  return true;
}

// ---------------------------------------------------------------- harmonics
inline long double factl(int n) { long double r = 1; for (int i = 2; i <= n; ++i) r *= i; return r; }

// Spin-weight -2 spherical harmonic at azimuth 0 through the Wigner d-matrix
// sum: -2Y_lm(i, 0) = sqrt((2l+1)/(4 pi)) d^l_{m,2}(i).
template <class T>
T ylm(int l, int m, const T& iota) {
  using std::cos; using std::sin; using std::pow;
  const T c = cos(iota * K<T>(0.5L)), s = sin(iota * K<T>(0.5L));
  const int kmin = (m - 2 > 0) ? m - 2 : 0;
  const int kmax = (l + m < l - 2) ? l + m : l - 2;
  T d = K<T>(0);
  for (int k = kmin; k <= kmax; ++k) {
    const long double num = sqrtl(factl(l + m) * factl(l - m) * factl(l + 2) * factl(l - 2));
    const long double den = factl(l + m - k) * factl(l - 2 - k) * factl(k) * factl(k + 2 - m);
    const long double sign = (k % 2) ? -1.0L : 1.0L;
    T term = K<T>(sign * num / den);
    const int pc = 2 * l + m - 2 - 2 * k, ps = 2 * k + 2 - m;
    for (int i = 0; i < pc; ++i) term = term * c;
    for (int i = 0; i < ps; ++i) term = term * s;
    d = d + term;
  }
  return K<T>(sqrtl((2.0L * l + 1.0L) / (4.0L * kPi))) * d;
}

// Plus/cross projections of mode h_{l,-m} (positive frequencies), from
// h_+ - i h_x = sum_lm h_lm Y_lm and h_{l,-m} = (-1)^l conj(h_lm):
//   h_+ = 1/2 [Y_{l,-m} + (-1)^l Y_lm] h_{l,-m},  h_x = i/2 [Y_{l,-m} - (-1)^l Y_lm] h_{l,-m}.
template <class T>
void pol_coeffs(int l, int m, const T& iota, Cx<T>& Kp, Cx<T>& Kc) {
  const T ym = ylm<T>(l, -m, iota), yp = ylm<T>(l, m, iota);
  const T sgn = K<T>((l % 2) ? -1.0L : 1.0L);
  Kp = Cx<T>(K<T>(0.5L) * (ym + sgn * yp), K<T>(0));
  Kc = Cx<T>(K<T>(0), K<T>(0.5L) * (ym - sgn * yp));
}

// ---------------------------------------------------------------- waveform modes
// |H_lm(v)| of the leading post-Newtonian mode amplitudes, and the constant
// phase of h_{l,-m} = (-1)^l conj(H_lm) / |H_lm| (H21 ~ i, H33 ~ -i, H32 ~ 1, H44 ~ -1).
template <class T>
T mode_hmag(int l, int m, const Source<T>& s, const T& v) {
  const T one = K<T>(1);
  if (l == 2 && m == 2) return one;
  if (l == 2 && m == 1) return s.delta * v / K<T>(3);
  if (l == 3 && m == 3) return K<T>(0.75L * sqrtl(15.0L / 14.0L)) * s.delta * v;
  if (l == 3 && m == 2) return K<T>(sqrtl(5.0L / 7.0L) / 3.0L) * (one - K<T>(3) * s.eta) * v * v;
  if (l == 4 && m == 4) return K<T>(8.0L / 9.0L * sqrtl(5.0L / 7.0L)) * (one - K<T>(3) * s.eta) * v * v;
  return K<T>(0);
}
inline void mode_unit(int l, int m, long double& re, long double& im) {
  re = 1; im = 0;
  if (l == 2 && m == 1) { re = 0; im = -1; }
  if (l == 3 && m == 3) { re = 0; im = -1; }
  if (l == 3 && m == 2) { re = -1; im = 0; }
  if (l == 4 && m == 4) { re = -1; im = 0; }
}

// C^2 termination taper on x = f / f_cut: 1 below 0.9, 0 above 1.
template <class T>
T taper(const T& x) {
  if (val(x) <= 0.9) return K<T>(1);
  if (val(x) >= 1.0) return K<T>(0);
  const T u = (x - K<T>(0.9L)) / K<T>(0.1L);
  return K<T>(1) - u * u * u * (K<T>(10) - K<T>(15) * u + K<T>(6) * u * u);
}

template <class T>
struct ModeVal {
  bool on;
  Cx<T> h;   // h_{l,-m}(f)
  T Psi;     // h = |h| * unit_lm * e^{-i Psi}
  T tf;      // t_f^{lm}(f), eq. (eq_tf)
};

// One SPA mode of the stand-in at frequency f.  The mode phase follows the
// SPA scaling of the 22 phase, Psi_lm(f) = 2 pi f t_c - (m/2) phi_c - pi/4 +
// (m/2) Psibar(v_lm), v_lm = (2 pi M f / m)^{1/3}, with the TaylorF2
// Psibar(v) = 3/(128 eta v^5) sum_k psi_k v^k.  The paper's phase is Phi = -Psi,
// so eq. (eq_tf) t_f = -(1/2pi) dPhi/df = (1/2pi) dPsi/df, written out in
// closed form from the same series.
template <class T>
ModeVal<T> mode_eval(const Source<T>& s, int l, int m, const T& f) {
  using std::cbrt; using std::log; using std::sqrt; using std::pow;
  ModeVal<T> r;
  const T mm = K<T>(m);
  const T fcut = (mm / K<T>(2)) * K<T>(kMfIsco) / s.M;
  const T x = f / fcut;
  r.on = val(x) < 1.0;
  if (!r.on) return r;
  const T pi = K<T>(kPi);
  const T v = cbrt(K<T>(2) * pi * s.M * f / mm);
  const T lnv = log(v);
  T vk = K<T>(1), sph = K<T>(0), stf = K<T>(0);
  for (int k = 0; k < 8; ++k) {
    const T g = s.psi[k] + s.psil[k] * lnv;
    sph = sph + g * vk;
    stf = stf + (K<T>(k - 5) * g + s.psil[k]) * vk;
    vk = vk * v;
  }
  const T v2 = v * v, v4 = v2 * v2, v5 = v4 * v, v8 = v4 * v4;
  const T Psibar = K<T>(3) / (K<T>(128) * s.eta * v5) * sph;
  r.Psi = K<T>(2) * pi * f * s.tc - (mm / K<T>(2)) * s.phic - pi / K<T>(4) +
          (mm / K<T>(2)) * Psibar;
  r.tf = s.tc + s.M / (K<T>(256) * s.eta * v8) * stf;
  const T amp = sqrt(K<T>(2) / mm) * pi * sqrt(K<T>(2) * s.eta / K<T>(3)) * s.M * s.M *
                pow(v, -3.5) * mode_hmag(l, m, s, v) / s.DL;
  const T W = taper(x);
  long double ure, uim;
  mode_unit(l, m, ure, uim);
  const Cx<T> unit(K<T>(ure), K<T>(uim));
  r.h = (W * amp) * (unit * expi(-r.Psi));
  return r;
}

// ---------------------------------------------------------------- orbits
// Analytic orbits (the paper names the Keplerian heliocentric orbits for LISA
// and Taiji and the Keplerian geocentric orbit for TianQin without printing
// them).  Heliocentric: the first-order-in-eccentricity Keplerian orbit of
// three spacecraft, e = L/(2 sqrt(3) AU), guiding centre at 1 AU with
// revolution phase alpha = 2 pi t / yr + phase0; this triangle is exactly
// equilateral with side L.  With orbit = 1 the same three Kepler ellipses
// exactly (the arms then flex at order e^2 AU).  Geocentric: a ring of radius L/sqrt(3) about the
// Earth (circular 1-AU orbit), normal to (tq_lon, tq_lat), period tq_period_s.
// Output in light-seconds.
template <class T>
void orbit(const or_detector& d, const T& t, T x[3][3]) {
  using std::cos; using std::sin; using std::sqrt;
  const T pi = K<T>(kPi);
  const T alpha = K<T>(2) * pi * t / K<T>(kYear) + K<T>(d.phase0);
  const T AUc = K<T>(kAU / kC);
  if (d.kind == OR_TIANQIN) {
    const long double lon = d.tq_lon, lat = d.tq_lat;
    const long double nh[3] = {cosl(lat) * cosl(lon), cosl(lat) * sinl(lon), sinl(lat)};
    const long double u[3] = {-sinl(lon), cosl(lon), 0.0L};
    const long double w[3] = {nh[1] * u[2] - nh[2] * u[1], nh[2] * u[0] - nh[0] * u[2],
                              nh[0] * u[1] - nh[1] * u[0]};
    const T R = K<T>((long double)d.arm_m / sqrtl(3.0L) / kC);
    const T phi = K<T>(2) * pi * t / K<T>(d.tq_period_s);
    for (int n = 0; n < 3; ++n) {
      const T ph = phi + K<T>(2.0L * kPi * n / 3.0L);
      const T cph = cos(ph), sph = sin(ph);
      const T RE[3] = {AUc * cos(alpha), AUc * sin(alpha), K<T>(0)};
      for (int i = 0; i < 3; ++i) x[n][i] = RE[i] + R * (cph * K<T>(u[i]) + sph * K<T>(w[i]));
    }
    return;
  }
  const T e = K<T>((long double)d.arm_m / (2.0L * sqrtl(3.0L) * kAU));
  if (d.orbit == 1) {
    // Exact Kepler ellipses with the elements whose first-order expansion in
    // e is the triangle below: semi-major axis 1 AU (period 1 yr), eccentricity
    // e, inclination sin(i) = sqrt(3) e = L / (2 AU), longitude of perihelion
    // b_n = 2 pi n / 3, ascending node b_n + pi/2 (argument of perihelion
    // -pi/2); mean anomaly alpha - b_n.  Kepler's equation E - e sin E = M by
    // Newton's method to the working precision.
    using std::fabs;
    const T si = sqrt(K<T>(3)) * e, ci = sqrt(K<T>(1) - si * si);
    const T sq = sqrt(K<T>(1) - e * e);
    for (int n = 0; n < 3; ++n) {
      const T b = K<T>(2.0L * kPi * n / 3.0L);
      const T M = alpha - b;
      T E = M + e * sin(M);
      for (int it = 0; it < 8; ++it) E = E - (E - e * sin(E) - M) / (K<T>(1) - e * cos(E));
      const T xo = AUc * (cos(E) - e), yo = AUc * sq * sin(E);
      // argument of perihelion -pi/2: (xo, yo) -> (yo, -xo) in the orbital plane
      const T u = yo, v = -xo;
      const T Om = b + K<T>(0.5L * kPi);
      const T cO = cos(Om), sO = sin(Om);
      x[n][0] = u * cO - v * ci * sO;
      x[n][1] = u * sO + v * ci * cO;
      x[n][2] = v * si;
    }
    return;
  }
  for (int n = 0; n < 3; ++n) {
    const T b = K<T>(2.0L * kPi * n / 3.0L);
    x[n][0] = AUc * cos(alpha) + K<T>(0.5L) * e * AUc * (cos(K<T>(2) * alpha - b) - K<T>(3) * cos(b));
    x[n][1] = AUc * sin(alpha) + K<T>(0.5L) * e * AUc * (sin(K<T>(2) * alpha - b) - K<T>(3) * sin(b));
    x[n][2] = -sqrt(K<T>(3)) * e * AUc * cos(alpha - b);
  }
}

// ---------------------------------------------------------------- link + TDI
// eq. (eq_fd_resp): y_rs(f) = -i pi f L sinc[pi f L (1 - k.n_rs)]
//   exp{-i pi f [L + k.(x_r + x_s)]} n_rs . h(f) . n_rs, n_rs = (x_r - x_s)/L,
// added into y[r][s] for every ordered pair r != s.
// With unit = true the link direction is the unit vector of the actual
// separation (exact orbits, whose arms flex); the transfer function keeps the
// nominal L (the paper evaluates the response on the rigid equilateral
// approximation and lets the flexing enter only the laser-noise TDI).
template <class T>
void add_links(const T& f, const T& L, const T k[3], const T x[3][3], const Cx<T> H[3][3],
               Cx<T> y[3][3], bool unit = false) {
  using std::sin; using std::sqrt;
  const T pi = K<T>(kPi);
  for (int r = 0; r < 3; ++r)
    for (int s = 0; s < 3; ++s) {
      if (r == s) continue;
      T n[3];
      T Ln = L;
      if (unit) {
        T d2 = K<T>(0);
        for (int i = 0; i < 3; ++i) d2 = d2 + (x[r][i] - x[s][i]) * (x[r][i] - x[s][i]);
        Ln = sqrt(d2);
      }
      for (int i = 0; i < 3; ++i) n[i] = (x[r][i] - x[s][i]) / Ln;
      T kn = K<T>(0), kx = K<T>(0);
      for (int i = 0; i < 3; ++i) { kn = kn + k[i] * n[i]; kx = kx + k[i] * (x[r][i] + x[s][i]); }
      Cx<T> nhn;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) nhn = nhn + (n[i] * n[j]) * H[i][j];
      const T arg = pi * f * L * (K<T>(1) - kn);
      const T sinc = (val(arg) == 0.0) ? K<T>(1) : sin(arg) / arg;
      const Cx<T> pre(K<T>(0), -(pi * f * L));
      const Cx<T> ph = expi(-(pi * f * (L + kx)));
      y[r][s] = y[r][s] + (pre * (sinc * (ph * nhn)));
    }
}

// FD TDI with the delay factor z = e^{-2 pi i f L}:
//   X_1.5 = (1 - z^2) [y13 - y12 + z (y31 - y21)],  X_2.0 = (1 - z^2 - z^4 + z^6)[...],
// Y, Z by the cyclic permutation 1 -> 2 -> 3 -> 1; then
//   A = (Z - X)/sqrt2, E = (X - 2Y + Z)/sqrt6, T = (X + Y + Z)/sqrt3.
// y indices are 0-based: y[r][s] is y_{r+1, s+1}.
template <class T>
void tdi(const T& f, const T& L, int gen, const Cx<T> y[3][3], Cx<T> xyz[3], Cx<T> aet[3]) {
  const T pi = K<T>(kPi);
  const Cx<T> z = expi(-(K<T>(2) * pi * f * L));
  const Cx<T> one(K<T>(1), K<T>(0));
  const Cx<T> z2 = z * z, z4 = z2 * z2, z6 = z4 * z2;
  const Cx<T> fac = (gen == 15) ? (one - z2) : (one - z2 - z4 + z6);
  for (int c = 0; c < 3; ++c) {
    const int a = c, b = (c + 1) % 3, d = (c + 2) % 3;  // X: (1,2,3) -> indices (0,1,2)
    const Cx<T> inner = y[a][d] - y[a][b] + z * (y[d][a] - y[b][a]);
    xyz[c] = fac * inner;
  }
  const T r2 = K<T>(sqrtl(2.0L)), r6 = K<T>(sqrtl(6.0L)), r3 = K<T>(sqrtl(3.0L));
  aet[0] = (K<T>(1) / r2) * (xyz[2] - xyz[0]);
  aet[1] = (K<T>(1) / r6) * (xyz[0] - K<T>(2) * xyz[1] + xyz[2]);
  aet[2] = (K<T>(1) / r3) * (xyz[0] + xyz[1] + xyz[2]);
}

// ---------------------------------------------------------------- response
// Noise-free A/E/T of one detector at one frequency: every mode (l,m) is
// propagated through its own geometry at t_f^{lm}(f); the six links are summed
// over modes before TDI (TDI is linear).
template <class T>
void response_at(const Source<T>& s, const or_config& cfg, const or_detector& d, const T& f,
                 Cx<T> aet[3]) {
  const T L = K<T>((long double)d.arm_m / kC);
  Cx<T> y[3][3];
  for (int im = 0; im < cfg.n_modes; ++im) {
    const int l = cfg.modes[im][0], m = cfg.modes[im][1];
    const ModeVal<T> mv = mode_eval(s, l, m, f);
    if (!mv.on) continue;
    Cx<T> Kp, Kc;
    pol_coeffs(l, m, s.iota, Kp, Kc);
    const Cx<T> hp = Kp * mv.h, hc = Kc * mv.h;
    Cx<T> H[3][3];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) H[i][j] = s.ep[i][j] * hp + s.ec[i][j] * hc;
    T x[3][3];
    orbit(d, mv.tf, x);
    add_links(f, L, s.k, x, H, y, d.kind != OR_TIANQIN && d.orbit == 1);
  }
  Cx<T> xyz[3];
  tdi(f, L, d.tdi_gen, y, xyz, aet);
}

// ---------------------------------------------------------------- PSD
// Noise model (fractional frequency): every link y_rs carries an independent
// optical-metrology noise n_rs and the test-mass noise of both ends,
// y_rs += delta_rs + z delta_sr.  The channel PSD is the plain propagation of
// the twelve independent sources through the same TDI map,
// S_c = sum_j |dC/dn_j|^2 S_j.  Single-link PSDs use the LISA-like budget with
// the stated amplitudes: S_oms = a_oms^2 (1 + (2 mHz/f)^4) (2 pi f/c)^2 and
// S_acc = a_acc^2 (1 + (0.4 mHz/f)^2)(1 + (f/8 mHz)^4) / (2 pi f c)^2.
template <class T>
void psd_at(const or_detector& d, const T& f, T& S_a, T& S_e, T& S_t) {
  using std::pow;
  const T pi = K<T>(kPi), c = K<T>(kC);
  const T L = K<T>((long double)d.arm_m / kC);
  const T two_pi_f = K<T>(2) * pi * f;
  const T r1 = K<T>(2e-3L) / f, r2 = K<T>(4e-4L) / f, r3 = f / K<T>(8e-3L);
  const T S_oms = K<T>((long double)d.oms_asd * d.oms_asd) * (K<T>(1) + r1 * r1 * r1 * r1) *
                  (two_pi_f / c) * (two_pi_f / c);
  const T S_acc = K<T>((long double)d.acc_asd * d.acc_asd) * (K<T>(1) + r2 * r2) *
                  (K<T>(1) + r3 * r3 * r3 * r3) / ((two_pi_f * c) * (two_pi_f * c));
  const Cx<T> z = expi(-(K<T>(2) * pi * f * L));
  T acc[3] = {K<T>(0), K<T>(0), K<T>(0)};
  for (int src = 0; src < 12; ++src) {
    Cx<T> y[3][3];
    int idx = 0;
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) {
        if (r == s) continue;
        if (src < 6) {
          if (idx == src) y[r][s] = Cx<T>(K<T>(1), K<T>(0));  // OMS n_rs
        } else {
          if (idx == src - 6) {                            // test mass delta_rs
            y[r][s] = y[r][s] + Cx<T>(K<T>(1), K<T>(0));   // enters y_rs directly
            y[s][r] = y[s][r] + z;                         // and y_sr delayed
          }
        }
        ++idx;
      }
    Cx<T> xyz[3], aet[3];
    tdi(f, L, d.tdi_gen, y, xyz, aet);
    const T Sj = (src < 6) ? S_oms : S_acc;
    for (int ch = 0; ch < 3; ++ch) acc[ch] = acc[ch] + norm2(aet[ch]) * Sj;
  }
  S_a = acc[0];
  S_e = acc[1];
  S_t = acc[2];
}

// The likelihood uses the A channel's PSD for both A and E (equal by symmetry
// of the noise model; the tests check S_A = S_E).
template <class T>
void psd_at(const or_detector& d, const T& f, T& S_ae, T& S_t) {
  T S_e;
  psd_at(d, f, S_ae, S_e, S_t);
}

// ---------------------------------------------------------------- likelihood
template <class T, class Fl>
T loglike_one(const or_config& cfg, const double* data, const T* th) {
  Source<T> s;
  if (!make_source(th, s)) return K<T>(-INFINITY);
  T sum = K<T>(0);
  const int64_t N = cfg.n_bins;
  for (int id = 0; id < cfg.n_det; ++id) {
    const or_detector& d = cfg.det[id];
    for (int64_t kb = 0; kb < N; ++kb) {
      const Fl fl = (Fl)cfg.f0 + (Fl)kb * (Fl)cfg.df;
      const T f = K<T>(fl);
      Cx<T> h[3];
      response_at(s, cfg, d, f, h);
      T Sae, St;
      psd_at(d, f, Sae, St);
      for (int c = 0; c < 3; ++c) {
        const T S = (c == 2) ? St : Sae;
        if (val(S) == 0.0) continue;
        const double* dp = data + 2 * ((id * 3 + c) * N + kb);
        const Cx<T> r = Cx<T>(K<T>(dp[0]), K<T>(dp[1])) - h[c];
        // eq. (eq_ll_fd): -2 |d - h|^2 / (S T) with 1/T = df
        sum = sum + K<T>(4) * K<T>((long double)cfg.df) * norm2(r) / S;
      }
    }
  }
  return K<T>(-0.5L) * sum;
}

inline int threads(int n) {
#ifdef _OPENMP
  return n > 0 ? n : omp_get_max_threads();
#else
  (void)n; return 1;
#endif
}

bool config_ok(const or_config* cfg) {
  if (!cfg || cfg->n_det < 1 || cfg->n_det > 3 || cfg->n_bins < 0 || cfg->n_modes < 1 ||
      cfg->n_modes > 5)
    return false;
  for (int i = 0; i < cfg->n_modes; ++i) {
    const int l = cfg->modes[i][0], m = cfg->modes[i][1];
    const bool known = (l == 2 && (m == 2 || m == 1)) || (l == 3 && (m == 3 || m == 2)) ||
                       (l == 4 && m == 4);
    if (!known) return false;
  }
  for (int i = 0; i < cfg->n_det; ++i) {
    const or_detector& d = cfg->det[i];
    if (d.tdi_gen != 15 && d.tdi_gen != 20) return false;
    if (d.kind < 0 || d.kind > 2 || !(d.arm_m > 0)) return false;
  }
  return true;
}

}  // namespace orc

using namespace orc;
typedef Dual<11> D11;

extern "C" {

int or_loglike(const or_config* cfg, const double* data, const double* theta, int64_t B,
               int prec, int nthreads, double* logl) {
  if (!config_ok(cfg) || B < 0 || !theta || !logl || (!data && cfg->n_bins > 0)) return -1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads(nthreads))
  for (int64_t b = 0; b < B; ++b) {
    if (prec == 1) {
      long double th[11];
      for (int i = 0; i < 11; ++i) th[i] = theta[11 * b + i];
      logl[b] = (double)loglike_one<long double, long double>(*cfg, data, th);
    } else {
      logl[b] = loglike_one<double, double>(*cfg, data, theta + 11 * b);
    }
  }
  return 0;
}

int or_grad(const or_config* cfg, const double* data, const double* theta, int64_t B,
            int nthreads, double* logl, double* grad) {
  if (!config_ok(cfg) || B < 0 || !theta || !logl || !grad) return -1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads(nthreads))
  for (int64_t b = 0; b < B; ++b) {
    D11 th[11];
    for (int i = 0; i < 11; ++i) { th[i] = D11(theta[11 * b + i]); th[i].d[i] = 1.0; }
    const D11 L = loglike_one<D11, double>(*cfg, data, th);
    logl[b] = L.v;
    for (int i = 0; i < 11; ++i) grad[11 * b + i] = std::isfinite(L.v) ? L.d[i] : 0.0;
  }
  return 0;
}

int or_fisher(const or_config* cfg, const double* theta, int64_t B, int nthreads, double* F) {
  if (!config_ok(cfg) || B < 0 || !theta || !F) return -1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads(nthreads))
  for (int64_t b = 0; b < B; ++b) {
    double* Fb = F + 121 * b;
    for (int i = 0; i < 121; ++i) Fb[i] = 0.0;
    D11 th[11];
    for (int i = 0; i < 11; ++i) { th[i] = D11(theta[11 * b + i]); th[i].d[i] = 1.0; }
    Source<D11> s;
    if (!make_source(th, s)) { for (int i = 0; i < 121; ++i) Fb[i] = NAN; continue; }
    for (int id = 0; id < cfg->n_det; ++id) {
      const or_detector& d = cfg->det[id];
      for (int64_t kb = 0; kb < cfg->n_bins; ++kb) {
        const double f = cfg->f0 + (double)kb * cfg->df;
        Cx<D11> h[3];
        response_at(s, *cfg, d, D11(f), h);
        double Sae, St;
        psd_at(d, f, Sae, St);
        for (int c = 0; c < 3; ++c) {
          const double S = (c == 2) ? St : Sae;
          if (S == 0.0) continue;
          const double w = 4.0 * cfg->df / S;
          // eq. (eq_inner_product) applied to the partial derivatives of h
          for (int i = 0; i < 11; ++i)
            for (int j = 0; j < 11; ++j)
              Fb[11 * i + j] += w * (h[c].re.d[i] * h[c].re.d[j] + h[c].im.d[i] * h[c].im.d[j]);
        }
      }
    }
  }
  return 0;
}

int or_response(const or_config* cfg, const double* theta, int prec, double* aet) {
  if (!config_ok(cfg) || !theta || !aet) return -1;
  const int64_t N = cfg->n_bins;
  if (prec == 1) {
    long double th[11];
    for (int i = 0; i < 11; ++i) th[i] = theta[i];
    Source<long double> s;
    if (!make_source(th, s)) return -2;
    for (int id = 0; id < cfg->n_det; ++id)
      for (int64_t kb = 0; kb < N; ++kb) {
        const long double f = (long double)cfg->f0 + (long double)kb * (long double)cfg->df;
        Cx<long double> h[3];
        response_at(s, *cfg, cfg->det[id], f, h);
        for (int c = 0; c < 3; ++c) {
          aet[2 * ((id * 3 + c) * N + kb)] = (double)h[c].re;
          aet[2 * ((id * 3 + c) * N + kb) + 1] = (double)h[c].im;
        }
      }
    return 0;
  }
  Source<double> s;
  if (!make_source(theta, s)) return -2;
  for (int id = 0; id < cfg->n_det; ++id)
    for (int64_t kb = 0; kb < N; ++kb) {
      const double f = cfg->f0 + (double)kb * cfg->df;
      Cx<double> h[3];
      response_at(s, *cfg, cfg->det[id], f, h);
      for (int c = 0; c < 3; ++c) {
        aet[2 * ((id * 3 + c) * N + kb)] = h[c].re;
        aet[2 * ((id * 3 + c) * N + kb) + 1] = h[c].im;
      }
    }
  return 0;
}

double or_inner(const or_config* cfg, const double* a, const double* b) {
  if (!config_ok(cfg)) return NAN;
  const int64_t N = cfg->n_bins;
  double sum = 0.0;
  for (int id = 0; id < cfg->n_det; ++id)
    for (int64_t kb = 0; kb < N; ++kb) {
      const double f = cfg->f0 + (double)kb * cfg->df;
      double Sae, St;
      psd_at(cfg->det[id], f, Sae, St);
      for (int c = 0; c < 3; ++c) {
        const double S = (c == 2) ? St : Sae;
        if (S == 0.0) continue;
        const int64_t o = 2 * ((id * 3 + c) * N + kb);
        // eq. (eq_inner_product): 4 Re sum a* b / (S T), 1/T = df
        sum += 4.0 * cfg->df * (a[o] * b[o] + a[o + 1] * b[o + 1]) / S;
      }
    }
  return sum;
}

int or_psd(const or_detector* det, const double* f, int64_t n, double* S) {
  if (!det || !f || !S || n < 0) return -1;
  for (int64_t i = 0; i < n; ++i) psd_at(*det, f[i], S[3 * i], S[3 * i + 1], S[3 * i + 2]);
  return 0;
}

int or_orbit(const or_detector* det, double t, double* x) {
  if (!det) return -1;
  double xx[3][3];
  orbit(*det, t, xx);
  std::memcpy(x, xx, sizeof(xx));
  return 0;
}

int or_link_fd(double f, double L_s, const double* k, const double* x, const double* H,
               double* y, int unit) {
  if (unit != 0 && unit != 1) return -1;
  double kk[3] = {k[0], k[1], k[2]};
  double xx[3][3];
  std::memcpy(xx, x, sizeof(xx));
  Cx<double> HH[3][3], yy[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) HH[i][j] = Cx<double>(H[2 * (3 * i + j)], H[2 * (3 * i + j) + 1]);
  add_links(f, L_s, kk, xx, HH, yy, unit == 1);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) { y[2 * (3 * i + j)] = yy[i][j].re; y[2 * (3 * i + j) + 1] = yy[i][j].im; }
  return 0;
}

int or_tdi(double f, double L_s, int gen, const double* y, double* xyz, double* aet) {
  if (gen != 15 && gen != 20) return -1;
  Cx<double> yy[3][3], X[3], A[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) yy[i][j] = Cx<double>(y[2 * (3 * i + j)], y[2 * (3 * i + j) + 1]);
  tdi(f, L_s, gen, yy, X, A);
  for (int c = 0; c < 3; ++c) {
    xyz[2 * c] = X[c].re; xyz[2 * c + 1] = X[c].im;
    aet[2 * c] = A[c].re; aet[2 * c + 1] = A[c].im;
  }
  return 0;
}

double or_ylm(int l, int m, double iota) { return ylm<double>(l, m, iota); }

int or_pol_coeffs(int l, int m, double iota, double* Kp, double* Kc) {
  Cx<double> a, b;
  pol_coeffs(l, m, iota, a, b);
  Kp[0] = a.re; Kp[1] = a.im; Kc[0] = b.re; Kc[1] = b.im;
  return 0;
}

int or_mode(const double* theta, int l, int m, const double* f, int64_t n, double* h,
            double* psi, double* tf) {
  Source<double> s;
  if (!make_source(theta, s)) return -2;
  for (int64_t i = 0; i < n; ++i) {
    const ModeVal<double> mv = mode_eval(s, l, m, f[i]);
    h[2 * i] = mv.on ? mv.h.re : 0.0;
    h[2 * i + 1] = mv.on ? mv.h.im : 0.0;
    psi[i] = mv.on ? mv.Psi : NAN;
    tf[i] = mv.on ? mv.tf : NAN;
  }
  return 0;
}

int or_sky_basis(double lambda, double beta, double psi, double* k, double* ep, double* ec) {
  double kk[3], e1[3][3], e2[3][3];
  sky_basis(lambda, beta, psi, kk, e1, e2);
  std::memcpy(k, kk, sizeof(kk));
  std::memcpy(ep, e1, sizeof(e1));
  std::memcpy(ec, e2, sizeof(e2));
  return 0;
}

}  // extern "C"
