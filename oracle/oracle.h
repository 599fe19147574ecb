/*
 * TEST INFRASTRUCTURE ONLY -- the oracle.
 *
 * Plain, slow CPU reference for the batched frequency-domain response and
 * Whittle likelihood of massive-black-hole-binary signals in LISA-, Taiji- and
 * TianQin-like detectors (arXiv:2602.12011, Sec. 2.1 "Response model" and
 * Sec. 2.2 "Parameter estimation").  Only the test-suite, the smoke check and
 * the benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library; the product path never calls
 * it.
 *
 * All arrays are host memory, owned by the caller.  Complex arrays are
 * interleaved (re, im) doubles.  Functions return 0 on success and a negative
 * value on invalid arguments.
 */
#ifndef PES_ORACLE_H
#define PES_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_LISA = 0, OR_TAIJI = 1, OR_TIANQIN = 2 };

typedef struct {
  int kind;            /* OR_LISA / OR_TAIJI: heliocentric; OR_TIANQIN: geocentric */
  int tdi_gen;         /* 15 or 20 */
  double arm_m;        /* arm length L [m] */
  double phase0;       /* initial revolution phase of the constellation centre [rad] */
  double tq_period_s;  /* TianQin: constellation rotation period [s] */
  double tq_lon;       /* TianQin: ecliptic longitude of the plane normal [rad] */
  double tq_lat;       /* TianQin: ecliptic latitude of the plane normal [rad] */
  double oms_asd;      /* optical-metrology displacement ASD [m/sqrt(Hz)] */
  double acc_asd;      /* test-mass acceleration ASD [m/s^2/sqrt(Hz)] */
  int orbit;           /* heliocentric kinds: 0 first order in eccentricity, 1 exact Kepler ellipses */
} or_detector;

typedef struct {
  int n_det;
  or_detector det[3];
  int64_t n_bins;      /* frequency grid f_k = f0 + k*df, k = 0..n_bins-1 */
  double f0;
  double df;
  int n_modes;
  int modes[5][2];     /* (l, m) from {(2,2),(2,1),(3,3),(3,2),(4,4)} */
} or_config;

/* theta layout, 11 doubles per sample:
   [M_tot (Msun, detector frame), q = m2/m1 in (0,1], chi1, chi2, D_L (Gpc),
    iota, phi_c, lambda, beta, psi, t_c (s from the orbit epoch)] */

/* log L for B samples; prec 0 = double, 1 = long double.  data is
   [n_det][3][n_bins] complex (A, E, T).  nthreads <= 0 means all cores. */
int or_loglike(const or_config* cfg, const double* data, const double* theta,
               int64_t B, int prec, int nthreads, double* logl);

/* log L and its exact gradient (forward-mode dual numbers) w.r.t. theta. */
int or_grad(const or_config* cfg, const double* data, const double* theta,
            int64_t B, int nthreads, double* logl, double* grad);

/* Fisher matrix F_ij = <d_i h | d_j h>, [B][11][11]. */
int or_fisher(const or_config* cfg, const double* theta, int64_t B,
              int nthreads, double* F);

/* Noise-free A/E/T response h(theta): out [n_det][3][n_bins] complex. */
int or_response(const or_config* cfg, const double* theta, int prec, double* aet);

/* <a|b> over all detectors and channels of a config (a, b shaped like data). */
double or_inner(const or_config* cfg, const double* a, const double* b);

/* One-sided PSDs of the A, E and T channels: out [n][3]. */
int or_psd(const or_detector* det, const double* f, int64_t n, double* S);

/* Spacecraft positions at time t [s]: x[3][3] in light-seconds. */
int or_orbit(const or_detector* det, double t, double* x);

/* Six single-link transfer functions for a static geometry.
   k[3]: propagation direction; x[3][3]: spacecraft positions [light-s];
   H[3][3] complex: Fourier-domain strain tensor at f; L_s: arm [s].
   unit = 0: link directions (x_r - x_s) / L_s (the rigid triangle); unit = 1:
   the unit separations (x_r - x_s) / |x_r - x_s| (exact Kepler orbits), the
   transfer function keeping L_s.
   out y[3][3] complex, y[r][s] = link received at r, sent from s (diag 0). */
int or_link_fd(double f, double L_s, const double* k, const double* x,
               const double* H, double* y, int unit);

/* TDI X, Y, Z and A, E, T from the six links y[3][3] (layout as above). */
int or_tdi(double f, double L_s, int gen, const double* y, double* xyz, double* aet);

/* Spin-weight -2 spherical harmonic at phi = 0 (real). */
double or_ylm(int l, int m, double iota);

/* Plus/cross coefficients of mode h_{l,-m}: h_+ = Kp h, h_x = Kc h (complex). */
int or_pol_coeffs(int l, int m, double iota, double* Kp, double* Kc);

/* One waveform mode h_{l,-m}(f) on a list of frequencies: complex h, the
   phase Psi (h = |h| e^{-i Psi} up to the constant mode phase), and t_f. */
int or_mode(const double* theta, int l, int m, const double* f, int64_t n,
            double* h, double* psi, double* tf);

/* Sky basis: k[3], e_plus[3][3], e_cross[3][3]. */
int or_sky_basis(double lambda, double beta, double psi, double* k,
                 double* ep, double* ec);

#ifdef __cplusplus
}
#endif
#endif
