/*
 * libpes -- batched FP64 frequency-domain response and likelihood of
 * massive-black-hole-binary signals in LISA-, Taiji- and TianQin-like
 * detectors on AMD Instinct MI355X (gfx950).
 *
 * The operations follow arXiv:2602.12011:
 *   Sec. 2.1  the single-link response eq. (eq_fd_resp) evaluated at the SPA
 *             time-frequency map eq. (eq_tf), the FD TDI 1.5 / 2.0 combinations
 *             and the A, E, T channels;
 *   Sec. 2.2  the Whittle likelihood eq. (eq_ll_fd), joint over channels and
 *             detectors, the inner product eq. (eq_inner_product) and the
 *             Fisher matrix F_ij = <d_i s | d_j s>.
 * The waveform is a closed-form post-Newtonian stand-in for PhenomXAS/XHM:
 * TaylorF2 phase (3.5PN, aligned spins), leading-order mode amplitudes, SPA
 * mode scaling, modes (2,2), (2,1), (3,3), (3,2), (4,4).
 *
 * Conventions shared by every entry point
 *   - Parameter vector theta, 11 doubles per sample, row-major [B][11]:
 *       [M_tot (Msun, detector frame), q = m2/m1 in (0,1], chi1, chi2,
 *        D_L (Gpc), iota, phi_c, lambda, beta, psi, t_c (s from orbit epoch)].
 *   - Frequency grid f_k = f0 + k df, k = 0 .. n_bins-1.
 *   - Complex arrays are interleaved (re, im) doubles.
 *   - Every pointer argument named "dev" is device memory owned by the
 *     caller; the library never frees it and keeps no reference after the
 *     call returns.  "stream" is a hipStream_t (NULL = default stream).
 *   - All compute calls are asynchronous on the given stream and never
 *     synchronize the host.  A context must not be used from two streams
 *     at the same time.
 *   - Return value: PES_OK or a negative pes_status; nothing is thrown.
 *     A sample with an unphysical theta (non-finite, M_tot <= 0, q outside
 *     (0,1], |chi| >= 1, D_L <= 0) gets log L = -inf and a zero gradient; the
 *     call still returns PES_OK.
 */
#ifndef PES_H
#define PES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PES_OK = 0,
  PES_EINVAL = -1,  /* bad argument (null pointer, unknown mode, bad size) */
  PES_ESHAPE = -2,  /* sizes inconsistent with the context */
  PES_ENOMEM = -3,  /* device allocation failed */
  PES_EHIP = -4,    /* a HIP runtime call failed */
  PES_ESTATE = -5   /* call order violated (e.g. log L before data was set) */
} pes_status;

enum { PES_LISA = 0, PES_TAIJI = 1, PES_TIANQIN = 2 };
/* Heliocentric orbit model: the first-order-in-eccentricity Keplerian
 * triangle (exactly equilateral), or the exact Kepler ellipses whose first
 * order it is (arms flexing at order e^2 AU).  Sec. 2.1 names Keplerian
 * heliocentric orbits. */
enum { PES_ORBIT_FIRST_ORDER = 0, PES_ORBIT_KEPLER = 1 };

typedef struct {
  int kind;            /* PES_LISA / PES_TAIJI: heliocentric orbit; PES_TIANQIN: geocentric */
  int tdi_gen;         /* 15 or 20 (TDI generation 1.5 or 2.0) */
  double arm_m;        /* arm length L [m] */
  double phase0;       /* initial revolution phase of the constellation centre [rad] */
  double tq_period_s;  /* TianQin: rotation period of the constellation [s] */
  double tq_lon;       /* TianQin: ecliptic longitude of the constellation-plane normal [rad] */
  double tq_lat;       /* TianQin: ecliptic latitude of the plane normal [rad] */
  double oms_asd;      /* optical-metrology noise ASD [m / sqrt(Hz)] */
  double acc_asd;      /* test-mass acceleration noise ASD [m s^-2 / sqrt(Hz)] */
  int orbit;           /* PES_LISA / PES_TAIJI: PES_ORBIT_FIRST_ORDER or PES_ORBIT_KEPLER (every
                          heliocentric detector of a context takes the same); TianQin: 0.
                          With PES_ORBIT_KEPLER the link directions are the unit separations
                          of the spacecraft at t_f, the transfer function and the TDI factor
                          keep the nominal L. */
} pes_detector;

typedef struct {
  int n_det;               /* 1..3 */
  pes_detector det[3];
  int64_t n_bins;          /* 1 .. 2^26 */
  double f0;               /* first frequency [Hz], > 0 */
  double df;               /* spacing [Hz], > 0; also 1/T in the likelihood weights */
  int n_modes;             /* 1..5 */
  int modes[5][2];         /* (l, m) pairs from {(2,2),(2,1),(3,3),(3,2),(4,4)} */
} pes_config;

typedef struct pes_ctx pes_ctx;

/* Create a context on the current HIP device: copies the configuration,
 * allocates the per-bin tables (frequency powers, TDI delay factors, noise
 * weights 4 df / S_c(f) of the analytic PSD) and fills them on the device.
 * Sec. 2.1 (response model) and Sec. 3.2 (noise: OMS + acceleration only).
 * Errors: PES_EINVAL for an invalid config, PES_ENOMEM, PES_EHIP. */
int pes_create(const pes_config* cfg, pes_ctx** out);

/* Release all device memory of the context (synchronizes the device). */
int pes_destroy(pes_ctx* ctx);

/* Reserve workspace for batches of up to max_walkers samples so that later
 * pes_loglike, pes_response, pes_probe, pes_grad and pes_fisher calls with a
 * batch of at most that size allocate nothing (needed before capturing them
 * in a graph).  The derivative part (the walker tangent table, 25 KiB per
 * walker, and per-tile partial sums, under 1 KiB per walker per 1024 bins) is
 * sized for min(max_walkers, 65535), the batch limit of pes_grad and
 * pes_fisher.  Without it those calls grow their workspace on the first call
 * with a larger batch than any before.
 * Errors: PES_EINVAL (negative size), PES_ENOMEM. */
int pes_reserve(pes_ctx* ctx, int64_t max_walkers);

/* Upload the observed data: d (dev) is [n_det][3][n_bins] complex, channels
 * A, E, T of the configured TDI generation.  Precomputes the noise-weighted,
 * TDI-factor-folded data and <d|d>.  The array is copied; it may be freed
 * after the call's work completes on the stream. */
int pes_set_data(pes_ctx* ctx, const double* d, void* stream);

/* One realisation of stationary Gaussian noise in the layout of pes_set_data
 * (Sec. 2.2, eq. eq_diag_Sigma_to_Sn: the noise covariance is diagonal in
 * frequency with <|n_k|^2> = T S_c(f_k) / 2, T = 1 / df): out (dev)
 * [n_det][3][n_bins] complex, real and imaginary parts independent
 * N(0, S_c(f_k) / (4 df)) for channel c of the context's PSD (A and E share
 * S_A), exactly zero where S_c vanishes.  Philox4x32-10 keyed by seed with
 * counter (bin, detector, channel, 0xD0), Box-Muller on its two uniform pairs.
 * Noisy data are the response plus this array. */
int pes_noise(pes_ctx* ctx, uint64_t seed, double* out, void* stream);

/* Stages of the response for testing, from the same evaluation code with
 * hooks that write them out (a plain launch, one thread per (walker, bin),
 * every mode its own unit; not a fast path).  out (dev), by stage:
 *   PES_PROBE_MODE  [B][n_modes][n_bins][3]: mode amplitude with the cutoff
 *     taper (0 beyond the cutoff), SPA phase in cycles mod 1 (the mode's
 *     h = amplitude e^{-2 pi i phase}, Sec. 2.1), t_f - t_c [s] (eq. eq_tf;
 *     NaN beyond the cutoff);
 *   PES_PROBE_GEOM  [B][n_det][n_modes][n_bins][12]: at the mode's t_f, for
 *     arms t = 0, 1, 2 (arm t opposite spacecraft t): k.n_t, (n_t.p)^2 -
 *     (n_t.q)^2, (n_t.p)(n_t.q), then k.(x_0 - c), k.(x_1 - c) and k.c [light-s]
 *     (x_s spacecraft, c the constellation centre; eq. eq_fd_resp's geometry;
 *     n_t the unit separation on exact Kepler orbits);
 *   PES_PROBE_LINKS [B][n_det][n_bins][12]: per arm t (Re, Im) of the forward
 *     and backward link sums of eq. eq_fd_resp over modes, divided by the
 *     common factor -i pi f L e^{-i pi f L}: arm 0 carries y_32 / y_23, arm 1
 *     y_13 / y_31, arm 2 y_21 / y_12.
 * B <= 65535; PES_EINVAL for another stage. */
enum { PES_PROBE_MODE = 0, PES_PROBE_GEOM = 1, PES_PROBE_LINKS = 2 };
int pes_probe(pes_ctx* ctx, const double* theta, int64_t B, int stage, double* out, void* stream);

/* Noise-free response: out (dev) [B][n_det][3][n_bins] complex = A, E, T of
 * h(theta_b) (eqs. eq_tf, eq_fd_resp, FD TDI, A/E/T).  theta (dev) [B][11].
 * B <= 65535; PES_EINVAL otherwise or for a null pointer with B > 0. */
int pes_response(pes_ctx* ctx, const double* theta, int64_t B, double* out, void* stream);

/* log L(theta_b) = -1/2 sum_det sum_{A,E,T} sum_k 4 df |d - h|^2 / S
 * (eq. eq_ll_fd joint over channels and detectors; constants dropped).
 * theta (dev) [B][11], logl (dev) [B].  Requires pes_set_data (PES_ESTATE
 * before it).  B <= 2^24; PES_EINVAL otherwise or for a null pointer with
 * B > 0.  PES_ESHAPE when the work plan, ceil(B / walkers per item) x
 * ceil(n_bins / bin tile) items, exceeds 2^31 - 65537 (its int32 counters);
 * a larger walkers-per-item tuning (pes_set_tuning) lowers the count. */
int pes_loglike(pes_ctx* ctx, const double* theta, int64_t B, double* logl, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pes_loglike
 * with the same arguments, kernels and results, whose workspace is a 64 MiB
 * device array of the library (one per GPU, held until the process ends)
 * instead of the context's; it calls no allocator.  A batch needs, rounded up
 * to 256 bytes per part, 3456 B (walker tables, FP64 and FP32) + 12 B (plan)
 * per walker plus 16 B per walker per bin tile (ceil(n_bins / (256 x bins per
 * lane)) tiles), and on exact Kepler orbits 1600 B per walker and detector
 * (the projected orbit series; 800 B more in single precision): about 970
 * walkers at 2^20 bins and one bin per lane, about 12000 at 32703 bins.  PES_ESHAPE (message in pes_last_error) for a larger batch, PES_EHIP
 * if the array has no address on the context's device; otherwise as
 * pes_loglike.  Every call on one GPU works in that GPU's single array: calls
 * that overlap in time on one GPU (other streams, other contexts, other
 * threads) race and must be serialized by the caller.  No state carries from
 * one call to the next (each call writes every scratch entry it reads). */
int pes_loglike_noalloc(pes_ctx* ctx, const double* theta, int64_t B, double* logl, void* stream);

/* Arithmetic of pes_loglike and pes_response (and of the sampler's
 * likelihood): bits = 64 (default) evaluates everything in FP64; bits = 32
 * keeps in FP64 only what needs more than 24 bits -- each mode's SPA phase
 * and t_f series (eq. eq_tf), f t_c, the cutoff test, the exact removal of
 * whole cycles before every sine and cosine, and the noise-weighted inner
 * products -- and evaluates the amplitudes, orbits, projections, link
 * transfer functions (eq. eq_fd_resp) and TDI combinations in FP32 with FP32
 * fits (the paper compares both precisions, Sec. 3.1, Fig. fig_cost); on
 * exact Kepler orbits the orbit series are evaluated in FP32 from FP32
 * copies of their coefficients.  Gradients and Fisher matrices stay FP64.
 * PES_EINVAL for other values. */
int pes_set_precision(pes_ctx* ctx, int bits);

/* Gradient of log L with respect to theta (Sec. 2.3 differentiates the
 * response in reverse mode): logl (dev) [B] (may be NULL), grad (dev) [B][11]
 * in the units of theta.  Requires pes_set_data.  Unphysical samples:
 * logl = -inf, grad = 0.  B <= 65535.  The method is chosen per context by
 * pes_set_grad_method; both give the same values up to rounding. */
int pes_grad(pes_ctx* ctx, const double* theta, int64_t B, double* logl, double* grad, void* stream);

/* Gradient method of pes_grad:
 *   PES_GRAD_ADJOINT (default): hand-written reverse sweep per bin with the
 *     forward values recomputed (no per-bin storage); adjoints of the walker
 *     table's mode entries contracted with their theta-derivatives, those of
 *     the sky projections reduced through the orthonormal sky basis (this
 *     needs, on the first-order orbit, spacecraft offsets that sum to zero,
 *     as that orbit has; pes_grad returns PES_EINVAL otherwise; on exact
 *     Kepler orbits the projections of the orbit series on all three sky
 *     basis vectors carry it).
 *   PES_GRAD_FORWARD: forward-mode tangents, one (bin, parameter direction)
 *     pair per lane (the evaluation of pes_fisher); the cross-check.
 * PES_EINVAL for another value. */
enum { PES_GRAD_ADJOINT = 0, PES_GRAD_FORWARD = 1 };
int pes_set_grad_method(pes_ctx* ctx, int method);

/* Fisher matrix F_ij = <d_i h | d_j h> (Sec. 2.2, eqs. eq_ll_fisher and
 * eq_inner_product) from the forward-mode Jacobian of the A/E/T response, the
 * J^T W J contraction on FP64 matrix cores: F (dev) [B][11][11], symmetric,
 * in the units of theta.  Independent of the data.  Unphysical samples: NaN.
 * B <= 65535.  On exact Kepler orbits the projected orbit series carry their
 * sky-angle derivatives into the tangents. */
int pes_fisher(pes_ctx* ctx, const double* theta, int64_t B, double* F, void* stream);

/* ---- Sampler.  Bayes' theorem splits the posterior into prior and
 * likelihood (Sec. 2.2); the sampler combines a box prior with pes_loglike. */
enum {
  PES_PRIOR_UNIFORM = 0,     /* flat on [lo, hi] */
  PES_PRIOR_LOGUNIFORM = 1,  /* proportional to 1/x on [lo, hi], lo > 0 */
  PES_PRIOR_SIN = 2,         /* proportional to sin x on (lo, hi) within [0, pi] */
  PES_PRIOR_COS = 3,         /* proportional to cos x on (lo, hi) within [-pi/2, pi/2] */
  PES_PRIOR_PERIODIC = 4,    /* flat, proposals wrapped into [lo, hi) */
  PES_PRIOR_FIXED = 5        /* held at its initial value */
};
typedef struct {
  int kind[11];
  double lo[11];
  double hi[11];
} pes_prior;

typedef struct pes_sampler pes_sampler;

/* Ensemble of n_walkers (>= 4) chains on the context's likelihood.  Every step
 * updates the two halves of the ensemble in turn with differential-evolution
 * proposals drawn against the other half (ter Braak's DE-MC: gamma =
 * 2.38/sqrt(2 d), gamma = 1 with probability 0.1, jitter 1e-6 of the prior
 * width) and Metropolis-Hastings acceptance with the exact FP64 log L.  All
 * random numbers are Philox4x32-10 blocks keyed by seed with counter (walker,
 * step, purpose), so runs are reproducible and graph replays advance by the
 * step counter kept in device memory.  chain_len > 0 keeps a ring of the last
 * chain_len states ([chain_len][n_walkers][11], device).  Reserves the
 * context's workspace for half the ensemble.  Requires pes_set_data. */
int pes_sampler_create(pes_ctx* ctx, const pes_prior* prior, int64_t n_walkers, uint64_t seed,
                       int64_t chain_len, pes_sampler** out);
int pes_sampler_destroy(pes_sampler* s);

/* Set the walkers (theta dev [n_walkers][11]), evaluate their log L and log
 * prior, zero the acceptance counts and the step counter.  Synchronizes. */
int pes_sampler_set_state(pes_sampler* s, const double* theta, void* stream);

/* Checkpoint / resume: set the completed-step counter, which keys every
 * random number of the following steps.  A sampler created with the same
 * context, prior and seed, given a saved state by pes_sampler_set_state and
 * the saved step count here, continues the saved run bitwise (the acceptance
 * counts restart from zero).  Synchronizes the device. */
int pes_sampler_set_step(pes_sampler* s, uint64_t steps);

/* Advance n_steps steps (asynchronous). */
int pes_sampler_step(pes_sampler* s, int64_t n_steps, void* stream);

/* Capture one step in a HIP graph (kernels only, no allocation or memset) and
 * replay it n_steps times; the replay is bitwise identical to
 * pes_sampler_step.  The graph's kernels point into the context's and the
 * flow's workspaces: a later call on the context with a larger batch than the
 * sampler's (pes_loglike, pes_response, pes_probe, pes_grad, pes_fisher,
 * pes_reserve) or a flow call with more rows may reallocate them, and
 * pes_sampler_set_flow may change the flow.  pes_sampler_launch then returns
 * PES_ESTATE without launching anything; capture again.  pes_reserve before
 * the capture avoids the reallocation. */
int pes_sampler_capture(pes_sampler* s, void* stream);
int pes_sampler_launch(pes_sampler* s, int64_t n_steps, void* stream);

/* Copy the state into caller buffers (dev; any may be NULL): theta
 * [n_walkers][11], logl [n_walkers], accepts [n_walkers] (int64); *steps
 * (host) receives the completed step count.  Synchronizes the stream. */
int pes_sampler_state(pes_sampler* s, double* theta, double* logl, int64_t* accepts, uint64_t* steps,
                      void* stream);

/* Device pointer of the chain ring (NULL without one). */
int pes_sampler_chain(pes_sampler* s, const double** chain);

/* The stored states in step order, oldest first: out (dev) [*n_states][n_walkers][11]
 * with *n_states = min(steps done, chain_len) (host).  Synchronizes the stream. */
int pes_sampler_read_chain(pes_sampler* s, double* out, int64_t* n_states, void* stream);

/* One proposal for half `half` (0 or 1) of the ensemble from the current
 * state: theta_prop (dev) [half size][11], log_qratio (dev) [half size]
 * (log q(theta|theta') - log q(theta'|theta); 0 for the symmetric DE move).
 * kind: PES_PROPOSE_DE, or PES_PROPOSE_FLOW for the mixture set by
 * pes_sampler_set_flow (PES_ESTATE without a flow). */
enum { PES_PROPOSE_DE = 0, PES_PROPOSE_FLOW = 1 };
int pes_propose(pes_sampler* s, int kind, int half, double* theta_prop, double* log_qratio, void* stream);

/* ---- Learned proposal.  An affine-coupling normalizing flow q(theta) on the
 * 11 parameters, trained on posterior samples and used as an independence
 * Metropolis-Hastings proposal mixed with the DE move (the proposal is the
 * sampler's choice, Sec. 2.2).  Definition: u = float(L^-1 (theta - mu)) with
 * L lower triangular (whitening; forward substitution in FP64);
 * 8 layers, layer 2p conditions on C_p = {i : (i + 3p) mod 11 < 6} and
 * transforms the rest, layer 2p + 1 conditions on the rest and transforms
 * C_p; conditioner networks n_C -> 256 (ReLU) -> 256 (ReLU) -> 2 n_T with
 * outputs (s_hat, t), s = 3 tanh(s_hat / 3); normalizing map y_T = x_T e^s + t;
 * base N(0, I); log q(theta) = log N(z) + sum s - sum log L_kk.  Network
 * products take BF16 operands (weights, inputs, hidden activations rounded to
 * nearest even) with FP32 accumulation on the matrix cores; FP32 master
 * weights; Adam (beta 0.9, 0.999, eps 1e-8).  Parameters: per layer W1
 * [n_C][256], b1 [256], W2 [256][256], b2 [256], W3 [256][2 n_T], b3 [2 n_T]
 * (y = x W + b), flat FP32 in that order, pes_flow_num_params() in total. */
typedef struct pes_flow pes_flow;
int pes_flow_create(uint64_t seed, pes_flow** out);   /* random init, near identity; mu 0, L = I */
int pes_flow_destroy(pes_flow* f);
int64_t pes_flow_num_params(void);
/* params (dev) FP32 [pes_flow_num_params()]; set also resets the Adam state. */
int pes_flow_set_params(pes_flow* f, const float* params, void* stream);
int pes_flow_get_params(pes_flow* f, float* params, void* stream);
/* Whitening map (host arrays): mu [11] and L [11][11] row-major, lower
 * triangular (entries above the diagonal ignored), L_kk > 0, else PES_EINVAL.
 * set_norm is the diagonal case L = diag(sigma). */
int pes_flow_set_affine(pes_flow* f, const double* mu, const double* L);
int pes_flow_get_affine(pes_flow* f, double* mu, double* L);
int pes_flow_set_norm(pes_flow* f, const double* mu, const double* sigma);
/* Temperature tau > 0 of the base density N(0, tau^2 I) used by forward,
 * inverse (latent tau z) and the sampler's proposals; training is unaffected
 * (default 1; tau > 1 widens the proposal's tails). */
int pes_flow_set_temperature(pes_flow* f, double tau);
/* log q(theta) for theta (dev) [n][11] -> logq (dev) [n]; z (dev) [n][11] or NULL. */
int pes_flow_forward(pes_flow* f, const double* theta, int64_t n, double* z, double* logq, void* stream);
/* theta = inverse map of tau z, z (dev) [n][11]; logdet (dev) [n] or NULL: sum s at theta. */
int pes_flow_inverse(pes_flow* f, const double* z, int64_t n, double* theta, double* logdet, void* stream);
/* Test entry point: pes_flow_forward (inverse = 0: in = theta, out = z, lq =
 * logq) or pes_flow_inverse (inverse = 1: in = z, out = theta, lq = logdet or
 * NULL) through the same kernels, that also writes the FP32 coupling state of
 * the n rows before the first layer and after every layer, in the order the
 * layers are applied, to states (dev) FP32 [9][n][11] (slot 0: the
 * standardized u, or the latent tau z), and the running sum of s at the same
 * points to logdet (dev) FP32 [9][n].  Slot 8 holds z (forward) or u
 * (inverse).  acts (dev) FP32 [8][n][576] or NULL receives, for layer l (by
 * its index, not the order applied), the conditioner's stages as the matrix
 * cores saw them: columns 0..31 the BF16 input x_C (zero padded), 32..287 and
 * 288..543 the two BF16 hidden layers, 544..575 the FP32 output (s_hat, t,
 * zero padded).  Each rounding decision and each layer's map can so be checked
 * on the values the library itself fed it (the affine coupling of Dinh et al.
 * 2017, the proposal's definition above).  PES_EINVAL for a null pointer with
 * n > 0. */
int pes_flow_probe(pes_flow* f, const double* in, int64_t n, int inverse, double* out, double* lq,
                   float* states, float* logdet, float* acts, void* stream);
/* Mean negative log-likelihood of the rows of theta (dev) [n][11] in the
 * standardized space, -(1/n) sum log q_u(u_j), into nll (dev) [1] (may be
 * NULL), and its gradient into grad (dev) FP32 [pes_flow_num_params()]. */
int pes_flow_nll_grad(pes_flow* f, const double* theta, int64_t n, double* nll, float* grad, void* stream);
/* One Adam update with grad (dev, FP32) or, when NULL, the last gradient. */
int pes_flow_adam_step(pes_flow* f, const float* grad, float lr, void* stream);
/* steps Adam updates on minibatches of `batch` rows of samples (dev) [n][11]
 * (drawn with replacement; all rows in order when batch == n); standardize
 * != 0 first sets mu to the samples' mean and L to the Cholesky factor of
 * their covariance (synchronizes; PES_EINVAL if it is not positive definite).
 * The learning rate decays as lr (1 + cos(pi t / steps)) / 2.  loss (dev)
 * [steps] or NULL receives each step's NLL. */
int pes_flow_fit(pes_flow* f, const double* samples, int64_t n, int64_t steps, int64_t batch, float lr,
                 uint64_t seed, int standardize, double* loss, void* stream);
const char* pes_flow_last_error(pes_flow* f);

/* Use flow f in the sampler's steps: every walker of the half being updated
 * takes the flow's independence proposal with probability p_flow (Philox
 * purpose 19; latent draws purposes 20..30, Box-Muller) and the DE move
 * otherwise; log q ratio = log q(current) - log q(proposal); a flow proposal
 * outside [lo, hi) of a periodic parameter is rejected.  f = NULL returns to
 * DE only.  Every prior must be free (PES_EINVAL with a fixed parameter).
 * The flow must outlive its use; set it before pes_sampler_capture. */
int pes_sampler_set_flow(pes_sampler* s, pes_flow* f, double p_flow);

/* Philox4x32-10 (Salmon et al., SC'11) blocks for the counters
 * (c0 + i, c1, c2, c3), i = 0..n-1 (first word wraps modulo 2^32), with the
 * 64-bit key split into two words (low first): out (dev) [n][4] uint32. */
int pes_philox(uint64_t key, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n, uint32_t* out,
               void* stream);

/* Tuning of the persistent log-likelihood kernel: bins per lane (1 or 2),
 * walkers per work item (1..64) and resident blocks per compute unit
 * (0 = the occupancy limit, else at most that limit).  Defaults 1, 16, 0.
 * Applies to later calls on the context. */
int pes_set_tuning(pes_ctx* ctx, int bins_per_lane, int walkers_per_group, int blocks_per_cu);
int pes_get_tuning(pes_ctx* ctx, int* bins_per_lane, int* walkers_per_group, int* blocks_per_cu);

/* Work schedule of pes_loglike (the batching of many samples per launch that
 * the paper lists as future work, Sec. 4):
 *   PES_SCHED_QUEUE (default): walkers sorted by their active tile count
 *     (bins below the highest mode cutoff), a persistent grid taking
 *     (walker group, tile) items from an atomic ticket over active tiles only.
 *   PES_SCHED_GRID: a plain grid of one block per (walker group, tile) over
 *     every tile of the frequency grid, walkers in batch order (each mode still
 *     skips the bins beyond its cutoff).  Kept for measuring what the queue
 *     saves; PES_ESHAPE when the item count exceeds 2^31 - 1.
 * Both give bitwise the same log-likelihoods.  PES_EINVAL for another value. */
enum { PES_SCHED_QUEUE = 0, PES_SCHED_GRID = 1 };
int pes_set_schedule(pes_ctx* ctx, int schedule);

/* Autotuner: runs pes_loglike on the given batch (theta dev [B][11], logl
 * dev [B] receives the results) for every tuning candidate (bins per lane 1
 * or 2, walkers per item 8, 16, 32 or 64, blocks per CU at the occupancy
 * limit or half of it): the mean of two calls after a warm-up, then the three
 * fastest again as the least of three single calls.  Keeps the fastest, or
 * among those finalists within 1% of it the one with the most walkers per item
 * (each item reads its bin tile's tables once, so it moves the fewest bytes),
 * and returns its time per call [ms] in *best_ms; on an error the previous
 * tuning stays.  Synchronizes the stream; the results do not depend on the
 * tuning. */
int pes_autotune(pes_ctx* ctx, const double* theta, int64_t B, double* logl, double* best_ms,
                 void* stream);

/* Kernel timing for measurement: with enable != 0 every later pes_loglike
 * records HIP events around its main (persistent log-likelihood) kernel on
 * the call's stream, up to 4096 launches.  pes_timing_read waits for the
 * recorded events, returns the summed kernel time [ms] and the number of
 * launches, and clears the record.  Events are created and destroyed by the
 * library. */
int pes_timing(pes_ctx* ctx, int enable);
int pes_timing_read(pes_ctx* ctx, double* total_ms, int64_t* launches);

/* Human-readable message of a status code (static storage). */
const char* pes_strerror(int status);

/* Last HIP error text recorded by the context (static per context). */
const char* pes_last_error(pes_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* PES_H */
