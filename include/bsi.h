/*
 * bsi.h -- C ABI of the Bayesian shear inference library for MI355X (gfx950).
 *
 * The method is that of arXiv 2604.22048 ("Differentiable Forward Modeling
 * for Efficient and Accurate Shear Inference").  Phase 1 samples the interim
 * posterior of each galaxy's properties from its pixel stamp
 * (eq. interim-post with the pixel likelihood eq. likelihood-pixels and the
 * interim prior eq. interim-prior); phase 2 evaluates the Monte-Carlo shear
 * likelihood eq. likelihood-shear from the fixed interim samples, with the
 * shear Jacobian of eq. true-prior-jacobian-shear.  Beyond that path: the
 * multiplicative and additive bias by shape-noise cancellation with
 * bootstrap errors (Section 3.5), Spergel profiles (Appendix B), correlated
 * noise and several exposures per galaxy (Appendix C), and the No-U-Turn
 * sampler of Section 3.3 beside fixed-length HMC.
 *
 * Conventions for every call
 *   - Return value: BSI_OK (0) or a negative BSI_E* code.  Arguments are
 *     validated synchronously before anything is enqueued; on a validation
 *     error nothing is enqueued and no output is written.  The message of
 *     the last error on a handle is returned by bsi_last_error().
 *   - Asynchronous device failures are sticky on the handle and reported by
 *     the next call (BSI_EHIP).
 *   - Numerical trouble in one galaxy never fails a call; it sets that
 *     galaxy's status bits (BSI_STATUS_*).
 *   - Pointers marked [device] are caller-owned device memory on the
 *     handle's device; [host] pointers are read during the call only.  The
 *     library never frees caller memory.  It allocates only handle-owned
 *     workspace (see "Workspace, streams and graph capture" below).
 *   - Calls are stream-ordered on `stream` (a hipStream_t; NULL means the
 *     default stream).  A handle must be used from one host thread at a
 *     time.
 *   - Stamps: square N x N single-precision images stored row-major
 *     ([y][x]), packed back to back in one buffer; stamp i starts at
 *     element off[i] (one stamp per galaxy unless bsi_batch.n_exp > 1).
 *     Pixel centres are at x_i = i - (N-1)/2 (same in y).
 *   - Physical parameters (params): float[6] per galaxy =
 *     {flux F, half-light radius s [arcsec] of the circular pre-shear
 *      profile, e1, e2 (reduced-shear convention, eq. ellip-phi-transform),
 *      dx, dy [pixels from the stamp centre]}.
 *   - Sampling coordinates (theta): float[6] =
 *     {log10 F, log10 s, e1, e2, Dx, Dy} with (Dx, Dy) the offset in pixels
 *     from a per-galaxy reference centroid ref_xy (the prior of eq.
 *     interim-prior centres the offsets on the true centroid).
 */
#ifndef BSI_H
#define BSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BSI_VERSION 4

enum {
  BSI_OK = 0,
  BSI_EINVAL = -1,        /* invalid argument (message in bsi_last_error)  */
  BSI_ENOMEM = -2,        /* device workspace allocation failed             */
  BSI_EHIP = -3,          /* HIP runtime error (possibly from earlier work)  */
  BSI_EUNSUPPORTED = -4,  /* size or device not supported (gfx950 only)     */
  BSI_ENODEV = -5         /* no usable device                                */
};

/* Per-galaxy status bits (OR-ed over all of a galaxy's chains).  For
 * bsi_hmc_sample they cover the start positions and the stored iterations;
 * warmup trajectories (whose step-size probes routinely leave the support)
 * are not reported. */
enum {
  BSI_STATUS_OUT_OF_SUPPORT = 1,  /* a parameter set or trajectory left the prior support */
  BSI_STATUS_NONFINITE = 2,       /* a non-finite log-likelihood or energy was met        */
  BSI_STATUS_DIVERGENT = 4        /* |dH| > 1000 in some trajectory                       */
};

/* Galaxy light profiles.  EXPONENTIAL is the model of Section 3.2 (its
 * Fourier transform (1 + r0^2 k^2)^(-3/2)); SPERGEL is the Spergel (2010)
 * profile of fixed index nu used for the model-bias fits of Appendix B, with
 * Fourier transform (1 + r0^2 k^2)^(-(1+nu)) (nu = 1/2 is the exponential,
 * nu near -0.6 close to de Vaucouleurs); GAUSSIAN is a test profile.  The size
 * parameter is always the half-light radius. */
enum { BSI_PROFILE_EXPONENTIAL = 0, BSI_PROFILE_GAUSSIAN = 1, BSI_PROFILE_SPERGEL = 2 };

/* Spergel indices accepted (BSI_EINVAL outside). */
#define BSI_SPERGEL_NU_MIN (-0.85f)
#define BSI_SPERGEL_NU_MAX 4.0f

/* Log-likelihood evaluation method for bsi_loglik_grad. */
enum {
  BSI_LIK_KSPACE = 0,  /* exact Parseval form on the stamp's DFT grid (default) */
  BSI_LIK_PIXEL = 1    /* render, pixel residual, adjoint transform             */
};

typedef struct bsi_ctx* bsi_handle;
typedef void* bsi_stream;   /* hipStream_t */

/* Library version (BSI_VERSION). */
int bsi_version(void);

/* Number of visible HIP devices in *n (0 when none); BSI_OK or BSI_EHIP. */
int bsi_device_count(int32_t* n);

/* Create a handle bound to `device` (HIP ordinal).  Fails with BSI_ENODEV
 * when no device exists, BSI_EUNSUPPORTED when it is not gfx950.
 *
 * tune_cache [host, nullable or empty: none]: path of a tuning cache, a text
 * file holding the slot plans and render transforms chosen per stamp side.
 * If the file exists and was written by this library version for this device
 * (architecture and compute-unit count), the handle starts with its choices;
 * a file of another version or device is ignored, a missing file is an empty
 * cache, and a file that does not parse fails the call with BSI_EINVAL
 * (message from bsi_last_error(NULL)).  bsi_autotune and
 * bsi_autotune_transform then rewrite the file with the handle's choices at
 * that moment (explicit bsi_set_plan / bsi_set_transform choices included),
 * by writing a private file and renaming it over the cache; a failed write
 * makes those calls return BSI_EINVAL (the handle keeps its new choices).
 * Format, one item per line: "bsi-tune-cache 1", "library <version>",
 * "device <arch> <compute units>", then "plan <N> <P>" and
 * "transform <N> <method>" lines.  (A runtime facility: the paper's
 * method does not depend on these settings, only the speed of the kernels
 * that evaluate it.) */
int bsi_create(bsi_handle* out, int32_t device, const char* tune_cache);

/* Release a handle and its workspace; NULL is ignored.  Waits for the
 * handle's outstanding work. */
void bsi_destroy(bsi_handle h);

/* Message of the last failing call on h (empty string if none; never NULL).
 * With h == NULL returns the last error of bsi_create on this thread. */
const char* bsi_last_error(bsi_handle h);

/*
 * Workspace, streams and graph capture.
 *   - Each call sizes the handle's workspace for its arguments before it
 *     enqueues anything.  Growing allocates new device buffers; the buffers
 *     they replace stay allocated (work enqueued earlier may still read
 *     them) until bsi_reserve or bsi_destroy.  No call synchronises the
 *     device.
 *   - Host inputs the device needs (a batch's stamp plan from n and off, and
 *     host-side shear points) are packed into a pinned, device-mapped
 *     staging buffer of the handle and copied by a kernel; a call first waits
 *     on the host until the previous call's copy out of that buffer has run.
 *   - Calls on different streams: a call waits (on the device) for the
 *     handle's previous call when that was made on another stream, because
 *     they share the workspace.
 *   - Graph capture (the two phases of Section 3.3 run as fixed launch
 *     sequences, so a caller can capture them): a call whose stream is being
 *     captured (relaxed or thread-local mode) records kernel nodes only,
 *     never allocates, and fails with BSI_EINVAL before enqueueing anything
 *     when the workspace is smaller than it needs, so call bsi_reserve first.
 *     The graph reads the handle's workspace and staging buffer at every
 *     replay: until it is destroyed, use the handle for no other call
 *     (one handle per live graph), and replay it after bsi_reserve only if
 *     that reserve came first.  bsi_hmc_sample under capture ignores
 *     use_graph and records its trajectory launches (the stamp sizes in
 *     sequence) into the caller's graph.
 *   - bsi_autotune, bsi_autotune_transform and the slot server allocate
 *     their own buffers and are not for capture.
 */

/* Workspace limits of bsi_reserve (every field >= 0). */
typedef struct {
  int64_t max_stamps;     /* stamps (galaxies x exposures) of the largest batch of
                             bsi_render_stamps, bsi_loglik_grad and bsi_hmc_sample, packed
                             (their offsets span at most max_stamps max_n^2 elements)      */
  int32_t max_n;          /* largest stamp side of those batches, 8..128 (any slot plan)  */
  int32_t max_chains;     /* largest n_chains of bsi_hmc_sample, 0..16                    */
  int32_t weighted;       /* nonzero: batches with n_exp > 1 or noise_ps                  */
  int32_t pixel_method;   /* nonzero: bsi_loglik_grad with BSI_LIK_PIXEL                  */
  int64_t max_shear_gal;  /* galaxies of bsi_shear_posterior, _galaxy_loglik, _hmc, _bias */
  int32_t max_points;     /* points of bsi_shear_posterior / bsi_shear_galaxy_loglik (host
                             or device points), chains of bsi_shear_hmc, grid points of
                             bsi_shear_bias                                               */
  int32_t bias;           /* nonzero: bsi_shear_bias with max_points grid points          */
  int32_t max_boot;       /* bootstrap resamples of bsi_shear_bias                        */
} bsi_reserve_cfg;

/*
 * bsi_reserve -- size the handle's workspace for every call within the
 * limits, so that such calls neither allocate nor fail under graph capture
 * (Section 3.3's two phases: the per-galaxy sampler and the shear
 * posterior).  Synchronises the device, frees the buffers earlier growth
 * replaced, and grows (never shrinks) each buffer.  Graphs captured before
 * the call may read freed buffers: capture after reserving.
 * Returns BSI_EINVAL (negative limits, max_chains > 16, bias without
 * 1..8192 points), BSI_EUNSUPPORTED (max_n outside 8..128 with
 * max_stamps > 0), BSI_ENOMEM, or BSI_EHIP.
 */
int bsi_reserve(bsi_handle h, const bsi_reserve_cfg* cfg);

/* A ragged batch of square stamps. */
typedef struct {
  int32_t n_gal;             /* number of galaxies, >= 0                              */
  const int32_t* n;          /* [host] stamp side N_i, 8 <= N_i <= 128                  */
  const int64_t* off;        /* [host] element offset of stamp i in the packed buffer   */
  const float* psf_fwhm;     /* [device] Gaussian PSF FWHM per galaxy, arcsec, > 0      */
  const float* sigma;        /* [device] pixel noise sigma per galaxy (b = sigma^2), > 0 */
  float pixel_scale;         /* arcsec per pixel, > 0                                   */
  int32_t profile;           /* BSI_PROFILE_*                                           */
  float spergel_nu;          /* Spergel index for BSI_PROFILE_SPERGEL, in
                                [BSI_SPERGEL_NU_MIN, BSI_SPERGEL_NU_MAX]; else ignored   */
  int32_t n_exp;             /* exposures per galaxy (Appendix C), 0..BSI_MAX_EXPOSURES;
                                0 and 1: one.  With E > 1 exposures, stamp i E + j is
                                exposure j of galaxy i: n, off, psf_fwhm and sigma hold
                                n_gal E entries (per stamp) and the exposures of a galaxy
                                share N; params, ref_xy, init, outputs stay per galaxy.
                                log L and its gradient are sums over the exposures        */
  const float* noise_ps;     /* [device] stationary correlated noise (Appendix C), or NULL
                                for white noise: per stamp, float[N][N] at element off[s]
                                (the stamps' packing), lambda(v, u) for the DFT mode
                                (u, v) in FFT order (index (v mod N) N + (u mod N)), the
                                noise covariance being sigma^2 times the circulant matrix
                                with these eigenvalues (lambda = sum_x c(x) e^{-i k.x} of
                                the covariance function c, c(0) = 1 for unit variance);
                                every lambda > 0 and lambda(-k) = lambda(k).  All ones is
                                white noise                                               */
} bsi_batch;

/* Largest n_exp of a batch. */
#define BSI_MAX_EXPOSURES 16

/*
 * bsi_render_stamps -- noiseless model stamps (Section 3.2: the batch's
 * profile -- exponential, Spergel or Gaussian -- sheared, convolved with the
 * known Gaussian PSF and integrated over pixels), through the
 * handle's transform for each stamp side (bsi_set_transform).
 * The stamp is the truncated Fourier series on the stamp's frequency grid:
 *   m[j,i] = N^-2 sum_{u,v} w_u w_v T(u,v) exp(i(k_u x_i + k_v y_j)),
 *   k_u = 2 pi u / N, u in -floor(N/2)..floor(N/2), w = 1/2 at u = +-N/2 for
 *   even N and 1 otherwise,
 *   T = F G(q) exp(-sigma_psf^2 |k|^2 / 2) sinc(u/N) sinc(v/N) exp(-i k.d),
 * with G the Fourier transform of the sheared, unit-flux profile.
 *   params [device] float[n_gal][6] physical parameters.
 *   out    [device] packed stamps, element off[s] .. off[s] + N_s^2 - 1 for
 *          every stamp s (with n_exp > 1 each exposure with its own PSF).
 */
int bsi_render_stamps(bsi_handle h, const bsi_batch* batch, const float* params, float* out,
                      bsi_stream stream);

/*
 * bsi_loglik_grad -- pixel log-likelihood of eq. likelihood-pixels,
 *   log L = -1/2 sum_p (d_p - m_p)^2 / sigma^2   (constant C = 0),
 * and its gradient with respect to the physical parameters.
 *   data    [device] packed stamps.
 *   params  [device] float[n_gal][6].
 *   loglik  [device] double[n_gal] or NULL.
 *   grad    [device] float[n_gal][6] d log L / d params, or NULL.
 *   status  [device] uint32[n_gal] or NULL (bit OUT_OF_SUPPORT when
 *           |e| >= 1 or s <= 0 or F <= 0; NONFINITE when log L is not finite).
 *   method  BSI_LIK_KSPACE or BSI_LIK_PIXEL (same value up to rounding).
 * With n_exp > 1 or noise_ps (Appendix C, eq. covar-pixel-likelihood):
 *   log L = -1/2 sum_j (d_j - m_j)^T Sigma_j^-1 (d_j - m_j),
 * evaluated on the DFT grid, where Sigma_j^-1 is diagonal with entries
 * 1 / (sigma_j^2 lambda_j(k)); BSI_LIK_KSPACE only (BSI_EUNSUPPORTED else).
 */
int bsi_loglik_grad(bsi_handle h, const bsi_batch* batch, const float* data, const float* params,
                    double* loglik, float* grad, uint32_t* status, int32_t method,
                    bsi_stream stream);

/* Interim prior of eq. interim-prior (paper values in brackets). */
typedef struct {
  float log10f_lo, log10f_hi;   /* uniform log10 F support   [-1, 9]  */
  float log10s_lo, log10s_hi;   /* uniform log10 s support   [-2, 1]  */
  float sigma_d;                /* Gaussian sigma of Dx, Dy  [0.5 px] */
  float sigma_e;                /* ellipticity prior sigma   [0.3]    */
} bsi_interim;

enum { BSI_METRIC_GIVEN = 0, BSI_METRIC_FISHER = 1 };
/* Transition of bsi_hmc_sample: fixed-length HMC (n_leapfrog steps, step
 * jitter) or the No-U-Turn sampler of Section 3.3 (the paper's sampler). */
enum { BSI_SAMPLER_HMC = 0, BSI_SAMPLER_NUTS = 1 };
#define BSI_NUTS_MAX_DEPTH 10
enum { BSI_FORM_BATCHED = 0, BSI_FORM_PLAIN = 1 };

/* Hamiltonian sampler settings.  One iteration = one trajectory of
 * n_leapfrog steps followed by the Metropolis test. */
typedef struct {
  int32_t n_chains;          /* chains per galaxy, 1..16                                   */
  int32_t n_leapfrog;        /* leapfrog steps per trajectory, >= 1                        */
  int32_t n_warmup;          /* warmup iterations (not stored), >= 0                       */
  int32_t n_samples;         /* stored iterations, >= 0                                    */
  int32_t adapt;             /* 1: dual-averaging step-size adaptation during warmup       */
  int32_t metric;            /* BSI_METRIC_GIVEN (inv_mass or identity) or _FISHER          */
  float step_size;           /* initial (adapt) or fixed step size, > 0                    */
  float target_accept;       /* dual-averaging target delta in (0, 1) [0.8]                */
  float jitter;              /* relative step-size jitter in [0, 1) [0 = none]             */
  int32_t form;              /* BSI_FORM_BATCHED: all galaxies per launch;
                                BSI_FORM_PLAIN: one galaxy and one leapfrog step per launch */
  int32_t iters_per_launch;  /* batched form: trajectories per kernel launch (>= 1)        */
  int32_t use_graph;         /* batched form: 1 = replay each launch round from a captured
                                HIP graph (the stamp sizes' launches in sequence on one
                                stream); 0 = direct launches, the sizes concurrently on
                                forked streams                                             */
  uint64_t seed;             /* Philox key                                                 */
  uint64_t uid_base;         /* chain uid = uid_base + galaxy * n_chains + chain           */
  float* trace;              /* [device] float[n_gal][n_chains][n_warmup + n_samples][4] or
                                NULL: per iteration {base step size, dH, acceptance
                                statistic min(1, exp(-dH)) (0 if rejected for support or
                                non-finiteness), accepted (0 or 1)}                          */
  int32_t waves_per_chain;   /* 0 or 1: one wave per chain (throughput); 2 or 4: up to that
                                many waves share each chain's evaluations (latency), for the
                                workload stamp sizes with their default slot plan and the
                                exponential or Spergel profile (fewer where a size has fewer super-rows
                                or n_chains * waves would exceed 4).  The sums are split
                                differently, so samples agree with the one-wave form to
                                float32 rounding, and bitwise between calls with equal
                                settings                                                     */
  int32_t sampler;           /* BSI_SAMPLER_HMC (0) or BSI_SAMPLER_NUTS.  NUTS: each
                                iteration doubles its trajectory up to max_tree_depth times
                                (multinomial sampling of the points, momentum-sum U-turn
                                criterion at every node of the trajectory's binary tree,
                                divergence at H - H0 > 1000); n_leapfrog, jitter and
                                waves_per_chain are ignored; iters_per_launch counts
                                transitions; each chain runs on its own wave (with an even
                                n_chains on the 25-, 41- and 53-pixel kernels of the default
                                plans: its own half-wave, stepping its tree independently),
                                so chains of different trajectory lengths do not wait for
                                each other (a galaxy's workgroup ends with its slowest
                                chain); trace rows hold {step size, leapfrog steps,
                                acceptance statistic, doublings}                              */
  int32_t max_tree_depth;    /* NUTS: 1..BSI_NUTS_MAX_DEPTH (the paper uses 5)              */
} bsi_hmc_cfg;

/*
 * bsi_hmc_sample -- phase 1: sample every galaxy's interim posterior.
 *   data       [device] packed stamps.
 *   ref_xy     [device] float[n_gal][2] reference centroid (pixels from the
 *              stamp centre); the model centroid is ref_xy + (Dx, Dy).
 *   inv_mass   [device] float[n_gal][6] diagonal inverse metric or NULL
 *              (identity); ignored with BSI_METRIC_FISHER.
 *   init       [device] float[n_gal][n_chains][6] start positions (theta).
 *   samples    [device] float[n_gal][n_chains][n_samples][6] (theta) or NULL.
 *   chain_stats[device] float[n_gal][n_chains][4] = {accept rate over the
 *              stored iterations, final step size, divergent stored trajectories,
 *              final potential energy} or NULL.
 *   status     [device] uint32[n_gal] or NULL.
 * Random numbers: Philox4x32-10 keyed by seed, counter (uid, t, tag, block)
 * with t the iteration index; so the output of a chain does not depend on
 * which other galaxies share the call.
 * With n_exp > 1 or noise_ps the potential uses the likelihood of
 * bsi_loglik_grad's Appendix C form (and the Fisher metric its weighted
 * curvature); those batches ignore waves_per_chain (one wave per chain, or two
 * chains per wave for a single exposure on the kernels specialised per stamp
 * size) and need n_chains <= 4.
 */
int bsi_hmc_sample(bsi_handle h, const bsi_batch* batch, const float* data, const float* ref_xy,
                   const float* inv_mass, const float* init, const bsi_interim* interim,
                   const bsi_hmc_cfg* cfg, float* samples, float* chain_stats, uint32_t* status,
                   bsi_stream stream);

/* True prior of the intrinsic properties used in phase 2. */
enum { BSI_E_BA14 = 0, BSI_E_TRUNC_GAUSS = 1 };
typedef struct {
  int32_t e_kind;            /* BSI_E_BA14: (1-E)^2 exp(-E/2 sigma_e^2) on |e| < 1
                                (eq. ellip-mag-prior in (e1, e2) form);
                                BSI_E_TRUNC_GAUSS: exp(-E/2 sigma_e^2) on |e| < e_max   */
  float e_max;
  int32_t size_term;         /* 1: include ln s ~ N(mu_ln_s, sigma_ln_s)                  */
  int32_t flux_term;         /* 1: include ln F ~ N(mu_ln_f, sigma_ln_f)                  */
  double mu_ln_f, sigma_ln_f;
} bsi_true_prior;

/*
 * bsi_shear_posterior -- phase 2: Monte-Carlo shear log-likelihood
 * (eq. likelihood-shear) at n_pts points of (g1, g2, mu_ln_s, sigma_ln_s,
 * sigma_e):
 *   ln P = sum_n [ ln sum_k w_nk - ln K ] (+ 0 inside the uniform priors,
 *          -inf outside: |g| < 1, 1e-4 < sigma_e < 1, |mu_ln_s| < 2 ln 10,
 *          0 < sigma_ln_s < ln 10 / 2),
 *   ln w_nk = ln p_e(h_g^-1(e'_nk)) + ln|d eps/d eps'| - ln P0_e(e'_nk)
 *             + size and flux terms (true minus interim density, in log10
 *             coordinates).  Centroid terms cancel (Section 3.3).
 * The log-sum-exp over k and the sum over galaxies are carried in float64.
 *   e1p, e2p, log10s, log10f  [device] float[n_gal][K] interim samples
 *              (structure of arrays; log10f may be NULL when flux_term = 0).
 *              Any K >= 1: up to 1024 samples per galaxy (512 when
 *              n_pts <= 16) are held at once; larger K is taken in chunks of
 *              512 whose float64 sums are combined exactly (a rescaling to
 *              the larger reference).
 *   pts      [host or device, see pts_on_device] double[n_pts][5].
 *   logpost  [device] double[n_pts].
 *   grad     [device] double[n_pts][5] gradient of ln P, or NULL.
 * Samples whose intrinsic ellipticity falls outside the true prior's
 * support get weight 0; a galaxy with all weights 0 gives ln P = -inf.
 */
int bsi_shear_posterior(bsi_handle h, int32_t n_gal, int32_t K, const float* e1p,
                        const float* e2p, const float* log10s, const float* log10f,
                        const bsi_true_prior* tp, const bsi_interim* interim, int32_t n_pts,
                        const double* pts, int32_t pts_on_device, double* logpost, double* grad,
                        bsi_stream stream);

/* Capacity of the device scratch of bsi_shear_posterior_noalloc (per device). */
#define BSI_NOALLOC_SCRATCH_BYTES (16 << 20)

/*
 * bsi_shear_posterior_noalloc -- bsi_shear_posterior for callers that cannot
 * allocate device memory (code under graph capture, tight serving loops,
 * harnesses that forbid allocation): the same kernels and results (bitwise),
 * with the per-block partial sums of the evaluation pass kept in a fixed
 * device array of BSI_NOALLOC_SCRATCH_BYTES that the library holds on every
 * device it runs on until the process ends, instead of handle workspace.
 * The call allocates nothing and uses no handle workspace.
 *   pts      [device] double[n_pts][5] (host points would need staging memory).
 *   other arguments as for bsi_shear_posterior.
 * The pass needs blocks x n_pts x 48 bytes of scratch for its partial sums,
 * blocks = min(ceil(n_gal / 4), max(16, R / ceil(n_pts / 64))), R = 768 for
 * n_pts <= 16 and 512 otherwise; every
 * n_pts <= 21845 fits, larger counts fail with BSI_EINVAL when they exceed
 * it.  All calls on
 * one device share its scratch, and the array keeps the last call's contents
 * (every entry a call reads, it has written first): calls that overlap on one
 * device -- on different streams or handles, or different host threads --
 * race.
 */
int bsi_shear_posterior_noalloc(bsi_handle h, int32_t n_gal, int32_t K, const float* e1p,
                                const float* e2p, const float* log10s, const float* log10f,
                                const bsi_true_prior* tp, const bsi_interim* interim, int32_t n_pts,
                                const double* pts, double* logpost, double* grad, bsi_stream stream);

/*
 * bsi_shear_galaxy_loglik -- the per-galaxy terms of bsi_shear_posterior's
 * sum (eq. likelihood-shear) at n_pts points:
 *   ell[p][n] = ln sum_k w_nk(point p) - ln K,
 * -inf where no sample of galaxy n lies in the true prior's support at point
 * p.  The points are not checked against the hyper-prior support (every
 * point is evaluated).
 *   e1p .. log10f, tp, interim, pts, pts_on_device   as for bsi_shear_posterior.
 *   ell   [device] double[n_pts][n_gal].
 */
int bsi_shear_galaxy_loglik(bsi_handle h, int32_t n_gal, int32_t K, const float* e1p,
                            const float* e2p, const float* log10s, const float* log10f,
                            const bsi_true_prior* tp, const bsi_interim* interim, int32_t n_pts,
                            const double* pts, int32_t pts_on_device, double* ell,
                            bsi_stream stream);

/*
 * bsi_shear_bias -- multiplicative and additive shear bias by shape-noise
 * cancellation with bootstrap errors (Section 3.5; Table 2).  Two datasets
 * hold the same galaxies and noise, sheared by +g and -g with g = (g_abs, 0).
 * With the population parameters fixed, the shear posterior of a galaxy
 * resample that draws galaxy n c_n times is ln P(g_p) = sum_n c_n ell_n(g_p)
 * (+ const), and the estimator is its mean over the dataset's grid points:
 *   g_hat = sum_p g_p e^(ln P(g_p) - max) / sum_p e^(ln P(g_p) - max).
 * Row r = 0 uses every galaxy once; rows r = 1..n_boot use counts[r - 1].
 *   m_r = (g_hat+_1 - g_hat-_1) / (2 g_abs) - 1,   c_r = (g_hat+_2 + g_hat-_2) / 2.
 * The sums over galaxies are one float64 product on the matrix cores (the
 * order of the additions differs from a sequential sum).
 *   ell_plus, ell_minus  [device] double[n_pts][n_gal]: bsi_shear_galaxy_loglik
 *                        of each dataset at its grid points.
 *   gpts    [device] double[2][n_pts][2]: the grid points' (g1, g2), those of
 *           the +g dataset, then those of the -g dataset.
 *   counts  [device] int32[n_boot][n_gal]: times galaxy n is drawn in each
 *           resample (rows of the classic bootstrap sum to n_gal; not
 *           checked); may be NULL when n_boot = 0.
 *   gmean   [device] double[2][n_boot + 1][2]: g_hat of the +g rows, then of
 *           the -g rows, or NULL.
 *   mc      [device] double[n_boot + 1][2]: (m_r, c_r), or NULL.
 *   stats   [device] double[4] = {m_0, c_0, sd(m_1..m_B), sd(c_1..c_B)}
 *           (population standard deviations; 0 when n_boot = 0).
 * ell = -inf is carried as -1e300, so a galaxy not drawn adds exactly 0; a
 * row whose every grid point is -inf has no meaningful mean.
 * Limits: 1 <= n_pts <= 8192, n_boot >= 0, g_abs > 0.  Uses handle
 * workspace (n_boot + 1) x 2 n_pts doubles per galaxy split.
 */
int bsi_shear_bias(bsi_handle h, int32_t n_gal, int32_t n_pts, const double* ell_plus,
                   const double* ell_minus, const double* gpts, double g_abs, int32_t n_boot,
                   const int32_t* counts, double* gmean, double* mc, double* stats,
                   bsi_stream stream);

/* Shear-level sampler settings (the per-galaxy sampler's scheme on the five
 * population parameters). */
typedef struct {
  int32_t n_chains;          /* chains, 1..64 (evaluated together in one pass)            */
  int32_t n_leapfrog;        /* leapfrog steps per trajectory, >= 1                        */
  int32_t n_warmup;          /* warmup iterations (not stored), >= 0                       */
  int32_t n_samples;         /* stored iterations, >= 0                                    */
  int32_t adapt;             /* 1: dual-averaging step-size adaptation during warmup       */
  float step_size;           /* initial (adapt) or fixed step size, > 0                    */
  float target_accept;       /* dual-averaging target delta in (0, 1) [0.8]                */
  float jitter;              /* relative step-size jitter in [0, 1)                        */
  double inv_mass[5];        /* diagonal inverse metric, every entry > 0                   */
  uint64_t seed;             /* Philox key                                                 */
  uint64_t uid_base;         /* chain uid = uid_base + chain                               */
  int32_t use_graph;         /* replay each trajectory from a captured HIP graph           */
  float* trace;              /* [device] float[n_chains][n_warmup + n_samples][4] or NULL,
                                as in bsi_hmc_cfg                                          */
} bsi_shear_hmc_cfg;

/*
 * bsi_shear_hmc -- phase 2 sampling: Hamiltonian Monte Carlo on
 * x = (g1, g2, mu_ln_s, sigma_ln_s, sigma_e) with potential
 * U(x) = -ln P(g, alpha | d) of bsi_shear_posterior (Section 3.4 samples the
 * shear and population parameters from this posterior; its gradient is the
 * softmax-weighted closed-form derivative of the log importance weights).
 * The iteration is that of bsi_hmc_sample (Philox4x32-10 momenta with the
 * same counters, float64 energies and Metropolis test, dual-averaging
 * warmup); position, momentum and energies are float64.  Every leapfrog step
 * evaluates all chains in one pass over the interim samples; the chain state
 * stays on the device for the whole call.
 *   e1p .. log10f, tp, interim   as for bsi_shear_posterior.
 *   init        [host] double[n_chains][5] start points (inside the support).
 *   samples     [device] double[n_chains][n_samples][5] or NULL.
 *   chain_stats [device] double[n_chains][4] = {accept rate over the stored
 *               iterations, final step size, divergent trajectories, ln P at
 *               the final position} or NULL.
 */
int bsi_shear_hmc(bsi_handle h, int32_t n_gal, int32_t K, const float* e1p, const float* e2p,
                  const float* log10s, const float* log10f, const bsi_true_prior* tp,
                  const bsi_interim* interim, const bsi_shear_hmc_cfg* cfg, const double* init,
                  double* samples, double* chain_stats, bsi_stream stream);

/* ---- Slot plans and their autotuning ---------------------------------------
 *
 * The k-space loop of a stamp side N walks the half-plane bins in pair-slots
 * (the bins (+kx, ky) and (-kx, ky) of one row per slot), as super-rows of R
 * rows spread over P iterations of the 64 lanes (the "slot plan"); P fixes R
 * and the padding.  By default each N uses the P with the fewest pair-slots.
 * A handle can hold another choice per N, set explicitly or measured by
 * bsi_autotune; every later call on the handle (and every request server
 * created afterwards) uses it.  Results do not depend on the plan beyond
 * float32 rounding (the order of the sums changes).  The trajectory kernel
 * runs several chains per wave on the plans 25: P 3, 41: P 1, 53: P 3
 * (exponential or Spergel profile, one wave per chain requested, an even
 * number of chains up to 4): four (16 lanes each, one wave per galaxy) for
 * fixed-length trajectories of exactly four chains (one exposure, white
 * noise), else two (32 lanes each); one chain per wave otherwise.  The choice
 * depends only on the size, plan and configuration, never on the batch. */

/* Set (P > 0) or reset to the default (P = 0) the slot plan of stamp side n.
 * BSI_EINVAL unless 8 <= n <= 128 and P is 0 or one of 1, 2, 3, 4, 5, 6, 8
 * with at least one row per super-row. */
int bsi_set_plan(bsi_handle h, int32_t n, int32_t P);

/* The slot plan stamp side n uses on this handle (*P), and its number of
 * bin slots per evaluation (*slots, nullable: two per pair-slot, padding
 * included). */
int bsi_get_plan(bsi_handle h, int32_t n, int32_t* P, int32_t* slots);

/* Measure, for each stamp side sizes[i], the trajectory kernel with each
 * candidate plan (those within 10 % of the fewest pair-slots, at most three) on a
 * synthetic batch that fills the device (about 16,384 chains of n_chains per
 * galaxy, exponential profile, 20 leapfrog steps, best of five launches),
 * and keep the fastest on the handle; the default plan is kept unless
 * another is at least 2 % faster.  chosen [host] int32[n_sizes] receives
 * the plans, ms [host] float[n_sizes] the measured milliseconds per launch
 * (both nullable).  Allocates and frees its own device buffers; synchronous. */
int bsi_autotune(bsi_handle h, int32_t n_sizes, const int32_t* sizes, int32_t n_chains,
                 int32_t* chosen, float* ms);

/* ---- Render transform per stamp side ------------------------------------
 *
 * bsi_render_stamps evaluates the spectrum on the half plane and transforms
 * it to pixels in one of two ways (results agree to float32 rounding, about
 * 1e-6 of the peak):
 *   BSI_TRANSFORM_DIRECT  direct DFT sums in float64 on the vector ALUs,
 *                         stamp, spectrum row and half-transform in LDS;
 *   BSI_TRANSFORM_MFMA    two dense DFT products (rows, then columns) on the
 *                         FP32 matrix cores (v_mfma_f32_16x16x4_f32), sizes
 *                         padded to tiles of 16, spectrum and half-transform
 *                         in LDS (the default).
 * The same choice applies to the forward transform of stamps (data, or data
 * minus model for BSI_LIK_PIXEL) at the likelihood's half-plane bins, done
 * per galaxy before sampling: direct FP32 sums, or two FP32 DFT products on
 * the matrix cores (sides whose LDS need exceeds 160 KiB use the direct
 * sums).  The k-space likelihood of the sampler needs no per-step transform. */
enum { BSI_TRANSFORM_DEFAULT = 0, BSI_TRANSFORM_DIRECT = 1, BSI_TRANSFORM_MFMA = 2 };

/* Set the render transform of stamp side n (8..128); DEFAULT resets it. */
int bsi_set_transform(bsi_handle h, int32_t n, int32_t method);

/* The transform stamp side n uses on this handle. */
int bsi_get_transform(bsi_handle h, int32_t n, int32_t* method);

/* Time, for a synthetic batch of n_gal galaxies of each side sizes[i]
 * (exponential profile, best of five), the render and the forward transform
 * of the stamps at the likelihood's bins with each method, and keep the
 * method with the smaller sum on the handle (it serves both directions).
 * chosen [host] int32[n_sizes] and ms [host] float[n_sizes][4] (render
 * direct, render MFMA, forward direct, forward MFMA; milliseconds per batch)
 * are nullable.  Allocates and frees its own device buffers; synchronous. */
int bsi_autotune_transform(bsi_handle h, int32_t n_sizes, const int32_t* sizes, int32_t n_gal,
                           int32_t* chosen, float* ms);

/* ---- Request serving: slot-based continuous batching of phase 1 ----------
 *
 * A server keeps the chains of many independent galaxy-fit requests resident
 * on the device.  Requests of any of the configured stamp sizes are admitted
 * while their device footprint fits in the server's HBM budget (a fixed part
 * per request -- chain states and stored samples -- plus the stamp and its
 * spectrum, carved from an arena); each bsi_slots_advance moves every
 * resident request forward by a number of HMC iterations, one launch per
 * stamp size, the sizes running concurrently; a request that has run
 * n_warmup + n_samples iterations (or, with an ESS target, reached it at a
 * check) is finished and is returned by bsi_slots_harvest, which frees its
 * slot and memory for new admissions.
 * Chain c of request `id` uses Philox counter uid id * n_chains + c, and the
 * iteration is exactly that of bsi_hmc_sample, so a request's samples do not
 * depend on which other requests share the device: with
 * uid_base = id * n_chains a one-galaxy bsi_hmc_sample call gives the same
 * samples.  A server is used from one host thread, with its handle, and
 * orders all its work on the stream given at creation. */
typedef struct bsi_slots_s* bsi_slots;

typedef struct {
  int32_t n_sizes;             /* number of stamp sizes served, 1..16                     */
  const int32_t* sizes;        /* [host] the stamp sides, 8..128, distinct                  */
  int64_t hbm_budget;          /* device bytes held by the server for request state, > 0    */
  int32_t max_slots;           /* resident-request limit; 0 = as many as the budget allows  */
  bsi_hmc_cfg hmc;             /* n_chains, n_leapfrog, n_warmup, n_samples, adapt, metric,
                                  step_size, target_accept, jitter and seed are used; form,
                                  iters_per_launch, use_graph, uid_base and trace are not   */
  bsi_interim interim;
  float pixel_scale;
  int32_t profile;             /* BSI_PROFILE_*                                             */
  float spergel_nu;            /* Spergel index (BSI_PROFILE_SPERGEL only)                  */
  int32_t pace;                /* 0: every size advances n_iter iterations per call;
                                  1: the slowest size advances n_iter and every other size
                                  about n_iter * tau_slowest / tau_N, tau the per-iteration
                                  time of a size's launch measured with events on earlier
                                  calls, so that the sizes' launches take about equally long */
  float ess_target;            /* 0: every request runs n_warmup + n_samples iterations.
                                  > 0: requests ask for this many effective samples: after
                                  n_warmup iterations a request is checked every ess_every
                                  draws (at ess_every, 2 ess_every, ...) and finishes at the
                                  first check where its effective sample size (multi-chain,
                                  mean over the six parameters, as bsi_ess computes it) is at
                                  least ess_target, else after n_samples draws.  A request's
                                  chains wait at each check until it has run (the check is
                                  enqueued by the same bsi_slots_advance), so the draws
                                  returned, like the samples, depend on the request alone    */
  int32_t ess_every;           /* draws between checks, >= 4 (used when ess_target > 0)     */
} bsi_slots_cfg;

typedef struct {
  uint64_t id;                 /* request id (chain uids id * n_chains + c)                 */
  int32_t n;                   /* stamp side, one of the configured sizes                   */
  const float* stamp;          /* [device] N * N floats, row-major; copied by the next
                                  bsi_slots_advance, so it must stay valid and unchanged
                                  until that call's work has run on the server's stream     */
  float psf_fwhm, sigma;       /* PSF FWHM [arcsec] and pixel noise sigma, > 0              */
  float ref_x, ref_y;          /* reference centroid, pixels from the stamp centre          */
  const float* init;           /* [host] float[n_chains][6] start positions (theta)         */
} bsi_request;

typedef struct {
  int32_t resident;            /* requests holding a slot (running or finished)             */
  int32_t finished;            /* of which finished and not yet harvested (as of the last
                                  poll when ess_target > 0)                                 */
  int32_t pending;             /* admitted since the last bsi_slots_advance                 */
  int32_t max_slots;
  int64_t budget;              /* bytes held (per-request arrays plus arena)                */
  int64_t slot_fixed_bytes;    /* per-request bytes independent of the stamp size           */
  int64_t arena_bytes, arena_free, arena_largest_free;
} bsi_slots_info;

/* Create a server on handle h (which must outlive it).  BSI_EINVAL when the
 * budget cannot hold one request of the largest size; BSI_EUNSUPPORTED when
 * a size with n_chains chains does not fit in LDS. */
int bsi_slots_create(bsi_handle h, const bsi_slots_cfg* cfg, bsi_stream stream, bsi_slots* out);

/* Wait for the server's work and release its device memory; NULL is ignored. */
void bsi_slots_destroy(bsi_slots s);

/* Device bytes request of side n would hold (fixed part plus stamp-dependent part). */
int bsi_slots_footprint(bsi_slots s, int32_t n, int64_t* bytes);

/* Admit request r if a slot is free and its footprint fits; *admitted = 1 if
 * so, 0 if the server is full (nothing changes then).  The request starts
 * running at the next bsi_slots_advance. */
int bsi_slots_admit(bsi_slots s, const bsi_request* r, int32_t* admitted);

/* Admit requests reqs[0..n-1] in order until one does not fit (first-come,
 * first-served: a request is never passed by a later one); *n_admitted
 * receives how many were admitted.  An invalid request fails the call with
 * the requests before it admitted. */
int bsi_slots_admit_many(bsi_slots s, int32_t n, const bsi_request* reqs, int32_t* n_admitted);

/* Enqueue n_iter >= 1 HMC iterations (scaled per size when cfg.pace is set)
 * for every resident, unfinished request
 * (admitted requests are first initialised: data spectrum, metric, start
 * potential).  Returns without waiting for the device. */
int bsi_slots_advance(bsi_slots s, int32_t n_iter);

/* Wait for the enqueued work and collect the requests that have finished;
 * *n_finished (nullable) receives the number finished and not yet handed out.
 * With ess_target > 0 this is how the host learns of finished requests (the
 * checks run on the device); bsi_slots_harvest polls by itself. */
int bsi_slots_poll(bsi_slots s, int32_t* n_finished);

/* Poll, then hand out up to max finished requests in the order they finished
 * (requests finishing in the same bsi_slots_advance in admission order) and
 * free their slots:
 *   ids          [host] uint64[max]
 *   samples      [device] float[max][n_chains][n_samples][6] (theta) or NULL;
 *                draws past a request's n_draws are NaN
 *   chain_stats  [device] float[max][n_chains][4] as in bsi_hmc_sample over the
 *                request's n_draws draws, or NULL
 *   status       [device] uint32[max] (BSI_STATUS_* bits) or NULL
 *   n_draws      [device] int32[max] draws per chain returned, or NULL
 *                (n_samples unless ess_target > 0)
 * *n_out receives the number handed out.  Outputs are complete on return. */
int bsi_slots_harvest(bsi_slots s, int32_t max, uint64_t* ids, float* samples,
                      float* chain_stats, uint32_t* status, int32_t* n_draws, int32_t* n_out);

/* Occupancy and memory of the server. */
int bsi_slots_get_info(bsi_slots s, bsi_slots_info* info);

/*
 * bsi_ess -- diagnostics of Section 4.1 for stored samples:
 * multi-chain effective sample size per parameter (autocorrelation with
 * Geyer's initial monotone sequence, no rank normalisation), the classic
 * potential scale reduction R-hat of the R-hat < 1.01 convergence test, and
 * its split form (each chain cut into its first and last floor(n_samples/2)
 * draws, the middle draw of an odd count dropped; the classic statistic over
 * the 2 n_chains halves), which also flags chains that drift.
 *   samples    [device] float[n_gal][n_chains][n_samples][n_par].
 *   ess        [device] float[n_gal][n_par] or NULL.
 *   rhat       [device] float[n_gal][n_par] or NULL.
 *   rhat_split [device] float[n_gal][n_par] or NULL.
 * At least one output must be non-NULL; n_samples >= 4, n_chains <= 16 and
 * n_chains * n_samples * 8 bytes within the LDS stage (else BSI_EUNSUPPORTED).
 */
int bsi_ess(bsi_handle h, int32_t n_gal, int32_t n_chains, int32_t n_samples, int32_t n_par,
            const float* samples, float* ess, float* rhat, float* rhat_split, bsi_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* BSI_H */
