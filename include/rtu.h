/*
 * rtu.h -- C ABI of the MI355X (gfx950) library for the ray-guided
 * transformed uniform (RTU) grid lens likelihood and its gradient.
 *
 * The method (Enzi et al., "Gaussian processes on ray-guided transformed
 * uniform grids"): supersampled image-plane rays are traced through a lens
 * (SIE + external shear + optional NFW subhaloes, App. A eqs. A1-A3), the
 * source-plane coordinates are mapped through a smoothed marginal CDF built
 * from the arc-masked rays (Sec. 2.2 eq. 5, App. C), the source is a
 * Gaussian process drawn in Fourier space on a uniform grid (Sec. 2.1,
 * eqs. 1-4) and evaluated by bilinear interpolation, the sub-rays of each
 * pixel are averaged, the image is convolved with the PSF and compared to the
 * data with a Gaussian likelihood (Sec. 3.1, Sec. 4).
 *
 * Conventions used by every entry point:
 *  - Return value: 0 on success, a negative RTU_E* code on misuse detected
 *    on the host.  No entry point synchronises the device unless its comment
 *    says so.  Numerical conditions of a sample are reported in its device
 *    status word (RTU_ST_* bits), never as a return code.
 *  - "device" pointers are allocations on the plan's device (hipMalloc or a
 *    torch CUDA tensor), contiguous, row-major, owned by the caller, and
 *    must stay valid until the work queued on the stream has finished.
 *  - "host" pointers are read during the call only.
 *  - stream is a hipStream_t passed as void*; NULL means the null stream.
 *  - A plan is not thread-safe: use one plan per stream.
 *
 * Image pixel (i, j) (row i <-> y, column j <-> x) is centred at
 * ((j - (N-1)/2) d, (i - (N-1)/2) d) arcsec, d = pixel_scale; its ss x ss
 * sub-rays sit on a regular lattice centred in the pixel.  Source grid node
 * (i, j) sits at ((j + 1/2)/n, (i + 1/2)/n) of the unit square of the
 * transformed coordinates; brightness outside the grid is zero (Sec. 2.1).
 */
#ifndef RTU_H
#define RTU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---------------------------------------------------- */
#define RTU_OK        0
#define RTU_EINVAL   -1   /* bad geometry or argument                         */
#define RTU_ENOMEM   -2   /* device allocation failed / budget exceeded       */
#define RTU_EBATCH   -3   /* batch larger than the plan's max_batch           */
#define RTU_EHIP     -4   /* a HIP runtime call or kernel launch failed        */
#define RTU_ESTATE   -5   /* call out of order (e.g. no observation set)      */
#define RTU_ENOTFOUND -6  /* unknown fit id                                   */
#define RTU_ETOOBIG  -7   /* more than the static scratch array holds          */

/* ---- per-sample status bits (device uint32 words) -------------------- */
#define RTU_ST_NONFINITE    1u  /* loss or a gradient is not finite                    */
#define RTU_ST_NONMONOTONE  2u  /* QF slope p'(u_k) <= eps or tied knots: slopes clamped */
#define RTU_ST_MASK_SMALL   4u  /* fewer masked pixels than nodes + 1 (uniform grid:
                                   fewer than 2, or a box of zero size)              */
#define RTU_ST_DOMAIN       8u  /* theta_E <= 0, |e| >= 1, r_s <= 0 or spectrum <= 0   */

/* Number of Chebyshev nodes of the quantile-function fit: degree 21 + 1
 * (App. C step iii and Fig. C1). */
#define RTU_K_NODES 22
/* Lens parameters: theta_E, e1, e2, x0, y0, gamma1, gamma2 (SIE + external
 * shear; with RTU_GEOM_EPL also the slope gamma of the elliptical power law,
 * App. A.1, eq. A1), then per subhalo kappa_s, r_s, x_s, y_s (App. A), then
 * per lens-light Gaussian
 * A, sigma, e1, e2, x_c, y_c (App. A, Multi Gaussian Expansion: the
 * component adds A/(2 pi) exp(-rho^2/(2 sigma^2)) to every sub-ray, with
 * rho^2 = q x'^2 + y'^2/q about (x_c, y_c) and q, angle from (e1, e2) as for
 * the mass).  Power-spectrum parameters: sigma_src, n_src, zeta_src,
 * alpha_src (eqs. 3-4). */
#define RTU_N_LENS_BASE 7
#define RTU_N_LENS_BASE_EPL 8
#define RTU_N_PER_SUB   4
#define RTU_N_PER_GAUSS 6
#define RTU_N_PS        4
#define RTU_MAX_SUB    10
#define RTU_MAX_GAUSS   8
#define RTU_MAX_LENS   (RTU_N_LENS_BASE_EPL + RTU_N_PER_SUB * RTU_MAX_SUB + RTU_N_PER_GAUSS * RTU_MAX_GAUSS)

typedef struct rtu_plan_s* rtu_plan;

typedef struct {
  int32_t  n_img;        /* image pixels per side, 8..1024                          */
  int32_t  supersample;  /* sub-rays per pixel per axis, 1..8                        */
  int32_t  n_src;        /* source grid pixels per side: power of two, 8..256        */
  int32_t  psf_size;     /* odd PSF width, 1..63                                    */
  int32_t  n_sub_max;    /* NFW subhalo slots per sample, 0..RTU_MAX_SUB            */
  int32_t  k_nodes;      /* must be RTU_K_NODES                                     */
  float    pixel_scale;  /* arcsec per image pixel, > 0                             */
  float    tnfw_tau;     /* subhalo projected-mass truncation in units of r_s;
                            0 = untruncated NFW                                     */
  uint32_t flags;        /* RTU_GEOM_* bits                                         */
  int32_t  n_gauss;      /* lens-light Gaussians per sample, 0..RTU_MAX_GAUSS
                            (0 = no lens light)                                     */
} rtu_geometry;

/* Geometry flag: select the quantile order statistics with the bounded-pass
 * radix select for every sample, instead of only where the value-linear
 * histogram cannot separate the target ranks.  Both selections return the
 * same rays (ties by index); the flag exists to exercise the fallback. */
#define RTU_GEOM_RADIX_SELECT 1u
/* Geometry flag: the uniform grid of Sec. 2.1 instead of the RTU grid.  The
 * source grid spans the smallest square box that holds the masked rays (pixel
 * centres, not supersampled): its side L is the larger of the two coordinate
 * ranges (x on a tie) and it is centred on the rays' range along both axes;
 * a ray maps to y = (beta - lo) / L.  The extremes are the masked rays of
 * rank 0 and M - 1 (ties by ray index) and the gradient flows through them
 * as selections.  Fewer than two masked rays, or zero ranges: status bit
 * RTU_ST_MASK_SMALL and a box of side 1 at the rays' minimum.  In this mode
 * RTU_DBG_SELECT holds per axis the indices of the minimum and the maximum in
 * its first two slots, RTU_DBG_STD (lo_x, lo_y, L), and RTU_DBG_KNOTS zeros. */
#define RTU_GEOM_UNIFORM 2u
/* Geometry flag: the main deflector is the elliptical power law of App. A.1,
 * eq. (A1), kappa = (3 - gamma)/2 (theta_E/rho)^(gamma - 1) with rho^2 =
 * q x'^2 + y'^2/q, whose slope gamma (in (1, 3); status RTU_ST_DOMAIN
 * outside) is lens parameter 7, the subhaloes and lens light following
 * (RTU_N_LENS_BASE_EPL parameters before the subhaloes).  Its deflection is
 * the hypergeometric series of Tessore & Metcalf (2015), summed to FP32
 * precision with at most 48 terms (|e| <= 0.68 reaches it), and gamma gets
 * its gradient.  At gamma = 2 it is the SIE. */
#define RTU_GEOM_EPL 4u

/* Number of lens parameters per sample: 7 + 4 n_sub_max + 6 n_gauss. */
int32_t rtu_n_lens(const rtu_geometry* g);

/* Device memory (bytes) a plan of this geometry and batch allocates; a
 * serving layer uses it for admission.  0 if the geometry is invalid. */
size_t rtu_workspace_bytes(const rtu_geometry* g, int32_t max_batch);

/* Creates a plan on `device` for batches of up to max_batch samples and
 * allocates all of its device memory once.  Returns RTU_EINVAL for a bad
 * geometry, RTU_ENOMEM if the allocation fails.  *out is set on success. */
int rtu_plan_create(const rtu_geometry* g, int32_t max_batch, int32_t device, rtu_plan* out);

/* Frees the plan and its device memory (synchronises the plan's device). */
int rtu_plan_destroy(rtu_plan p);

/* Observation of one lens system (host arrays, read during the call only):
 * image[N*N] and noise_sigma[N*N] (sigma > 0) in data units, psf[K*K]
 * (applied as given, not renormalised), arc_mask[N*N] (nonzero = pixel
 * used to build the RTU grid; Sec. 2.2, the rays are traced from the
 * observed pixel centres, not supersampled).  Builds the masked pixel list
 * and the quantile ranks (h = (M-1) u_k, in FP64) on the host, stages them
 * with the observation in the plan's pinned buffer and queues one copy to the
 * device on `stream`: evaluations queued after it on the same stream see the
 * new observation.  No device-wide synchronisation; the call waits only, if
 * the previous call's copy out of the staging buffer has not finished yet,
 * for that copy.  The device region was sized for any mask when the plan was
 * created, so nothing is reallocated.  RTU_EINVAL if a pointer is NULL. */
int rtu_set_observation(rtu_plan p, const float* image, const float* noise_sigma,
                        const float* psf, const uint8_t* arc_mask, void* stream);

/* Number of masked pixels M of the current observation (-1 if none). */
int32_t rtu_masked_count(rtu_plan p);

/* Weighted RTU grid (Sec. 6.3, "Extension to weighted RTU grid"): per-pixel
 * weights of the masked rays when the eCDFs are built (for example the
 * observed brightness or SNR), host float [n_img][n_img]; only masked pixels
 * are read.  A weight counts rays: a masked ray of weight w stands for w
 * rays, so integer weights give the quantiles of the rays repeated that many
 * times and unit weights the unweighted grid; with W the total weight, the
 * order statistic at cumulative-weight position r is the ray whose interval
 * of the weights summed in sorted order (ties by ray index) holds r, the
 * quantile at node u_k interpolates linearly between positions
 * floor((W-1) u_k) and that + 1, and the standardisation uses weighted
 * moments.  The weights are constants (no gradient).  RTU_EINVAL for a
 * negative or non-finite weight or W < 1; RTU_ESTATE before
 * rtu_set_observation.  NULL restores the unweighted grid; a new observation
 * drops the weights.  The copy is queued on `stream` through a pinned buffer
 * (no device-wide sync unless the scratch array must grow).  Not available
 * in rtu_loss_grad_noalloc and the fleet. */
int rtu_set_ray_weights(rtu_plan p, const float* weights, void* stream);

/* ---- allocation-free evaluation ----------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as rtu_loss_grad with no plan (equal bit for bit below 8192
 * masked pixels; above, a plan sums the masked rays' moments in another
 * order, and the two agree to rounding).  The geometry comes by value
 * (host), the observation as device arrays in rtu_set_observation's layout
 * (image[N*N], noise_sigma[N*N], psf[K*K], arc_mask[N*N] uint8), and the
 * per-sample inputs and outputs as for rtu_loss_grad.  Every intermediate
 * (the observation's tables, prepared on the device by this call, and the
 * evaluation's workspace) lives in a static device array of
 * RTU_NOALLOC_MAX_BYTES that each GPU the library runs on holds until the
 * process ends; nothing is allocated or freed and nothing is synchronised.
 * Queued on `stream` on the current device.  The first call on a device does
 * the library's set-up there (constant tables, the array's address) and must
 * not be captured into a graph.  Every call on a device shares that device's
 * array: calls that overlap on one device (other streams, other threads)
 * race and must be ordered by the caller.  RTU_ETOOBIG if the geometry and
 * batch need more than the array (C2 at 32 samples fits); RTU_EINVAL as for
 * rtu_loss_grad. */
#define RTU_NOALLOC_MAX_BYTES ((size_t)64 << 20)
int rtu_loss_grad_noalloc(const rtu_geometry* g, int32_t batch, const float* image,
                          const float* noise_sigma, const float* psf, const uint8_t* arc_mask,
                          const float* lens_params, const int32_t* n_sub, const float* ps_params,
                          const float* latent, double* loss, double* chi2_mask, float* grad_lens,
                          float* grad_ps, float* grad_latent, float* model_image, uint32_t* status,
                          void* stream);

/* One loss evaluation per sample, and its gradient, for `batch` samples.
 *   lens_params [B][rtu_n_lens(g)]    device, see RTU_N_LENS_BASE
 *   n_sub       [B] device int32, number of active subhaloes (<= n_sub_max),
 *               or NULL for none
 *   ps_params   [B][4]                device
 *   latent      [B][n_src][n_src]     device, 16-byte aligned, the white-noise
 *               field w of eq. 1
 * Outputs (device; any may be NULL except loss and status):
 *   loss        [B] double: chi^2/2 + |w|^2/2, chi^2 over all pixels
 *   chi2_mask   [B] double: mean of ((m - d)/sigma)^2 over the masked pixels
 *   grad_lens   [B][rtu_n_lens(g)], grad_ps [B][4], grad_latent [B][n_src^2]
 *               d loss / d parameters; if all three are NULL only the forward
 *               pass runs.  Gradient slots of inactive subhaloes are zero.
 *   model_image [B][n_img][n_img]: PSF-convolved model
 *   status      [B] uint32 RTU_ST_* bits of each sample
 * Asynchronous on `stream`.  RTU_ESTATE without an observation, RTU_EBATCH
 * if batch > max_batch, RTU_EINVAL for NULL required pointers or a latent
 * pointer that is not 16-byte aligned. */
int rtu_loss_grad(rtu_plan p, int32_t batch,
                  const float* lens_params, const int32_t* n_sub,
                  const float* ps_params, const float* latent,
                  double* loss, double* chi2_mask,
                  float* grad_lens, float* grad_ps, float* grad_latent,
                  float* model_image, uint32_t* status, void* stream);

/* Intermediates of the last rtu_loss_grad call, copied to host memory for
 * inspection (synchronises `stream`).  `what` selects:
 *   RTU_DBG_KNOTS   float[2][2][K]: per axis, knots X_k then slopes S_k of the
 *                   smoothed CDF in standardised units (App. C steps i-iv)
 *   RTU_DBG_SELECT  int32[2][2][K]: per axis, masked-ray index of the order
 *                   statistics at floor(h_k) and floor(h_k)+1
 *   RTU_DBG_STD     double[3]: mean x, mean y, scale s of the masked rays
 *   RTU_DBG_SOURCE  float[n_src^2]: source grid s (eq. 3)
 *   RTU_DBG_PREPSF  float[N^2]: sub-ray mean image before the PSF
 *   RTU_DBG_ONGRID  double[1]: number of sub-rays whose bilinear footprint
 *                   touches the zero-bordered source grid (the ones with a
 *                   nonzero adjoint), as the gradient pass counted them;
 *                   RTU_ESTATE if the last call computed no gradient
 * RTU_EINVAL if `bytes` is smaller than the item. */
#define RTU_DBG_KNOTS  1
#define RTU_DBG_SELECT 2
#define RTU_DBG_STD    3
#define RTU_DBG_SOURCE 4
#define RTU_DBG_PREPSF 5
#define RTU_DBG_ONGRID 6
int rtu_debug_fetch(rtu_plan p, int32_t what, int32_t sample, void* host_dst, size_t bytes,
                    void* stream);

/* ---- stage timing ------------------------------------------------------
 * Stages of one evaluation / fit step, in launch order. */
#define RTU_STAGE_PREP      0   /* masked rays, quantiles, CDF knots; GP source   */
#define RTU_STAGE_RAYS_FWD  1   /* supersampled rays -> pre-PSF image             */
#define RTU_STAGE_PSF_FWD   2   /* PSF, residual, chi^2 partials                  */
#define RTU_STAGE_PSF_ADJ   3   /* PSF adjoint                                    */
#define RTU_STAGE_RAYS_ADJ  4   /* ray adjoint: source, knot, lens gradients      */
#define RTU_STAGE_POST      5   /* knot adjoint, reductions, GP adjoint           */
#define RTU_STAGE_SAMPLE    6   /* fit: draw z = mu + exp(rho) eps (first step,
                                       restored state, given draws; else in ADAM) */
#define RTU_STAGE_ADAM      7   /* fit: ELBO value and Adam update                */
#define RTU_N_STAGES        8

/* Start recording HIP events around the stages selected by stage_mask (bit
 * k = stage k; 0 = every stage) of the next max_calls evaluations
 * (rtu_loss_grad or fit steps) of this plan, on the stream each evaluation
 * runs on.  Recording adds no synchronisation, but every event is a marker
 * in the stream: select only the stages to be timed. */
int rtu_profile_begin(rtu_plan p, int32_t max_calls, uint32_t stage_mask);
/* Stop recording; wait for the recorded events and return, per stage, the
 * summed GPU time in milliseconds (stage_ms[RTU_N_STAGES], host) and the
 * number of recorded launches of each stage (launches[RTU_N_STAGES], host,
 * may be NULL).  Synchronises the recorded events. */
int rtu_profile_end(rtu_plan p, double* stage_ms, int32_t* launches);

/* ---- stochastic variational fit (Sec. 4) -------------------------------
 * A mean-field Gaussian guide over z = (lens[n_lens], ps[4], latent[n_src^2])
 * with location mu and scale exp(rho).  One step draws S samples
 * z_s = mu + exp(rho) eps_s (eps from a counter-based Philox4x32-10 stream
 * keyed by the seed, or given), evaluates the loss and gradient of every
 * sample on the plan, records the ELBO estimate
 *   -mean_s loss_s - sum_p ln(sigma_p sqrt(2 pi)) - (n_src^2/2) ln 2 pi
 *   + sum(rho) + (dim/2)(1 + ln 2 pi)
 * (Gaussian likelihood, flat priors on lens and spectrum parameters, unit
 * normal prior on the latent) and takes one Adam step (beta 0.9, 0.999,
 * epsilon 1e-8) on (mu, rho) to maximise it.  State stays on the device. */
typedef struct rtu_fit_s* rtu_fit;

/* Lens and power-spectrum parameters whose guide lives in log space, as a
 * bit mask over the index i into (lens, ps) (word i / 32, bit i % 32; i <
 * n_lens + 4): their sample is z = exp(u), u = mu + exp(rho) eps, the
 * gradient is chained through z, and the prior is flat in u (log-uniform in
 * z; for positive parameters such as a subhalo's kappa_s and r_s or the
 * spectrum's sigma and zeta, which then never reach zero).  mu and rho of
 * such a parameter are those of u.  Bits at latent indices are ignored. */
#define RTU_LOG_MASK_WORDS 3

/* Creates a fit on plan p (which must hold an observation) with S samples per
 * step (S <= the plan's max_batch), initial guide mu0, rho0 (host, [dim]),
 * learning rate lr, Philox seed, room for max_steps ELBO values, n_sub
 * active subhaloes and the log-space mask (host [RTU_LOG_MASK_WORDS], or NULL
 * for none).  dim = n_lens + 4 + n_src^2. */
int rtu_fit_create(rtu_plan p, int32_t samples, const float* mu0, const float* rho0, float lr,
                   uint64_t seed, int32_t max_steps, int32_t n_sub, const uint32_t* log_mask, rtu_fit* out);
int rtu_fit_destroy(rtu_fit f);
int32_t rtu_fit_dim(rtu_fit f);
/* Queues n_steps fit steps on `stream`.  eps (device, [n_steps][S][dim]) or
 * NULL to draw from Philox.  RTU_EINVAL if the trace would overflow. */
int rtu_fit_step(rtu_fit f, int32_t n_steps, const float* eps, void* stream);
/* Copies the guide (host mu[dim], rho[dim], either may be NULL), the ELBO
 * trace (host elbo[max_trace]) and the OR of every sample's status word over
 * every step taken (host *status, may be NULL) out; *n_trace = steps taken.
 * Synchronises `stream`. */
int rtu_fit_read(rtu_fit f, float* mu, float* rho, double* elbo, int32_t max_trace,
                 int32_t* n_trace, uint32_t* status, void* stream);
/* Checkpoint / resume: the full optimiser state as host float[6][dim] in the
 * order mu, rho, Adam m(mu), v(mu), m(rho), v(rho), plus the number of steps
 * taken (the Philox counter and Adam's bias correction continue from it).
 * get synchronises `stream`; set is synchronous. */
int rtu_fit_get_state(rtu_fit f, float* state, int32_t* steps, void* stream);
int rtu_fit_set_state(rtu_fit f, const float* state, int32_t steps);

/* Copies the fit's sample buffers z_s to host z[S][dim] (synchronises
 * `stream`): after a step with given draws, that step's samples; with Philox
 * draws the Adam update of a step already draws the next step's samples (so
 * that no separate sampling launch is needed), and the buffers hold those. */
int rtu_fit_samples(rtu_fit f, float* z, void* stream);

/* Device pointers of the last step's per-sample loss [S] (double) and status
 * [S] (uint32), valid until the fit is destroyed. */
int rtu_fit_last_outputs(rtu_fit f, const double** loss, const uint32_t** status);

/* ---- serving: many fits in shared launches ------------------------------
 * A fleet owns one HBM arena of a fixed budget.  Requests (a lens system and
 * the settings of its variational fit) queue in arrival order and are
 * admitted, first come first served, whenever the arena and a slot have room
 * for the head of the queue.  Every round advances every admitted fit by one
 * ELBO + Adam step (rtu_fit_* semantics) in one set of kernel launches shared
 * by all of them, whatever their image, source or PSF sizes; each fit keeps its
 * optimiser state on the device.  A fit that has taken its steps is retired at
 * the next sync point (results copied to the host, memory returned), and
 * queued requests are admitted there.  Sync points happen at most every
 * sync_every rounds, or whenever no admitted fit has steps left. */
typedef struct rtu_fleet_s* rtu_fleet;

typedef struct {
  rtu_geometry geom;
  const float* image;        /* host [N*N] */
  const float* noise_sigma;  /* host [N*N] */
  const float* psf;          /* host [K*K] */
  const uint8_t* arc_mask;   /* host [N*N] */
  const float* mu0;          /* host [dim], dim = n_lens + 4 + n_src^2 */
  const float* rho0;         /* host [dim] */
  int32_t samples;           /* S per step */
  int32_t steps;             /* ELBO steps of the fit */
  int32_t n_sub;             /* active subhaloes (<= geom.n_sub_max) */
  float lr;
  uint64_t seed;             /* Philox key of the fit's draws */
  uint32_t log_mask[RTU_LOG_MASK_WORDS];  /* log-space lens parameters (see rtu_fit_create) */
} rtu_fit_request;

/* Creates a fleet on `device` with an arena of hbm_budget bytes and at most
 * max_fits fits admitted at once. */
int rtu_fleet_create(int32_t device, size_t hbm_budget, int32_t max_fits, int32_t sync_every, rtu_fleet* out);
int rtu_fleet_destroy(rtu_fleet f);
/* Arena bytes the request needs once admitted (0 if it is invalid). */
size_t rtu_fleet_request_bytes(const rtu_fit_request* r);
/* Queues a request; its host arrays are copied.  *ticket identifies it.
 * RTU_EINVAL for a bad request, RTU_ENOMEM if it can never fit the budget. */
int rtu_fleet_submit(rtu_fleet f, const rtu_fit_request* r, int64_t* ticket);
/* Queues up to `rounds` rounds on `stream` (sync points, which wait for the
 * stream, happen inside as described above).  Returns early when no fit has
 * steps left and none can be admitted. */
int rtu_fleet_run(rtu_fleet f, int32_t rounds, void* stream);
/* Forces a sync point now: waits for `stream`, retires finished fits, admits. */
int rtu_fleet_sync(rtu_fleet f, void* stream);
/* Tickets of fits retired since the last poll (host, up to max). */
int rtu_fleet_poll(rtu_fleet f, int64_t* tickets, int32_t max, int32_t* n);
/* Result of a retired fit (host copies; any pointer may be NULL), then forgets
 * it: guide mu[dim], rho[dim], ELBO per step elbo[max_trace] (*n_trace = steps),
 * and the OR of all its samples' status words.  RTU_ENOTFOUND if unknown. */
int rtu_fleet_result(rtu_fleet f, int64_t ticket, float* mu, float* rho, double* elbo, int32_t max_trace,
                     int32_t* n_trace, uint32_t* status);
/* Admitted fits, queued requests, arena bytes in use, rounds run. */
int rtu_fleet_stats(rtu_fleet f, int32_t* active, int32_t* queued, size_t* bytes_in_use, int64_t* rounds);

/* Human-readable text of a return code. */
const char* rtu_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* RTU_H */
