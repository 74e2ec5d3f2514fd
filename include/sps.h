/*
 * sps.h -- C ABI of the MI355X (gfx950) SPS photometry / likelihood / HMC library.
 *
 * Implements the per-galaxy forward model of "Bayesian Posteriors with Stellar
 * Population Synthesis on GPUs" (Zacharegkas, Hearin & Benson):
 *   SSP weights from the star-formation history and metallicity distribution
 *     (App. A.1 Eqs. totalMstarFormed, SFRsmooth, smoothPsfh, composite age
 *      weights, triweight; App. A.2),
 *   dust attenuation (App. A.3, Eq. DustAtt and the unobscured floor),
 *   exact photometry (Sec. 3, Eq. photo_integral_exact),
 *   approximate photometry with a precomputed SSP x band table interpolated in
 *     redshift (Sec. 3, Eqs. lambda_eff and photo_integral_approx),
 *   the Gaussian photometric log-likelihood and its gradient (App. D.1), and
 *   batched HMC chains on the unbounded parameters (Sec. 4; App. C bounding
 *     function and skew-normal prior; App. D.2).
 *
 * Conventions
 *  - Every array argument of a compute call is a DEVICE pointer on the
 *    context's device, contiguous, owned by the caller.  The library never
 *    frees or retains them.
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Calls
 *    enqueue work and return without synchronising, except where stated.
 *  - Parameters are structure-of-arrays: params[p * n_gal + g], p = 0..9 in
 *    this slot order (physical units):
 *      0 log10 M_formed [Msun]   1 tau [Gyr] (DPL) | t_peak [Gyr] (log-normal)
 *      2 alpha (DPL) | width w (log-normal, natural-log units)
 *      3 beta (DPL) | unused     4 F_burst     5 log10 T_peak [yr]
 *      6 mu_logZ                 7 tau_V       8 delta       9 F_floor
 *  - Magnitudes, observations and sigmas are [n_gal][n_band] row-major.
 *  - Return value: SPS_OK or an error code; sps_last_error() gives a
 *    thread-local message.  Invalid sizes, enums or NULL required pointers are
 *    errors.  NaN parameters propagate to NaN outputs and are not errors.  A
 *    redshift outside the context's z table gives NaN outputs for that galaxy
 *    on the approximate path and sets a device-side flag that the next
 *    sps_status call reports as SPS_E_RANGE (the compute call itself does not
 *    synchronise to find out).
 *  - Compute calls never allocate device memory: the context's workspaces are
 *    sized by sps_create / sps_reserve (approximate path, HMC chain state) and
 *    sps_reserve_exact (exact path); a call larger than they allow returns
 *    SPS_E_STATE (or SPS_E_INVAL for n_gal above the reserved galaxy count).
 *  - Calls on one context from several host threads must be serialised by the
 *    caller; work enqueued on different streams must not overlap in time when
 *    it uses the context's internal workspace (all compute calls do).
 */
#ifndef SPS_H
#define SPS_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define SPS_NPARAM 10
#define SPS_MAX_BAND 8

enum {
    SPS_OK = 0,
    SPS_E_INVAL = 1,   /* bad argument: size, enum, NULL pointer, unsupported grid */
    SPS_E_RANGE = 2,   /* value outside a supported range (e.g. z table bounds)   */
    SPS_E_NOMEM = 3,   /* device allocation failed                                */
    SPS_E_HIP = 4,     /* HIP runtime error                                       */
    SPS_E_STATE = 5    /* call out of order (e.g. no z table built yet)           */
};

typedef enum { SPS_F64 = 0, SPS_F32 = 1, SPS_BF16X = 2 } sps_prec;   /* exact-path arithmetic */
typedef enum { SPS_SFH_LOGNORMAL = 0, SPS_SFH_DPL = 1 } sps_sfh;
typedef enum { SPS_PATH_APPROX = 0, SPS_PATH_EXACT = 1 } sps_path;

/* Host FP64 descriptors, copied (and uploaded) at sps_create. */
typedef struct {
    int n_met, n_age, n_wave;
    const double *log10_met;     /* [n_met] increasing, log10 Z/Zsun                    */
    const double *log10_age_yr;  /* [n_age] increasing, log10 age / yr                 */
    const double *wave_A;        /* [n_wave] increasing rest-frame wavelength, Angstrom */
    const double *lum;           /* [n_met][n_age][n_wave] Lsun / A per Msun formed     */
} sps_ssp_desc;

typedef struct {
    int n_band;                  /* 1 .. SPS_MAX_BAND                                   */
    const double *center_A;      /* Gaussian transmission T(l) = exp(-(l-c)^2/(2 s^2)), */
    const double *sigma_A;       /* observed frame, peak 1                              */
} sps_filter_desc;

typedef struct {
    double H0;          /* km/s/Mpc, flat LCDM with matter + Lambda (e.g. 70)          */
    double Om;          /* matter density (e.g. 0.3)                                   */
    double sigma_logz;  /* width of the log-normal metallicity distribution, dex (0.2) */
    double burst_dlogt; /* log10 T_max - log10 T_peak of the triweight burst, dex (0.3) */
} sps_model_desc;

typedef struct sps_ctx sps_ctx;

/* Create a context on `device`: uploads the SSP grid (FP64 always; FP32 if
 * prec_mask has bit 1<<SPS_F32; BF16 hi+lo pair if bit 1<<SPS_BF16X), the
 * wavelength quadrature weights and the filter constants, and reserves
 * workspace for up to max_gal galaxies.  Supported SSP grid: n_age = 94,
 * n_met = 12 (compile-time register tiles); n_band <= 8.  On error *out is NULL. */
int sps_create(sps_ctx **out, int device, const sps_ssp_desc *ssp, const sps_filter_desc *filters,
               const sps_model_desc *model, unsigned prec_mask, int max_gal);

/* Grow the per-galaxy workspace to max_gal galaxies: the approximate path's records
 * (140 B per galaxy) and the approximate-path HMC's chain state for max_gal chain slots
 * (n_gal * n_chain; about 470 B per slot with its trajectory scratch).  Synchronises the
 * device; never shrinks. */
int sps_reserve(sps_ctx *ctx, int max_gal);

/* Size the exact path's workspace for calls of up to max_rows galaxies (or exact-path HMC
 * chains, n_gal * n_chain), for every precision uploaded at create, with the gradient:
 * the weights rows, partial band sums, Rbar and Wbar of the two GEMMs (about 34 KB per
 * row at 2000 wavelengths and 50 KB at 5000), the z-order buffer from 16,384 rows on, and
 * the exact-path HMC's chain state (~0.6 KB per chain).  Also grows
 * sps_reserve's galaxy count to max_rows.  Synchronises the device; never shrinks. */
int sps_reserve_exact(sps_ctx *ctx, int max_rows);

/* Synchronises the device, then reports and clears the device-side error flags raised by
 * compute calls since the last sps_status: SPS_E_STATE if an HMC resume blob did not match
 * its run, else SPS_E_RANGE if a redshift outside the z table reached the approximate
 * path, else SPS_OK. */
int sps_status(sps_ctx *ctx);

/* Build the SSP x band flux table c_SSP(z) on n_z uniform nodes in [z_lo, z_hi]
 * (Sec. 3, the precomputed c_SSP lookup table after Eq. photo_integral_approx).  Stored distance-free
 * and divided by the band normalisation: Q[k][b][j][i] =
 *   sum_l L[j][i][l] T_b((1+z_k) l) l q_l / sum_l T_b((1+z_k) l) q_l / l
 * with trapezoid weights q_l on the SSP wavelength grid; FP64 arithmetic,
 * FP32 storage.  Synchronises the device.  2 <= n_z <= 1024. */
int sps_build_ztable(sps_ctx *ctx, int n_z, double z_lo, double z_hi);

/* Copy the z table to host memory q[n_z][n_band][n_met][n_age] (FP32). */
int sps_get_ztable(sps_ctx *ctx, float *q_host);

void sps_destroy(sps_ctx *ctx);
const char *sps_last_error(void);

/* Instrumentation of the approximate path's model kernel (no part of the model).  With
 * n_pairs > 0 every later approximate-path call (sps_phot_approx, sps_loglike_grad with
 * SPS_PATH_APPROX, sps_logpost_grad) records a pair of HIP events on its stream right before
 * and after that kernel, cycling through n_pairs pairs; 0 turns this off and frees the
 * events.  Calls cost one extra event pair each while on.  n_pairs <= 4096. */
int sps_set_kernel_timing(sps_ctx *ctx, int n_pairs);

/* Elapsed milliseconds of the last min(n_pairs, calls since timing was set) recorded
 * launches, oldest first, into ms_out[0 .. max) (waits for those events); *count receives
 * the number written.  SPS_E_INVAL if timing is off. */
int sps_kernel_times(sps_ctx *ctx, float *ms_out, int max, int *count);

/* SSP weights W[g][j][i] = M_formed P_met(j) P_age(i) (Eq. galSED_decomposed;
 * sums to 10^params[0]).  params [10][n_gal], z [n_gal], w_out [n_gal][n_met][n_age]. */
int sps_weights(sps_ctx *ctx, void *stream, int n_gal, int sfh, const float *params, const float *z,
                float *w_out);

/* Approximate AB magnitudes (Eq. photo_integral_approx; attenuation evaluated at
 * the rest-frame effective wavelength, table interpolated linearly in z, in
 * flux).  Needs a z table.  mag_out [n_gal][n_band] FP32. */
int sps_phot_approx(sps_ctx *ctx, void *stream, int n_gal, int sfh, const float *params,
                    const float *z, float *mag_out);

/* Exact AB magnitudes (Eq. photo_integral_exact): dense (galaxies x SSPs) x
 * (SSPs x wavelengths) contraction on MFMA with the attenuation x redshifted
 * filter x quadrature weight applied in the epilogue.  prec = SPS_F64:
 * params/z/mag_out are double; SPS_F32 and SPS_BF16X (split hi+lo BF16 with
 * FP32 accumulation): float.  The requested precision's table must have been
 * uploaded at create.  The FP32 / BF16X paths skip wavelengths farther than 8 filter
 * sigmas from every band for all galaxies of a 128-galaxy tile (their contribution is below
 * exp(-32) of the band's), and from 16,384 galaxies on they process the galaxies in z order
 * internally (outputs are still in the caller's order).  n_gal <= the rows reserved by
 * sps_reserve_exact, else SPS_E_STATE. */
int sps_phot_exact(sps_ctx *ctx, void *stream, int n_gal, int sfh, int prec, const void *params,
                   const void *z, void *mag_out);

/* Gaussian log-likelihood  log L = sum_b mask_b [-(m_b - d_b)^2 / (2 s_b^2) - ln(s_b sqrt(2 pi))]
 * and its gradient w.r.t. the 10 physical parameters (hand-written adjoint).
 * path SPS_PATH_APPROX (prec ignored) or SPS_PATH_EXACT (prec SPS_F32 or SPS_BF16X).
 * obs, sigma [n_gal][n_band]; band_mask [n_gal] (bit b set = band used);
 * logl_out [n_gal]; grad_out [10][n_gal] or NULL for value only. */
int sps_loglike_grad(sps_ctx *ctx, void *stream, int n_gal, int sfh, int path, int prec,
                     const float *params, const float *z, const float *obs, const float *sigma,
                     const uint8_t *band_mask, float *logl_out, float *grad_out);

/* Vector-Jacobian product of the magnitudes: grad_out[p][g] = sum_b gbar[g][b] dm_b/dtheta_p
 * for the 10 physical parameters (Sec. 4: the gradients a gradient-based sampler or a
 * user's own loss needs; the backward of the magnitude outputs of Eq. photo_integral_approx
 * and Eq. photo_integral_exact).  It is the same hand-written adjoint as sps_loglike_grad's,
 * seeded with the caller's band adjoints gbar [n_gal][n_band] (FP32, every band used) in
 * place of the likelihood's residual terms.  path SPS_PATH_APPROX (prec ignored, needs a z
 * table) or SPS_PATH_EXACT (prec SPS_F32 or SPS_BF16X; n_gal <= the reserved exact rows).
 * All arrays are caller-owned device memory; grad_out [10][n_gal] FP32 is overwritten.
 * Errors: SPS_E_INVAL (null array, bad path or precision), SPS_E_STATE (no z table, table
 * not uploaded, too few reserved rows). */
int sps_phot_vjp(sps_ctx *ctx, void *stream, int n_gal, int sfh, int path, int prec,
                 const float *params, const float *z, const float *gbar, float *grad_out);

/* Log posterior on the unbounded parameters x (App. C): theta_p = F_B(x_p) with
 * bounds[p] = (y_lo, y_hi, k, x0), plus the skew-normal log prior with
 * prior[p] = (xi, omega, s) on x_p; value logp_out [n_gal] and gradient
 * grad_out [10][n_gal] w.r.t. x (approximate path).  bounds, prior: device [10][4], [10][3]. */
int sps_logpost_grad(sps_ctx *ctx, void *stream, int n_gal, int sfh, const float *x,
                     const float *z, const float *obs, const float *sigma, const uint8_t *band_mask,
                     const float *bounds, const float *prior, float *logp_out, float *grad_out);

/* Batched HMC (Sec. 4, App. D.2): n_chain chains per galaxy, n_leapfrog leapfrog
 * steps per iteration, per-chain step size adapted by dual averaging over n_warmup
 * iterations, then n_sample recorded iterations; momentum and accept draws from
 * Philox4x32-10 keyed by seed with counter (draw block, iteration, chain id =
 * c * n_gal + g, 0).  Hamiltonian and accept test in FP64.  Starting points: theta0, or
 * if theta0 is NULL a draw from the skew-normal prior of each parameter (App. C, Eq.
 * SkewNormPrior; half-normal representation, Philox counter (block 0..4, 0, chain id, 1)).
 * Mass matrix: identity if adapt_metric = 0.  If adapt_metric = 1 (and n_warmup >= 20),
 * a per-chain diagonal M is adapted in slow warm-up windows (fast buffer of 75
 * iterations, windows of 25, 50, 100, ... with the last stretched to the end of the
 * slow phase, final fast buffer of 50; 15 % / 75 % / 10 % of n_warmup when these do
 * not fit): at each window's end M^-1 = n/(n+5) var(x) + 1e-3 * 5/(n+5) over the
 * window's n iterates of the unbounded parameters, and dual averaging restarts from
 * the current step size.  The paper's warm-up tunes its sampler's parameters without
 * stating the scheme; this is the windowed scheme of the Stan manual.
 * All device pointers:
 *   theta0 [n_chain][10][n_gal] unbounded starting points, or NULL (prior draws),
 *   samples [n_sample][n_chain][10][n_gal] physical draws or NULL,
 *   post_mean, post_sd, rhat [10][n_gal] (physical parameters, pooled chains),
 *   accept [n_gal] acceptance fraction in the sampling phase,
 *   step [n_chain][n_gal] step size after warm-up,
 *   inv_metric [n_chain][10][n_gal] diagonal M^-1 after warm-up, or NULL.
 * path selects the photometry inside the likelihood (Sec. 3): SPS_PATH_APPROX (the z
 * table; needs sps_build_ztable; one fused kernel runs whole blocks of iterations) or
 * SPS_PATH_EXACT (the spectrum-level MFMA contraction and its adjoint in precision prec,
 * SPS_F32 or SPS_BF16X, whose table must have been uploaded; every leapfrog step is one
 * exact value+gradient call over all n_gal * n_chain chains).  prec is ignored on the
 * approximate path.  Both paths draw the same Philox streams.
 * Needs n_gal * n_chain <= the galaxy count reserved by sps_reserve (and, for
 * SPS_PATH_EXACT, <= the rows reserved by sps_reserve_exact).  The exact path ranks the
 * chains by z internally (on the z table's buckets if one was built, else on a fixed grid).
 *
 * Splitting a run over calls (checkpoint / resume, Sec. 4's long runs): cfg.it_begin and
 * cfg.it_end select the iterations [it_begin, it_end) of the n_warmup + n_sample that this
 * call runs (it_end = 0: to the end).  state_inout (device memory of
 * sps_hmc_state_bytes(n_gal, n_chain) bytes, owned by the caller) then carries every
 * chain's state between the calls: a call with it_begin = 0 starts the chains (theta0 or
 * prior draws) and one with it_begin > 0 continues from the state the previous call wrote
 * (its header must name the same n_gal, n_chain, n_warmup, n_sample, adapt_metric, seed,
 * n_leapfrog and it_begin iterations done, else sps_status reports SPS_E_STATE); every call
 * writes the state back.  The draws are those of the uninterrupted run, to the bit, for
 * either photometry path (the blob is the same for both).  samples are written for the
 * sampling iterations this call runs; the summaries (post_mean .. inv_metric, required
 * then) by the call that ends the run.  state_inout may be NULL for a whole run. */
typedef struct {
    int n_chain, n_leapfrog, n_warmup, n_sample;
    float target_accept, init_step;
    unsigned long long seed;
    int adapt_metric;
    int path, prec;
    int it_begin, it_end;
} sps_hmc_cfg;

int sps_hmc_run(sps_ctx *ctx, void *stream, const sps_hmc_cfg *cfg, int n_gal, int sfh,
                const float *z, const float *obs, const float *sigma, const uint8_t *band_mask,
                const float *bounds, const float *prior, const float *theta0, float *samples,
                float *post_mean, float *post_sd, float *rhat, float *accept, float *step,
                float *inv_metric, void *state_inout);

/* Bytes of an sps_hmc_run resume blob for n_gal galaxies x n_chain chains (0 if invalid):
 * a 256-byte header and 312 bytes per chain. */
size_t sps_hmc_state_bytes(int n_gal, int n_chain);

/* Launch choices of a context that never change any result, only the order or grouping in
 * which independent work is issued (every output is bitwise the same for every setting):
 *   exact_order      exact-path GEMM tile order: 0 the built-in policy (M fastest, N fastest
 *                    for the windowed forward GEMM), 1 M fastest, 2 N fastest, 3 bands of 8
 *                    row tiles (M fastest within a band that sweeps every column tile)
 *   exact_xcd        1: each of the 8 XCDs takes one contiguous run of tiles; 0: tiles in
 *                    dispatch order (round-robin over the XCDs)
 *   hmc_block_iters  approximate-path HMC iterations per kernel launch, 1..1000 (default 25)
 *   nuts_block_iters NUTS iterations per kernel launch, 1..1000 (default 10)
 *   hmcx_graph       exact-path HMC: 1 captures one iteration (about 10 kernels per leapfrog
 *                    step) as a hipGraph once per call and replays it, the iteration index read
 *                    from device memory; 0 launches the kernels one by one (default 1)
 *   exact_ring       BF16X exact-path GEMMs: 0 operands staged through registers into one LDS
 *                    stage, three blocks per CU; 1 a two-stage LDS ring filled by direct
 *                    global-to-LDS loads, two blocks per CU (default 0) */
typedef struct {
    int exact_order, exact_xcd, hmc_block_iters, nuts_block_iters, hmcx_graph, exact_ring;
} sps_launch_cfg;

int sps_get_launch(sps_ctx *ctx, sps_launch_cfg *out);
int sps_set_launch(sps_ctx *ctx, const sps_launch_cfg *cfg);   /* SPS_E_INVAL for a value out of range */

/* Autotuner of the launch choices above (setup calls: they synchronise the device and may
 * allocate).  Each times the candidates with HIP events on `stream`, on the caller's own
 * inputs (a few repetitions each, the median kept), sets the fastest in the context and writes
 * it to *chosen (may be NULL); *timed_ms (may be NULL) receives the chosen candidate's time, or
 * 0 if the choice came from the cache.  If the environment variable SPS_AUTOTUNE_CACHE names a
 * file, choices are looked up there first (key: the call kind, device name and CU count, and
 * the shape of the call) and new ones are added to it (a JSON object, one entry per line).
 *  sps_autotune_exact: exact_order x exact_xcd (x exact_ring for SPS_BF16X) on
 *    sps_loglike_grad(path = SPS_PATH_EXACT) of
 *    these inputs (obs, sigma, band_mask may be NULL: sps_phot_exact is timed instead).
 *  sps_autotune_hmc: hmc_block_iters (approximate path) or hmcx_graph (exact path) on a short
 *    run of cfg's sampler (cfg->n_warmup + cfg->n_sample iterations are not run: a few
 *    iterations of each candidate are) on these inputs. */
int sps_autotune_exact(sps_ctx *ctx, void *stream, int n_gal, int sfh, int prec, const float *params, const float *z,
                       const float *obs, const float *sigma, const uint8_t *band_mask, sps_launch_cfg *chosen,
                       float *timed_ms);
/* Autotuner of sps_hmc_run's launch choice (see sps_autotune_exact above for the protocol):
 * hmc_block_iters on the approximate path (candidates 5, 10, 25, 50; timed on 50 iterations)
 * or hmcx_graph on the exact path (timed on 10 iterations), each a throwaway run of cfg's
 * sampler on these inputs (at most n_warmup + n_sample iterations). */
int sps_autotune_hmc(sps_ctx *ctx, void *stream, const sps_hmc_cfg *cfg, int n_gal, int sfh, const float *z,
                     const float *obs, const float *sigma, const uint8_t *band_mask, const float *bounds,
                     const float *prior, const float *theta0, sps_launch_cfg *chosen, float *timed_ms);

/* sps_loglike_grad (approximate path) for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation.  Same
 * arguments, kernels and results as sps_loglike_grad with path = SPS_PATH_APPROX, but its
 * per-call buffers (sort order, bucket counts, input records) are a static device
 * array of the library, about 4.6 MB per device for SPS_STATIC_MAX_GAL galaxies, held until
 * the process ends; it allocates nothing and calls no allocating routine.  n_gal above
 * SPS_STATIC_MAX_GAL is SPS_E_INVAL.  Every call on one device shares that device's array,
 * which keeps the last call's contents (each call clears what it needs): calls that overlap in
 * time on one device (other streams, other contexts, other host threads) race and must be
 * serialised by the caller.  The context still provides the tables and the z table. */
#define SPS_STATIC_MAX_GAL 32768
int sps_loglike_grad_static(sps_ctx *ctx, void *stream, int n_gal, int sfh, const float *params, const float *z,
                            const float *obs, const float *sigma, const uint8_t *band_mask, float *logl_out,
                            float *grad_out);

/* No-U-Turn Sampler (the paper's second gradient-based sampler, Sec. 4 and App. D.2):
 * Hoffman & Gelman (2014), Algorithm 3 (slice variable, trajectory doubling in a random
 * direction, a new subtree's proposal taken with probability min(1, n'/n)) with the dual
 * averaging of their Algorithm 6 (acceptance statistic: the mean of min(1, exp(H0 - H)) over
 * the final tree's leaves, target target_accept); identity or windowed diagonal metric as in
 * sps_hmc_run.  Approximate photometry (the z table) only.  At most 2^max_depth - 1 leapfrog
 * steps per iteration, 1 <= max_depth <= 12.
 * Philox4x32-10 keyed by seed (chain id = c * n_gal + g): momentum and slice (counter
 * (blk 0..2, it, chain id, 0): words 0..9 the momentum as in HMC, word 10 the slice uniform),
 * per doubling j (j, it, chain id, 2: word 0 the direction, word 1 the subtree's acceptance),
 * per leaf (leaf index within the iteration, it, chain id, 3: the reservoir uniform).
 * Chains run in lock-step per wavefront (32 chains of a wave evaluate the model together):
 * sync_iterations = 1 makes a wave's chains start every iteration together, so that each
 * iteration lasts as long as the wave's deepest tree; 0 lets a chain whose tree is done start
 * its next iteration at once.  The draws are the same either way.
 * Arguments as sps_hmc_run (whole runs only: no resume blob), plus, all optional (NULL):
 *   depth [n_warmup + n_sample][n_chain][n_gal] int: tree depth (doublings) per iteration,
 *   n_leaf [n_chain][n_gal] int: leapfrog steps of each chain over the run,
 *   lockstep [2] unsigned long long: [0] the chains' leapfrog steps, [1] the steps the waves
 *     took times the chains they hold (the evaluations the hardware spent); [0] / [1] is the
 *     lock-step efficiency.
 * accept [n_gal] is the mean acceptance statistic of the sampling phase.  Needs a workspace
 * from sps_reserve_nuts for n_gal * n_chain chains at this max_depth (else SPS_E_STATE) and
 * n_gal <= the galaxies reserved by sps_reserve. */
typedef struct {
    int n_chain, max_depth, n_warmup, n_sample;
    float target_accept, init_step;
    unsigned long long seed;
    int adapt_metric;
    int sync_iterations;
} sps_nuts_cfg;

int sps_nuts_run(sps_ctx *ctx, void *stream, const sps_nuts_cfg *cfg, int n_gal, int sfh, const float *z,
                 const float *obs, const float *sigma, const uint8_t *band_mask, const float *bounds,
                 const float *prior, const float *theta0, float *samples, float *post_mean, float *post_sd,
                 float *rhat, float *accept, float *step, float *inv_metric, int *depth, int *n_leaf,
                 unsigned long long *lockstep);

/* Size the NUTS workspace for up to max_chains chains (n_gal * n_chain) at trees of up to
 * max_depth doublings: the chain state, the two ends of the trajectory, the proposals and
 * one checkpoint per doubling level (about (1.6 + 0.08 max_depth) KB per chain).  Also grows
 * sps_reserve's galaxy count to max_chains.  Synchronises the device; never shrinks. */
int sps_reserve_nuts(sps_ctx *ctx, int max_chains, int max_depth);

#ifdef __cplusplus
}
#endif
#endif /* SPS_H */
