/*
 * SPS hot-path ORACLE -- test infrastructure only.
 *
 * A plain, slow FP64 CPU implementation of the forward model, photometry,
 * likelihood and HMC sampler of "Bayesian Posteriors with Stellar Population
 * Synthesis on GPUs" (Zacharegkas, Hearin & Benson), written from the paper's
 * equations.  It exists to check the HIP library; only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header or table with the HIP library.
 *
 * All arrays are host FP64, row-major.  Parameters are AoS: theta[g][10] in the
 * slot order documented in synth/__init__.py.  Gradients come from forward-mode
 * dual numbers (an independent differentiation route from the library's
 * hand-written adjoint).
 *
 * Return codes: 0 ok, 1 invalid argument, 2 z outside the table range.
 */
#ifndef SPS_ORACLE_H
#define SPS_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NPARAM 10

typedef struct {
    int n_met, n_age, n_wave;
    const double *log10_met;     /* [n_met]  log10 Z/Zsun, increasing          */
    const double *log10_age_yr;  /* [n_age]  log10 age/yr, increasing          */
    const double *wave_A;        /* [n_wave] rest-frame wavelength, increasing  */
    const double *lum;           /* [n_met][n_age][n_wave] Lsun/A per Msun formed */
} orc_ssp;

typedef struct {
    int n_band;
    const double *center_A;      /* Gaussian transmission, peak 1, observed frame */
    const double *sigma_A;
} orc_filters;

typedef struct { double H0, Om; } orc_cosmo;   /* flat LCDM, km/s/Mpc */

typedef struct {
    double sigma_logz;   /* width of the log-normal metallicity distribution [dex] */
    double burst_dlogt;  /* log10 T_max - log10 T_peak [dex]                        */
} orc_model;

/* ---- cosmology (flat LCDM, matter + Lambda) ---- */
double orc_age_universe_gyr(const orc_cosmo *c, double z);
double orc_lum_distance_mpc(const orc_cosmo *c, double z);

/* ---- per-galaxy SSP weights ---- */
/* p_age[n_age], p_smooth[n_age], p_burst[n_age], p_met[n_met]; any may be NULL. */
int orc_age_weights(const orc_ssp *s, const orc_cosmo *c, const orc_model *m, int sfh,
                    const double *theta, double z,
                    double *p_age, double *p_smooth, double *p_burst);
int orc_met_weights(const orc_ssp *s, const orc_model *m, const double *theta, double *p_met);
/* w[g][n_met][n_age], summing to 10^theta[0] (mass formed) */
int orc_weights(const orc_ssp *s, const orc_cosmo *c, const orc_model *m, int sfh,
                int n_gal, const double *theta, const double *z, double *w);
/* smooth-SFH mass formed per age bin, unnormalised [n_age] (rate amplitude 1) */
int orc_smooth_bin_mass(const orc_ssp *s, const orc_cosmo *c, int sfh,
                        const double *theta, double z, double *mass);

/* ---- dust ---- */
double orc_dust_att(const double *theta, double lam_rest_A);

/* ---- filters ---- */
double orc_lambda_eff(const orc_filters *f, int band);

/* ---- photometry: AB magnitudes mags[g][n_band] ---- */
int orc_phot_exact(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                   int sfh, int n_gal, const double *theta, const double *z, double *mags);
/* Q[n_z][n_band][n_met][n_age]: distance-free SSP band fluxes on z nodes */
int orc_ztable(const orc_ssp *s, const orc_filters *f, int n_z, double z_lo, double z_hi, double *q);
int orc_phot_approx(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                    int n_z, double z_lo, double z_hi, const double *q,
                    int sfh, int n_gal, const double *theta, const double *z, double *mags);

/* ---- Gaussian log-likelihood and its gradient w.r.t. the 10 physical params ----
 * path 0 = approximate (needs q), 1 = exact.  obs, sigma [g][n_band]; mask[g] bit b = band used.
 * grad [g][10] may be NULL. */
int orc_loglike_grad(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                     int path, int n_z, double z_lo, double z_hi, const double *q,
                     int sfh, int n_gal, const double *theta, const double *z,
                     const double *obs, const double *sigma, const uint8_t *mask,
                     double *logl, double *grad);

/* magnitudes and their Jacobian d m_b / d theta_p: mags[g][b], jac[g][b][10] (path 0 approx, 1 exact) */
int orc_mags_jacobian(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m, int path,
                      int n_z, double z_lo, double z_hi, const double *q, int sfh, int n_gal, const double *theta,
                      const double *z, double *mags, double *jac);

/* ---- bounding function and skew-normal prior ---- */
/* bounds[p][4] = (y_lo, y_hi, k, x0); prior[p][3] = (xi, omega, s) on the unbounded value */
double orc_bound(const double *bnd, double x_unbounded);
double orc_unbound(const double *bnd, double theta);
double orc_log_prior(const double *pri, double x_unbounded);
/* log posterior on the unbounded parameters and its gradient [10]; path 0: approximate
 * photometry (needs the z table q), 1: exact photometry */
int orc_logpost_grad(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m, int path,
                     int n_z, double z_lo, double z_hi, const double *q, int sfh,
                     const double *theta_u, double z, const double *obs, const double *sigma,
                     uint8_t mask, const double *bounds, const double *prior,
                     double *logp, double *grad);

/* n_step leapfrog steps (half kick, drift, half kick) of the HMC dynamics from
 * (x, p) in place; logp = log target at the final x.  gauss_prec as in orc_hmc_run. */
int orc_leapfrog(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                 int n_z, double z_lo, double z_hi, const double *q, int sfh, double z, const double *obs,
                 const double *sigma, uint8_t mask, const double *bounds, const double *prior,
                 const double *gauss_prec, int n_step, double eps, double *x, double *p, double *logp);

/* ---- the n-point Gauss-Legendre rule on [-1, 1] (1 <= n <= 16), nodes increasing ---- */
int orc_gauss_legendre(int n, double *x, double *w);

/* ---- counter-based RNG (Philox4x32-10) ---- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* ---- HMC ---- */
typedef struct {
    int n_chain, n_leapfrog, n_warmup, n_sample;
    double target_accept, init_step;
    uint64_t seed;
    int adapt_metric;   /* 0: identity mass matrix; 1: diagonal, 2: dense, adapted in slow windows */
    int path;           /* photometry of the likelihood: 0 approximate (z table), 1 exact */
    int it_begin, it_end;  /* iterations [it_begin, it_end) of this call (it_end 0 = to the end) */
} orc_hmc_cfg;

/* Per-chain state carried between the calls of a run split over several calls, ORC_HMC_STATE
 * doubles per chain: [0,10) x, [10,20) grad log p, 20 log p, 21 step size, 22 mu, 23 Hbar,
 * 24 log eps bar, 25 iteration at which dual averaging last restarted, 26 metric window index,
 * 27 samples recorded, 28 samples accepted, [30,40) diagonal M^-1, [40,60) Welford mean and
 * M2 of the current metric window, [60,80) Welford mean and M2 of the physical draws,
 * [100,200) dense M^-1, [200,300) its Cholesky factor, [300,400) window co-moments. */
#define ORC_HMC_STATE 400

/* Starting point drawn from the skew-normal prior of every parameter (App. C): x[10]. */
void orc_hmc_prior_draw(const double *prior, uint64_t seed, uint32_t chain_id, double *x);

/* Slow adaptation windows of a warm-up of n_warmup iterations: window w covers
 * iterations [start[w], end[w]).  Returns the number of windows (0 if n_warmup < 20);
 * at most max_win are written. */
int orc_hmc_windows(int n_warmup, int max_win, int *start, int *end);

/* theta0[c][g][10] unbounded start, or NULL: drawn from the prior (orc_hmc_prior_draw with the
 * chain's Philox chain id); outputs:
 *   post_mean, post_sd, rhat [g][10] (physical parameters),
 *   accept [g] (fraction accepted in the sampling phase, all chains),
 *   step [c][g] (step size after warm-up),
 *   samples [n_sample][c][g][10] physical (may be NULL),
 *   trace_logp [n_warmup+n_sample][c][g] log posterior after each iteration (may be NULL).
 * gauss_prec (may be NULL): if set, the target is the zero-mean Gaussian with this
 * 10x10 precision matrix instead of the SPS posterior (sampler validation mode;
 * then the physical map is the identity).
 * gal_id (may be NULL): global galaxy indices when these galaxies are a subset of a batch of
 * n_gal_total galaxies; the Philox chain id is then chain * n_gal_total + gal_id[g].
 * inv_metric [c][g][10] (may be NULL): diagonal of the inverse mass matrix after warm-up.
 * trace_acc [n_warmup+n_sample][c][g][3] (may be NULL): per iteration the acceptance
 * probability, log u + (H1 - H0) (the proposal is accepted iff this is negative and it did not
 * diverge) and the step size the iteration used.
 * state [c][g][ORC_HMC_STATE] (may be NULL unless the call covers part of the run): read at
 * it_begin > 0, written at the end of every call.  Summaries are written by the call that ends
 * the run. */
int orc_hmc_run(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                int n_z, double z_lo, double z_hi, const double *q, int sfh,
                const orc_hmc_cfg *cfg, int n_gal, const double *z, const double *obs,
                const double *sigma, const uint8_t *mask, const double *bounds, const double *prior,
                const double *theta0, const double *gauss_prec,
                double *post_mean, double *post_sd, double *rhat, double *accept, double *step,
                double *samples, double *trace_logp, int n_gal_total, const uint32_t *gal_id,
                double *inv_metric, double *trace_acc, double *state);

/* ---- NUTS (Hoffman & Gelman 2014, Algorithm 3 with the dual averaging of Algorithm 6) ---- */
typedef struct {
    int n_chain, max_depth, n_warmup, n_sample;   /* max_depth: at most 2^max_depth - 1 leaves (<= 12) */
    double target_accept, init_step;
    uint64_t seed;
    int adapt_metric;   /* 0: identity; 1: diagonal, adapted in the HMC's slow windows */
    int path;           /* 0 approximate photometry, 1 exact */
} orc_nuts_cfg;

/* Arguments as orc_hmc_run; accept [g] is the mean acceptance statistic (mean over the leaves
 * of min(1, exp(H0 - H))) of the sampling phase; trace_depth / trace_steps
 * [n_warmup+n_sample][c][g] (may be NULL): the tree depth (doublings) and the leapfrog steps
 * of every iteration; trace_margin [n_warmup+n_sample][c][g][2] (may be NULL): per iteration
 * the smallest |log u + H| over the leaves (slice membership) and the smallest cosine between
 * a tested stretch and the velocity at its ends (U-turn tests), i.e. how near the iteration's
 * decisions came to their thresholds. */
int orc_nuts_run(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                 int n_z, double z_lo, double z_hi, const double *q, int sfh, const orc_nuts_cfg *cfg,
                 int n_gal, const double *z, const double *obs, const double *sigma, const uint8_t *mask,
                 const double *bounds, const double *prior, const double *theta0, const double *gauss_prec,
                 double *post_mean, double *post_sd, double *rhat, double *accept, double *step,
                 double *samples, int *trace_depth, int *trace_steps, double *trace_margin, double *inv_metric,
                 int n_gal_total, const uint32_t *gal_id);

/* classic Gelman-Rubin R-hat over x[c][n] (n_chain chains of n draws) */
double orc_rhat(int n_chain, int n, const double *x);

#ifdef __cplusplus
}
#endif
#endif
