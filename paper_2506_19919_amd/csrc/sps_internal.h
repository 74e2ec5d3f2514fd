// Internal declarations of the SPS HIP library (host + device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/sps.h"

namespace sps {

// Compile-time SSP grid tile: per-lane age weights live in registers.
constexpr int NA = 94;            // ages
constexpr int NZ = 12;            // metallicities
constexpr int NB_MAX = SPS_MAX_BAND;
constexpr int NP = SPS_NPARAM;
constexpr int NGL_DL = 12;        // half of the 24-point Gauss-Legendre rule for D_L

// Matrix-core fragment tables of the z table: B operands of v_mfma_f32_16x16x32_bf16, the
// table split as BF16 hi + lo (hi = bf16(Q), lo = bf16(Q - hi)).  With R = n_band * NZ table
// rows (r = b * NZ + j), per z node (QB_NODE bf16 values in each of the four arrays):
//   qf[nb][ks][lane][e] = Q[r = 16 nb + lane % 16][i = 32 ks + 8 (lane / 16) + e]   nb < 6, ks < 3
//   qa[na][ks][lane][e] = Q[r = 32 ks + 8 (lane / 16) + e][i = 16 na + lane % 16]   na < 6, ks < 3
// zero where r >= R or i >= NA; one 16-byte load per lane per fragment.
constexpr int AGE_BLK = 6;        // 96 padded ages = 6 blocks of 16
constexpr int KSTEPS = 3;         // 96 padded ages or rows = 3 k-steps of 32
constexpr int QB_NODE = 6 * KSTEPS * 64 * 8;
__host__ __device__ inline int row_blocks(int n_band) { return (n_band * NZ + 15) / 16; }
constexpr int S_PAD = 1152;       // SSP rows padded to a multiple of 128

// BF16 hi + lo pairs of a row-major matrix-core operand, interleaved per 32-element chunk of
// its contiguous (k) dimension: element k of row r (row length ld, a multiple of 32) has its
// hi at 2 ld r + 64 (k / 32) + k % 32 and its lo 32 further on, so that the hi and lo of a
// k-tile of 32 are one 128-byte line
__host__ __device__ inline size_t bfx_at(size_t r, int ld, int k) {
    return r * 2 * (size_t)ld + 64 * (size_t)(k >> 5) + (size_t)(k & 31);
}

// Kernel-facing constants, passed by value (kernarg segment).
struct DevConsts {
    int n_band, n_wave;
    int n_z;                      // z table nodes (0 = none)
    float z_lo, dz;               // z table: node k at z_lo + k dz
    float sigma_logz, burst_sig;  // dex; burst sigma = (log T_max - log T_peak)/3
    int burst_nbins;              // most age bins a triweight window of width 6 sigma can overlap
    double sigma_logz_d, burst_sig_d;
    float age_lo[NA], age_hi[NA]; // stellar-age limits of the bins [Gyr]; last hi = +inf
    float lage_lo[NA], lage_hi[NA];  // log10(age/yr) limits; -inf / +inf at the ends
    float met_lo[NZ], met_hi[NZ];    // log10 Z limits; -inf / +inf at the ends
    float lam_eff[NB_MAX];        // observed-frame effective wavelength of each band [A]
    float fc[NB_MAX], fs[NB_MAX]; // filter centre and sigma [A]
    double h0_gyr, om;            // H0 in 1/Gyr, matter density
    double dh_cm;                 // Hubble distance c/H0 [cm]
    double kfac;                  // Lsun / (4 pi c[A/s] 3631 Jy)  (AB normalisation)
    double gl_x[NGL_DL], gl_w[NGL_DL];  // positive Gauss-Legendre nodes/weights (24-point)
    double gl8_x[4], gl8_w[4];          // positive nodes/weights of the 8-point rule
    // t_obs(z) and the distance part of the magnitude offset, with their z derivatives, on
    // CT_N nodes over the z table's range: [CT_N][4] FP64 in device memory (null until a z
    // table is built)
    const double *ctab;
    double ct_lo, ct_dz, ct_inv_dz;
};
constexpr int CT_N = 1025;

}  // namespace sps

struct sps_ctx {
    int device = 0;
    int n_met = 0, n_age = 0, n_wave = 0, n_band = 0;
    unsigned prec_mask = 0;
    sps::DevConsts k{};
    std::vector<double> h_wave, h_trap;
    double h_fc[SPS_MAX_BAND] = {0}, h_fs[SPS_MAX_BAND] = {0};   // filter constants (FP64)
    // device tables
    double *d_lum64 = nullptr;     // [S][n_wave]
    // FP32 / BF16 hi+lo copies for the matrix-core GEMMs, zero-padded to S_PAD SSP rows and
    // LW = round_up(n_wave, 128) wavelengths, in both orientations (k contiguous):
    //   ls: [S_PAD][LW]  (B of the gradient GEMM, k = wavelength)
    //   lt: [LW][S_PAD]  (B of the forward GEMM, k = SSP)
    int lw = 0;
    float *d_ls32 = nullptr, *d_lt32 = nullptr;
    uint16_t *d_ls_bx = nullptr, *d_lt_bx = nullptr;   // BF16 hi + lo, interleaved (bfx_at)
    float *d_wc = nullptr;         // per wavelength [LW][4]: ln(l / 5500 A), l q_l, q_l / l, 0
    double *d_wave = nullptr, *d_trap = nullptr;
    double *d_edges = nullptr;     // FP64 bin edges: age_lo, age_hi [Gyr], lage_lo, lage_hi [NA each], met_lo, met_hi [NZ]
    float *d_q = nullptr;          // [n_z][n_band][n_met][n_age]
    uint16_t *d_qf = nullptr;      // z table fragments, forward contraction: hi [n_z][QB_NODE], then lo
    uint16_t *d_qa = nullptr;      // z table fragments, adjoint contraction: hi, then lo
    double *d_ctab = nullptr;      // cosmology table (DevConsts::ctab)
    // per-galaxy workspace
    int max_gal = 0;
    int *d_perm = nullptr;         // galaxies ordered by z bucket
    float *d_rec = nullptr;        // inputs in z-bucket order, one 128-byte record per galaxy
    int *d_hist = nullptr;         // z-bucket sort: bucket totals and per-block counts (sort_ws_ints)
    int *d_status = nullptr;       // device-side error bits (STATUS_*), read and cleared by sps_status
    void *d_hstate = nullptr;      // chain state of the approximate-path HMC, max_gal chain slots
    size_t hstate_bytes = 0;
    // exact path, sized by sps_reserve_exact for max_exact rows (galaxies or HMC chains)
    int max_exact = 0;
    void *d_work = nullptr;        // exact-path weights / partial fluxes
    size_t work_bytes = 0;
    void *d_hwork = nullptr;       // chain state of the exact-path HMC (d_work serves its model calls)
    size_t hwork_bytes = 0;
    void *d_xsort = nullptr;       // exact path: inputs and outputs in z order
    size_t xsort_bytes = 0;
    // NUTS, sized by sps_reserve_nuts: chain state, trajectory scratch and tree state
    void *d_nwork = nullptr;
    size_t nwork_bytes = 0;
    // launch choices (sps_set_launch, the autotuner); none changes a result
    sps_launch_cfg launch{0, 1, 25, 10, 1, 0};
    // the exact-path HMC's captured iteration: kept until the next capture or destroy, after
    // graph_done (recorded behind its last replay) has completed
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipEvent_t graph_done = nullptr;
    // kernel timing (sps_set_kernel_timing): 2 events per pair, pairs used cyclically
    std::vector<hipEvent_t> tev;
    long long tev_calls = 0;
};

namespace sps {

int set_error(int code, const std::string &msg);

// device-side error bits in sps_ctx::d_status (set by kernels, reported by sps_status)
enum { STATUS_Z_RANGE = 1, STATUS_HMC_STATE = 2 };
// the next timing event pair (start, stop) if kernel timing is on, else nullptr
hipEvent_t *timing_pair(sps_ctx *c);
int hip_check(hipError_t e, const char *what);
#define SPS_HIP(call)                                           \
    do {                                                        \
        hipError_t e_ = (call);                                 \
        if (e_ != hipSuccess) return ::sps::hip_check(e_, #call); \
    } while (0)

// launchers (defined in the kernel sources)
int launch_ztable(sps_ctx *c, hipStream_t s);   // also fills d_qf, d_qa
// Inputs gathered into z-bucket order by the sort (coalesced reads in the caller's order,
// one full-line record write per galaxy): record layout, REC floats per galaxy.
constexpr int REC = 32;
// slots 28..31: age of the universe at z [Gyr] and the distance part of the magnitude
// offset, each as an FP64 value in two words (low, high)
enum { REC_Z = 10, REC_OBS = 11, REC_SIG = 19, REC_MASK = 27, REC_TOBS = 28, REC_M0 = 30 };

// z-bucket sort workspace (ints): the buckets' totals, then one count row per block of
// SORT_T galaxies (at most SORT_MAX_BUCKETS buckets: z-table nodes <= 1024)
constexpr int SORT_T = 512;
constexpr int SORT_MAX_BUCKETS = 1024;
__host__ __device__ constexpr size_t sort_ws_ints(int max_gal) {
    return (size_t)SORT_MAX_BUCKETS * (1 + (size_t)((max_gal + SORT_T - 1) / SORT_T));
}
struct GatherArgs {
    const float *params, *obs, *sigma;  // obs, sigma may be null (magnitudes only)
    const uint8_t *mask;                // may be null (all bands)
    float *rec;                         // null: sort only
    int *status;                        // STATUS_Z_RANGE is set here for a z outside the table (or null)
};
// z buckets for ranking galaxies by redshift: the z table's nodes, or 64 buckets over
// 0 <= z < 8 when no table was built (z beyond goes to one overflow bucket)
inline DevConsts z_sort_grid(const sps_ctx *c) {
    DevConsts g = c->k;
    if (g.n_z == 0) {
        g.n_z = 65;
        g.z_lo = 0.0;
        g.dz = 0.125;
    }
    return g;
}
// grid: the z buckets (n_z, z_lo, dz of a DevConsts; n_z <= 1025); null: the z table's, and a z
// outside the table then sets STATUS_Z_RANGE
int launch_bucket_sort(sps_ctx *c, hipStream_t s, int n_gal, const float *z, const GatherArgs *ga = nullptr,
                       const DevConsts *grid = nullptr);
// device bytes of the workspaces, for the reservation calls
size_t exact_ws_bytes(const sps_ctx *c, int n, int prec, bool logl, bool grad);
size_t exact_xsort_bytes(const sps_ctx *c, int n);
size_t hmc_state_bytes(int nslot);
size_t chain_state_bytes_public(int nslot);   // chain state of nslot chains in a resume blob
size_t hmcx_state_bytes(const sps_ctx *c, int nslot);
int launch_weights(sps_ctx *c, hipStream_t s, int n_gal, int sfh, const float *params, const float *z,
                   float *w);
// the approximate path's per-call buffers: z-bucket order, the sort's bucket totals and block
// counts (sort_ws_ints), the input records; the context's, or another owner's
struct ApproxWs {
    int *perm, *hist;
    float *rec;
};
ApproxWs ctx_ws(sps_ctx *c);
int launch_bucket_sort_ws(sps_ctx *c, hipStream_t s, const ApproxWs &ws, int n, const float *z, const GatherArgs *ga,
                          const DevConsts *grid);
int launch_approx_ws(sps_ctx *c, hipStream_t s, const ApproxWs &ws, int n, int sfh, int mode, const float *params,
                     const float *z, const float *obs, const float *sigma, const uint8_t *mask, const float *bounds,
                     const float *prior, float *out_mag, float *out_val, float *out_grad);
int launch_approx(sps_ctx *c, hipStream_t s, int n_gal, int sfh, int mode, const float *params,
                  const float *z, const float *obs, const float *sigma, const uint8_t *mask,
                  const float *bounds, const float *prior, float *out_mag, float *out_val, float *out_grad);
// ordered: the galaxies already come in z order (the exact-path HMC ranks its chains); else the
// FP32 / BF16X paths rank them by z internally and return the outputs in the caller's order.
// vjp: obs holds the magnitudes' adjoints (sigma, mask and logl null) and grad receives their
// vector-Jacobian product
int launch_exact(sps_ctx *c, hipStream_t s, int n_gal, int sfh, int prec, const void *params,
                 const void *z, void *mag_out, const float *obs, const float *sigma,
                 const uint8_t *mask, float *logl, float *grad, bool ordered = false, bool vjp = false);
int launch_hmc(sps_ctx *c, hipStream_t s, const sps_hmc_cfg *cfg, int n_gal, int sfh, const float *z,
               const float *obs, const float *sigma, const uint8_t *mask, const float *bounds,
               const float *prior, const float *theta0, float *samples, float *post_mean,
               float *post_sd, float *rhat, float *accept, float *step, float *inv_metric, void *state);

size_t nuts_state_bytes(int nslot, int max_depth);
// waits for the replays of the exact-path HMC's captured iteration, then frees it
int release_graph(sps_ctx *c);
int launch_nuts(sps_ctx *c, hipStream_t s, const sps_nuts_cfg *cfg, int n_gal, int sfh, const float *z,
                const float *obs, const float *sigma, const uint8_t *mask, const float *bounds, const float *prior,
                const float *theta0, float *samples, float *post_mean, float *post_sd, float *rhat, float *accept,
                float *step, float *inv_metric, int *depth, int *n_leaf, unsigned long long *lockstep);

// modes of the approximate-path kernel
// MODE_VJP: the gradient pass with the magnitudes' adjoints supplied in place of observations
enum { MODE_MAGS = 0, MODE_LOGL = 1, MODE_LOGL_GRAD = 2, MODE_LOGPOST_GRAD = 3, MODE_VJP = 4 };

}  // namespace sps
