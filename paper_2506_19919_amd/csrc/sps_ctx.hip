// Context lifecycle, table uploads, the z-table build and the C ABI entry points.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "sps_model.h"

namespace sps {

// Scratch of sps_loglike_grad_static: the approximate path's per-call buffers (z-bucket order,
// the sort's bucket totals and block counts, the input records) for up to
// SPS_STATIC_MAX_GAL galaxies, laid out at 256-byte boundaries.  One copy per device, held
// until the process ends.  In host code the array's name is not a device address: kernels
// get the address hipGetSymbolAddress returned for the current device (g_scratch).
constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t ST_PERM = 0;
constexpr size_t ST_HIST = ST_PERM + al256((size_t)SPS_STATIC_MAX_GAL * sizeof(int));
constexpr size_t ST_REC = ST_HIST + al256(sort_ws_ints(SPS_STATIC_MAX_GAL) * sizeof(int));
constexpr size_t ST_BYTES = ST_REC + al256((size_t)SPS_STATIC_MAX_GAL * REC * sizeof(float));
static __device__ __align__(256) unsigned char scratch[ST_BYTES];

constexpr int MAX_DEVICES = 64;
static char *g_scratch[MAX_DEVICES];
static std::mutex g_scratch_mu;

}  // namespace sps

namespace {

thread_local std::string g_err;

constexpr double MPC_KM = 3.0856775814913673e19;
constexpr double MPC_CM = 3.0856775814913673e24;
constexpr double GYR_S = 3.15576e16;      // Julian Gyr
constexpr double C_KMS = 299792.458;
constexpr double C_ANGS = 2.99792458e18;  // A/s
constexpr double LSUN = 3.828e33;         // erg/s
constexpr double AB_FNU0 = 3631.0e-23;    // erg/s/cm^2/Hz

// positive half of the n-point Gauss-Legendre rule (Newton iteration on P_n)
void gauss_legendre_half(int n, double *x, double *w) {
    for (int i = 0; i < n / 2; ++i) {
        double r = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = r;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * r * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (r * p1 - p0) / (r * r - 1.0);
            double dr = p1 / dp;
            r -= dr;
            if (std::fabs(dr) < 1e-17) break;
        }
        x[i] = r;
        w[i] = 2.0 / ((1.0 - r * r) * dp * dp);
    }
}

uint16_t bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float bf16_to_f(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

bool increasing(const double *v, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(v[i]) || (i && !(v[i] > v[i - 1]))) return false;
    return true;
}

}  // namespace

namespace sps {

int set_error(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_check(hipError_t e, const char *what) {
    return set_error(e == hipErrorOutOfMemory ? SPS_E_NOMEM : SPS_E_HIP,
                     std::string(what) + ": " + hipGetErrorString(e));
}

// filter weights tw[kb][l] = T_b((1+z_k) l) l q_l / N_b(z_k), N_b = sum_l T_b((1+z_k) l) q_l / l
__global__ void __launch_bounds__(256) k_filter_weights(int nb, int nw, double z_lo, double dz,
                                                        const double *__restrict__ fc, const double *__restrict__ fs,
                                                        const double *__restrict__ wave, const double *__restrict__ trap,
                                                        double *__restrict__ tw) {
    __shared__ double red[256];
    const int kb = blockIdx.x, kz = kb / nb, b = kb % nb;
    const double z = z_lo + dz * kz;
    double s = 0.0;
    for (int l = threadIdx.x; l < nw; l += 256) {
        const double x = ((1.0 + z) * wave[l] - fc[b]) / fs[b];
        const double t = exp(-0.5 * x * x);
        tw[(size_t)kb * nw + l] = t * wave[l] * trap[l];
        s += t * trap[l] / wave[l];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    const double inv = 1.0 / red[0];
    for (int l = threadIdx.x; l < nw; l += 256) tw[(size_t)kb * nw + l] *= inv;
}

// Q[kz][b][s] = sum_l L[s][l] tw[kz*nb+b][l]; one block per SSP row s (row staged in LDS)
__global__ void __launch_bounds__(256) k_ztable(int n_ssp, int nkb, int nw, const double *__restrict__ lum,
                                                const double *__restrict__ tw, float *__restrict__ q) {
    extern __shared__ double row[];
    const int s = blockIdx.x;
    for (int l = threadIdx.x; l < nw; l += 256) row[l] = lum[(size_t)s * nw + l];
    __syncthreads();
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int kb = wid; kb < nkb; kb += 4) {
        double acc = 0.0;
        for (int l = lane; l < nw; l += 64) acc += row[l] * tw[(size_t)kb * nw + l];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) q[(size_t)kb * n_ssp + s] = (float)acc;
    }
}

__device__ inline uint16_t bf16_bits(float f) {   // round to nearest even
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// fragment-order BF16 hi/lo copies of the z table (layouts in sps_internal.h); one thread
// per table value of each layout
__global__ void __launch_bounds__(256) k_qswizzle(int n_z, int R, const float *__restrict__ q,
                                                  uint16_t *__restrict__ qf, uint16_t *__restrict__ qa) {
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    const size_t total = (size_t)n_z * QB_NODE;
    if (t >= total) return;
    const int node = (int)(t / QB_NODE);
    const int rem = (int)(t % QB_NODE);
    const int e = rem & 7, lane = (rem >> 3) & 63, blk = rem >> 9;   // blk = outer * KSTEPS + ks
    const int outer = blk / KSTEPS, ks = blk % KSTEPS;
    const float *qn = q + (size_t)node * R * NA;
    auto put = [&](uint16_t *dst, int r, int i) {
        const float v = (r < R && i < NA) ? qn[(size_t)r * NA + i] : 0.0f;
        const uint16_t hb = bf16_bits(v);
        dst[t] = hb;
        dst[total + t] = bf16_bits(v - __uint_as_float((uint32_t)hb << 16));
    };
    put(qf, 16 * outer + (lane & 15), 32 * ks + 8 * (lane >> 4) + e);
    put(qa, 32 * ks + 8 * (lane >> 4) + e, 16 * outer + (lane & 15));
}

// cosmology table rows: t_obs, dt/dz, mag_offset, dm/dz at z = lo + i dz
__global__ void __launch_bounds__(256) k_cosmo_table(DevConsts k, int n, double lo, double dz, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double z = lo + dz * (double)i, dl = lum_distance_cm(k, z);
    double dt, dm;
    cosmo_derivs(k, z, dl, dt, dm);
    out[4 * i] = age_universe_gyr(k, z);
    out[4 * i + 1] = dt;
    out[4 * i + 2] = -2.5 * log10((1.0 + z) * k.kfac) + 5.0 * log10(dl);
    out[4 * i + 3] = dm;
}

int launch_ztable(sps_ctx *c, hipStream_t st) {
    const int nb = c->n_band, nw = c->n_wave, nkb = c->k.n_z * nb, S = c->n_met * c->n_age;
    double *d_fc = nullptr, *d_fs = nullptr, *d_tw = nullptr;
    double fc[NB_MAX], fs[NB_MAX];
    for (int b = 0; b < nb; ++b) { fc[b] = c->h_fc[b]; fs[b] = c->h_fs[b]; }
    SPS_HIP(hipMalloc(&d_fc, nb * sizeof(double)));
    SPS_HIP(hipMalloc(&d_fs, nb * sizeof(double)));
    SPS_HIP(hipMalloc(&d_tw, (size_t)nkb * nw * sizeof(double)));
    SPS_HIP(hipMemcpy(d_fc, fc, nb * sizeof(double), hipMemcpyHostToDevice));
    SPS_HIP(hipMemcpy(d_fs, fs, nb * sizeof(double), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_filter_weights, dim3(nkb), dim3(256), 0, st, nb, nw, (double)c->k.z_lo,
                       (double)c->k.dz, d_fc, d_fs, c->d_wave, c->d_trap, d_tw);
    hipLaunchKernelGGL(k_ztable, dim3(S), dim3(256), nw * sizeof(double), st, S, nkb, nw, c->d_lum64, d_tw, c->d_q);
    {
        DevConsts k0 = c->k;
        k0.ctab = nullptr;
        hipLaunchKernelGGL(k_cosmo_table, dim3((CT_N + 255) / 256), dim3(256), 0, st, k0, CT_N, c->k.ct_lo,
                           c->k.ct_dz, c->d_ctab);
    }
    {
        const size_t total = (size_t)c->k.n_z * QB_NODE;
        hipLaunchKernelGGL(k_qswizzle, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, c->k.n_z, nb * NZ,
                           c->d_q, c->d_qf, c->d_qa);
    }
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d_fc);
    (void)hipFree(d_fs);
    (void)hipFree(d_tw);
    if (e != hipSuccess) return hip_check(e, "z-table build");
    return SPS_OK;
}

}  // namespace sps

using namespace sps;

namespace {

static void free_timing(sps_ctx *c) {
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    c->tev.clear();
    c->tev_calls = 0;
}

void free_ctx(sps_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    free_timing(c);
    (void)release_graph(c);
    if (c->graph_done) (void)hipEventDestroy(c->graph_done);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    (void)hipFree(c->d_lum64);
    (void)hipFree(c->d_ls32);
    (void)hipFree(c->d_lt32);
    (void)hipFree(c->d_ls_bx);
    (void)hipFree(c->d_lt_bx);
    (void)hipFree(c->d_wc);
    (void)hipFree(c->d_wave);
    (void)hipFree(c->d_trap);
    (void)hipFree(c->d_edges);
    (void)hipFree(c->d_q);
    (void)hipFree(c->d_qf);
    (void)hipFree(c->d_qa);
    (void)hipFree(c->d_ctab);
    (void)hipFree(c->d_perm);
    (void)hipFree(c->d_rec);
    (void)hipFree(c->d_hist);
    (void)hipFree(c->d_status);
    (void)hipFree(c->d_hstate);
    (void)hipFree(c->d_work);
    (void)hipFree(c->d_hwork);
    (void)hipFree(c->d_xsort);
    (void)hipFree(c->d_nwork);
    delete c;
}

int enter(sps_ctx *c) {
    if (!c) return set_error(SPS_E_INVAL, "null context");
    SPS_HIP(hipSetDevice(c->device));
    return SPS_OK;
}

int check_gal(sps_ctx *c, int n_gal, int sfh) {
    if (n_gal < 0) return set_error(SPS_E_INVAL, "n_gal < 0");
    if (n_gal > c->max_gal)
        return set_error(SPS_E_INVAL, "n_gal " + std::to_string(n_gal) + " exceeds the reserved " +
                                          std::to_string(c->max_gal) + " (call sps_reserve)");
    if (sfh != SPS_SFH_LOGNORMAL && sfh != SPS_SFH_DPL) return set_error(SPS_E_INVAL, "bad sfh kind");
    return SPS_OK;
}

}  // namespace

namespace sps {
hipEvent_t *timing_pair(sps_ctx *c) {
    if (c->tev.empty()) return nullptr;
    const size_t np = c->tev.size() / 2, i = (size_t)(c->tev_calls++ % (long long)np);
    return &c->tev[2 * i];
}
}  // namespace sps


extern "C" {

const char *sps_last_error(void) { return g_err.c_str(); }

int sps_reserve(sps_ctx *c, int max_gal) {
    int rc = enter(c);
    if (rc) return rc;
    if (max_gal < 1) return set_error(SPS_E_INVAL, "max_gal < 1");
    if (max_gal <= c->max_gal) return SPS_OK;
    SPS_HIP(hipDeviceSynchronize());
    (void)hipFree(c->d_perm);
    (void)hipFree(c->d_rec);
    (void)hipFree(c->d_hstate);
    (void)hipFree(c->d_hist);
    c->d_hist = nullptr;
    c->d_perm = nullptr;
    c->d_rec = nullptr;
    c->d_hstate = nullptr;
    c->hstate_bytes = 0;
    c->max_gal = 0;
    SPS_HIP(hipMalloc(&c->d_hist, sort_ws_ints(max_gal) * sizeof(int)));
    SPS_HIP(hipMalloc(&c->d_perm, (size_t)max_gal * sizeof(int)));
    SPS_HIP(hipMalloc(&c->d_rec, (size_t)max_gal * REC * sizeof(float)));
    const size_t hb = hmc_state_bytes(max_gal);
    SPS_HIP(hipMalloc(&c->d_hstate, hb));
    c->hstate_bytes = hb;
    c->max_gal = max_gal;
    return SPS_OK;
}

int sps_reserve_exact(sps_ctx *c, int max_rows) {
    int rc = enter(c);
    if (rc) return rc;
    if (max_rows < 1) return set_error(SPS_E_INVAL, "max_rows < 1");
    if (max_rows > c->max_gal && (rc = sps_reserve(c, max_rows))) return rc;
    if (max_rows <= c->max_exact) return SPS_OK;
    size_t wb = 0;
    for (int p = SPS_F64; p <= SPS_BF16X; ++p)
        if (c->prec_mask & (1u << p)) {
            const bool lik = (p != SPS_F64);   // the FP64 path computes magnitudes only
            wb = std::max(wb, exact_ws_bytes(c, max_rows, p, lik, lik));
        }
    const size_t xb = exact_xsort_bytes(c, max_rows), hb = hmcx_state_bytes(c, max_rows);
    SPS_HIP(hipDeviceSynchronize());
    (void)hipFree(c->d_work);
    (void)hipFree(c->d_xsort);
    (void)hipFree(c->d_hwork);
    c->d_work = c->d_xsort = c->d_hwork = nullptr;
    c->work_bytes = c->xsort_bytes = c->hwork_bytes = 0;
    c->max_exact = 0;
    SPS_HIP(hipMalloc(&c->d_work, wb));
    if (xb) SPS_HIP(hipMalloc(&c->d_xsort, xb));
    SPS_HIP(hipMalloc(&c->d_hwork, hb));
    c->work_bytes = wb;
    c->xsort_bytes = xb;
    c->hwork_bytes = hb;
    c->max_exact = max_rows;
    return SPS_OK;
}

int sps_reserve_nuts(sps_ctx *c, int max_chains, int max_depth) {
    int rc = enter(c);
    if (rc) return rc;
    if (max_chains < 1) return set_error(SPS_E_INVAL, "max_chains < 1");
    if (max_depth < 1 || max_depth > 12) return set_error(SPS_E_INVAL, "need 1 <= max_depth <= 12");
    if (max_chains > c->max_gal && (rc = sps_reserve(c, max_chains))) return rc;
    const size_t nb = nuts_state_bytes(max_chains, max_depth);
    if (nb <= c->nwork_bytes) return SPS_OK;
    SPS_HIP(hipDeviceSynchronize());
    (void)hipFree(c->d_nwork);
    c->d_nwork = nullptr;
    c->nwork_bytes = 0;
    SPS_HIP(hipMalloc(&c->d_nwork, nb));
    c->nwork_bytes = nb;
    return SPS_OK;
}

int sps_status(sps_ctx *c) {
    int rc = enter(c);
    if (rc) return rc;
    SPS_HIP(hipDeviceSynchronize());
    int bits = 0;
    SPS_HIP(hipMemcpy(&bits, c->d_status, sizeof(int), hipMemcpyDeviceToHost));
    SPS_HIP(hipMemset(c->d_status, 0, sizeof(int)));
    if (bits & STATUS_HMC_STATE)
        return set_error(SPS_E_STATE, "an HMC resume blob did not match its run (configuration or iteration)");
    if (bits & STATUS_Z_RANGE)
        return set_error(SPS_E_RANGE, "a redshift outside the z table was given to the approximate path (NaN outputs)");
    return SPS_OK;
}

size_t sps_hmc_state_bytes(int n_gal, int n_chain) {
    if (n_gal < 0 || n_chain < 1) return 0;
    return 256 + sps::chain_state_bytes_public(n_gal * n_chain);
}

int sps_create(sps_ctx **out, int device, const sps_ssp_desc *ssp, const sps_filter_desc *flt,
               const sps_model_desc *model, unsigned prec_mask, int max_gal) {
    if (!out) return set_error(SPS_E_INVAL, "null out pointer");
    *out = nullptr;
    if (!ssp || !flt || !model) return set_error(SPS_E_INVAL, "null descriptor");
    if (!ssp->log10_met || !ssp->log10_age_yr || !ssp->wave_A || !ssp->lum)
        return set_error(SPS_E_INVAL, "null SSP array");
    if (ssp->n_age != NA || ssp->n_met != NZ)
        return set_error(SPS_E_INVAL, "unsupported SSP grid: the kernels tile n_age = 94, n_met = 12");
    if (ssp->n_wave < 2) return set_error(SPS_E_INVAL, "n_wave < 2");
    if (!increasing(ssp->log10_met, NZ) || !increasing(ssp->log10_age_yr, NA) ||
        !increasing(ssp->wave_A, ssp->n_wave) || !(ssp->wave_A[0] > 0.0))
        return set_error(SPS_E_INVAL, "SSP grids must be finite and strictly increasing (wavelengths > 0)");
    if (flt->n_band < 1 || flt->n_band > NB_MAX || !flt->center_A || !flt->sigma_A)
        return set_error(SPS_E_INVAL, "n_band must be 1..8 with centre and sigma arrays");
    for (int b = 0; b < flt->n_band; ++b)
        if (!(flt->center_A[b] > 0.0) || !(flt->sigma_A[b] > 0.0))
            return set_error(SPS_E_INVAL, "filter centre and sigma must be positive");
    if (!(model->H0 > 0.0) || !(model->Om > 0.0 && model->Om <= 1.0) || !(model->sigma_logz > 0.0) ||
        !(model->burst_dlogt > 0.0))
        return set_error(SPS_E_INVAL, "bad model constants (H0 > 0, 0 < Om <= 1, widths > 0)");
    if (max_gal < 1) return set_error(SPS_E_INVAL, "max_gal < 1");
    if (prec_mask & ~7u) return set_error(SPS_E_INVAL, "bad precision mask");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return set_error(SPS_E_INVAL, "no such HIP device");

    sps_ctx *c = new sps_ctx();
    c->device = device;
    c->n_met = NZ;
    c->n_age = NA;
    c->n_wave = ssp->n_wave;
    c->n_band = flt->n_band;
    c->prec_mask = prec_mask | 1u;
    DevConsts &k = c->k;
    k.n_band = flt->n_band;
    k.n_wave = ssp->n_wave;
    k.n_z = 0;
    k.sigma_logz = (float)model->sigma_logz;
    k.burst_sig = (float)(model->burst_dlogt / 3.0);
    k.sigma_logz_d = model->sigma_logz;
    k.burst_sig_d = model->burst_dlogt / 3.0;
    // age bins: edges at midpoints of log age, open at both ends (0 and infinity)
    const double *la = ssp->log10_age_yr;
    for (int i = 0; i < NA; ++i) {
        double llo = (i == 0) ? -INFINITY : 0.5 * (la[i - 1] + la[i]);
        double lhi = (i == NA - 1) ? INFINITY : 0.5 * (la[i] + la[i + 1]);
        k.lage_lo[i] = (float)llo;
        k.lage_hi[i] = (float)lhi;
        k.age_lo[i] = (i == 0) ? 0.0f : (float)(std::pow(10.0, llo) * 1e-9);
        k.age_hi[i] = (i == NA - 1) ? INFINITY : (float)(std::pow(10.0, lhi) * 1e-9);
    }
    // widest run of age bins a burst window [v, v + 6 sigma] can touch: a window starting in
    // bin i0 ends below lage_hi[i0] + 6 sigma (padded against FP32 rounding of the edges)
    {
        const double win = 2.0 * model->burst_dlogt + 1e-3;
        int most = 1;
        for (int i0 = 0; i0 < NA - 1; ++i0) {
            const double top = (double)k.lage_hi[i0] + win;
            int cnt = 1;
            while (i0 + cnt < NA && (double)k.lage_lo[i0 + cnt] < top) ++cnt;
            most = std::max(most, cnt);
        }
        k.burst_nbins = most;
    }
    std::vector<double> edges(4 * NA + 2 * NZ);
    for (int i = 0; i < NA; ++i) {
        double llo = (i == 0) ? -INFINITY : 0.5 * (la[i - 1] + la[i]);
        double lhi = (i == NA - 1) ? INFINITY : 0.5 * (la[i] + la[i + 1]);
        edges[i] = (i == 0) ? 0.0 : std::pow(10.0, llo) * 1e-9;
        edges[NA + i] = (i == NA - 1) ? INFINITY : std::pow(10.0, lhi) * 1e-9;
        edges[2 * NA + i] = llo;
        edges[3 * NA + i] = lhi;
    }
    const double *lz = ssp->log10_met;
    for (int j = 0; j < NZ; ++j) {
        edges[4 * NA + j] = (j == 0) ? -INFINITY : 0.5 * (lz[j - 1] + lz[j]);
        edges[4 * NA + NZ + j] = (j == NZ - 1) ? INFINITY : 0.5 * (lz[j] + lz[j + 1]);
    }
    for (int j = 0; j < NZ; ++j) {
        k.met_lo[j] = (j == 0) ? -INFINITY : (float)(0.5 * (lz[j - 1] + lz[j]));
        k.met_hi[j] = (j == NZ - 1) ? INFINITY : (float)(0.5 * (lz[j] + lz[j + 1]));
    }
    for (int b = 0; b < NB_MAX; ++b) {
        const bool on = b < flt->n_band;
        k.fc[b] = on ? (float)flt->center_A[b] : 1.0f;
        k.fs[b] = on ? (float)flt->sigma_A[b] : 1.0f;
        // mean wavelength of a Gaussian transmission curve is its centre
        k.lam_eff[b] = k.fc[b];
        c->h_fc[b] = on ? flt->center_A[b] : 1.0;
        c->h_fs[b] = on ? flt->sigma_A[b] : 1.0;
    }
    k.h0_gyr = model->H0 / MPC_KM * GYR_S;
    k.om = model->Om;
    k.dh_cm = C_KMS / model->H0 * MPC_CM;
    k.kfac = LSUN / (4.0 * M_PI * C_ANGS * AB_FNU0);
    gauss_legendre_half(2 * NGL_DL, k.gl_x, k.gl_w);
    gauss_legendre_half(8, k.gl8_x, k.gl8_w);

    // wavelength trapezoid weights
    const int nw = ssp->n_wave;
    c->h_wave.assign(ssp->wave_A, ssp->wave_A + nw);
    c->h_trap.assign(nw, 0.0);
    for (int l = 0; l < nw; ++l) {
        double lo = ssp->wave_A[l == 0 ? 0 : l - 1], hi = ssp->wave_A[l == nw - 1 ? nw - 1 : l + 1];
        c->h_trap[l] = 0.5 * (hi - lo);
    }
    // keep filter descriptors in double for the table builds
    const size_t S = (size_t)NZ * NA, nl = S * nw;
    int rc = SPS_OK;
    auto fail = [&](int code) { free_ctx(c); return code; };
    if (hipSetDevice(device) != hipSuccess) return fail(set_error(SPS_E_HIP, "hipSetDevice failed"));
    {   // the static scratch's address on this device, looked up once per device
        if (device < 0 || device >= MAX_DEVICES) return fail(set_error(SPS_E_INVAL, "device index out of range"));
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch[device]) {
            void *p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(set_error(SPS_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)));
            g_scratch[device] = (char *)p;
        }
    }
    auto upload = [&](void **dst, const void *src, size_t bytes) -> int {
        SPS_HIP(hipMalloc(dst, bytes));
        SPS_HIP(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
        return SPS_OK;
    };
    if ((rc = upload((void **)&c->d_lum64, ssp->lum, nl * sizeof(double)))) return fail(rc);
    if ((rc = upload((void **)&c->d_wave, c->h_wave.data(), nw * sizeof(double)))) return fail(rc);
    if ((rc = upload((void **)&c->d_trap, c->h_trap.data(), nw * sizeof(double)))) return fail(rc);
    if ((rc = upload((void **)&c->d_edges, edges.data(), edges.size() * sizeof(double)))) return fail(rc);
    // matrix-core copies of the SSP table (see sps_internal.h), zero padded
    const int lw = (nw + 127) / 128 * 128;
    c->lw = lw;
    const size_t np = (size_t)S_PAD * lw;
    if (prec_mask & (1u << SPS_F32)) {
        std::vector<float> ls(np, 0.0f), lt(np, 0.0f);
        for (size_t s = 0; s < S; ++s)
            for (int l = 0; l < nw; ++l) {
                const float f = (float)ssp->lum[s * nw + l];
                ls[s * lw + l] = f;
                lt[(size_t)l * S_PAD + s] = f;
            }
        if ((rc = upload((void **)&c->d_ls32, ls.data(), np * sizeof(float)))) return fail(rc);
        if ((rc = upload((void **)&c->d_lt32, lt.data(), np * sizeof(float)))) return fail(rc);
    }
    if (prec_mask & (1u << SPS_BF16X)) {
        std::vector<uint16_t> ls_x(2 * np, 0), lt_x(2 * np, 0);
        for (size_t s = 0; s < S; ++s)
            for (int l = 0; l < nw; ++l) {
                const float f = (float)ssp->lum[s * nw + l];
                const uint16_t h = bf16_rne(f), lo = bf16_rne(f - bf16_to_f(h));
                const size_t a = bfx_at(s, lw, l), b = bfx_at(l, S_PAD, (int)s);
                ls_x[a] = h;
                ls_x[a + 32] = lo;
                lt_x[b] = h;
                lt_x[b + 32] = lo;
            }
        if ((rc = upload((void **)&c->d_ls_bx, ls_x.data(), np * 4))) return fail(rc);
        if ((rc = upload((void **)&c->d_lt_bx, lt_x.data(), np * 4))) return fail(rc);
    }
    {
        std::vector<float> wc((size_t)lw * 4, 0.0f);
        for (int l = 0; l < nw; ++l) {
            const double lam = c->h_wave[l], q = c->h_trap[l];
            wc[4 * l] = (float)std::log(lam / 5500.0);
            wc[4 * l + 1] = (float)(lam * q);
            wc[4 * l + 2] = (float)(q / lam);
            wc[4 * l + 3] = (float)lam;
        }
        if ((rc = upload((void **)&c->d_wc, wc.data(), wc.size() * sizeof(float)))) return fail(rc);
    }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->graph_done, hipEventDisableTiming) != hipSuccess)
        return fail(set_error(SPS_E_HIP, "stream / event creation failed"));
    if (hipMalloc(&c->d_status, sizeof(int)) != hipSuccess || hipMemset(c->d_status, 0, sizeof(int)) != hipSuccess)
        return fail(set_error(SPS_E_NOMEM, "workspace allocation failed"));
    if ((rc = sps_reserve(c, max_gal))) return fail(rc);
    *out = c;
    return SPS_OK;
}

void sps_destroy(sps_ctx *c) { free_ctx(c); }

int sps_set_kernel_timing(sps_ctx *c, int n_pairs) {
    if (!c || n_pairs < 0 || n_pairs > 4096) return set_error(SPS_E_INVAL, "sps_set_kernel_timing: bad arguments");
    SPS_HIP(hipSetDevice(c->device));
    SPS_HIP(hipDeviceSynchronize());
    free_timing(c);
    c->tev.resize(2 * (size_t)n_pairs, nullptr);
    for (auto &e : c->tev) {
        const hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
            e = nullptr;
            free_timing(c);
            return hip_check(r, "hipEventCreate");
        }
    }
    return SPS_OK;
}

int sps_kernel_times(sps_ctx *c, float *ms_out, int max, int *count) {
    if (!c || !ms_out || !count || max < 0) return set_error(SPS_E_INVAL, "sps_kernel_times: bad arguments");
    if (c->tev.empty()) return set_error(SPS_E_INVAL, "sps_kernel_times: kernel timing is off");
    SPS_HIP(hipSetDevice(c->device));
    const long long np = (long long)(c->tev.size() / 2);
    const long long k = std::min<long long>(std::min<long long>(np, c->tev_calls), max);
    for (long long j = 0; j < k; ++j) {
        const size_t i = (size_t)((c->tev_calls - k + j) % np);
        SPS_HIP(hipEventSynchronize(c->tev[2 * i + 1]));
        SPS_HIP(hipEventElapsedTime(&ms_out[j], c->tev[2 * i], c->tev[2 * i + 1]));
    }
    *count = (int)k;
    return SPS_OK;
}

int sps_build_ztable(sps_ctx *c, int n_z, double z_lo, double z_hi) {
    int rc = enter(c);
    if (rc) return rc;
    if (n_z < 2 || n_z > 1024) return set_error(SPS_E_INVAL, "n_z must be in 2..1024");
    if (!(z_lo >= 0.0) || !(z_hi > z_lo) || !std::isfinite(z_hi)) return set_error(SPS_E_INVAL, "need 0 <= z_lo < z_hi");
    SPS_HIP(hipDeviceSynchronize());
    (void)hipFree(c->d_q);
    (void)hipFree(c->d_qf);
    (void)hipFree(c->d_qa);
    (void)hipFree(c->d_ctab);
    c->d_q = nullptr;
    c->d_qf = c->d_qa = nullptr;
    c->d_ctab = nullptr;
    c->k.ctab = nullptr;
    c->k.n_z = 0;
    SPS_HIP(hipMalloc(&c->d_q, (size_t)n_z * c->n_band * NZ * NA * sizeof(float)));
    const size_t frag = (size_t)2 * n_z * QB_NODE * sizeof(uint16_t);   // hi and lo
    SPS_HIP(hipMalloc(&c->d_qf, frag));
    SPS_HIP(hipMalloc(&c->d_qa, frag));
    SPS_HIP(hipMalloc(&c->d_ctab, (size_t)4 * CT_N * sizeof(double)));
    c->k.z_lo = (float)z_lo;
    c->k.dz = (float)((z_hi - z_lo) / (n_z - 1));
    c->k.n_z = n_z;
    c->k.ct_lo = z_lo;
    c->k.ct_dz = (z_hi - z_lo) / (CT_N - 1);
    c->k.ct_inv_dz = 1.0 / c->k.ct_dz;
    rc = launch_ztable(c, nullptr);
    if (rc) c->k.n_z = 0;
    else c->k.ctab = c->d_ctab;
    return rc;
}

int sps_get_ztable(sps_ctx *c, float *q_host) {
    int rc = enter(c);
    if (rc) return rc;
    if (!q_host) return set_error(SPS_E_INVAL, "null output");
    if (c->k.n_z == 0) return set_error(SPS_E_STATE, "no z table built");
    SPS_HIP(hipMemcpy(q_host, c->d_q, (size_t)c->k.n_z * c->n_band * NZ * NA * sizeof(float), hipMemcpyDeviceToHost));
    return SPS_OK;
}

int sps_weights(sps_ctx *c, void *stream, int n_gal, int sfh, const float *params, const float *z, float *w_out) {
    int rc = enter(c);
    if (rc) return rc;
    if ((rc = check_gal(c, n_gal, sfh))) return rc;
    if (n_gal == 0) return SPS_OK;
    if (!params || !z || !w_out) return set_error(SPS_E_INVAL, "null array");
    return launch_weights(c, (hipStream_t)stream, n_gal, sfh, params, z, w_out);
}

int sps_phot_approx(sps_ctx *c, void *stream, int n_gal, int sfh, const float *params, const float *z,
                    float *mag_out) {
    int rc = enter(c);
    if (rc) return rc;
    if ((rc = check_gal(c, n_gal, sfh))) return rc;
    if (c->k.n_z == 0) return set_error(SPS_E_STATE, "build the z table first (sps_build_ztable)");
    if (n_gal == 0) return SPS_OK;
    if (!params || !z || !mag_out) return set_error(SPS_E_INVAL, "null array");
    return launch_approx(c, (hipStream_t)stream, n_gal, sfh, MODE_MAGS, params, z, nullptr, nullptr, nullptr,
                         nullptr, nullptr, mag_out, nullptr, nullptr);
}

int sps_phot_exact(sps_ctx *c, void *stream, int n_gal, int sfh, int prec, const void *params, const void *z,
                   void *mag_out) {
    int rc = enter(c);
    if (rc) return rc;
    if ((rc = check_gal(c, n_gal, sfh))) return rc;
    if (prec < SPS_F64 || prec > SPS_BF16X) return set_error(SPS_E_INVAL, "bad precision");
    if (!(c->prec_mask & (1u << prec))) return set_error(SPS_E_STATE, "this precision's SSP table was not uploaded");
    if (n_gal == 0) return SPS_OK;
    if (!params || !z || !mag_out) return set_error(SPS_E_INVAL, "null array");
    return launch_exact(c, (hipStream_t)stream, n_gal, sfh, prec, params, z, mag_out, nullptr, nullptr, nullptr,
                        nullptr, nullptr);
}

int sps_loglike_grad(sps_ctx *c, void *stream, int n_gal, int sfh, int path, int prec, const float *params,
                     const float *z, const float *obs, const float *sigma, const uint8_t *band_mask,
                     float *logl_out, float *grad_out) {
    int rc = enter(c);
    if (rc) return rc;
    if ((rc = check_gal(c, n_gal, sfh))) return rc;
    if (path != SPS_PATH_APPROX && path != SPS_PATH_EXACT) return set_error(SPS_E_INVAL, "bad path");
    if (n_gal == 0) return SPS_OK;
    if (!params || !z || !obs || !sigma || !band_mask || !logl_out)
        return set_error(SPS_E_INVAL, "null array");
    if (path == SPS_PATH_APPROX) {
        if (c->k.n_z == 0) return set_error(SPS_E_STATE, "build the z table first (sps_build_ztable)");
        return launch_approx(c, (hipStream_t)stream, n_gal, sfh, grad_out ? MODE_LOGL_GRAD : MODE_LOGL, params, z,
                             obs, sigma, band_mask, nullptr, nullptr, nullptr, logl_out, grad_out);
    }
    if (prec != SPS_F32 && prec != SPS_BF16X)
        return set_error(SPS_E_INVAL, "exact-path likelihood runs in SPS_F32 or SPS_BF16X");
    if (!(c->prec_mask & (1u << prec))) return set_error(SPS_E_STATE, "this precision's SSP table was not uploaded");
    return launch_exact(c, (hipStream_t)stream, n_gal, sfh, prec, params, z, nullptr, obs, sigma, band_mask,
                        logl_out, grad_out);
}

int sps_phot_vjp(sps_ctx *c, void *stream, int n_gal, int sfh, int path, int prec, const float *params,
                 const float *z, const float *gbar, float *grad_out) {
    int rc = enter(c);
    if (rc) return rc;
    if ((rc = check_gal(c, n_gal, sfh))) return rc;
    if (path != SPS_PATH_APPROX && path != SPS_PATH_EXACT) return set_error(SPS_E_INVAL, "bad path");
    if (n_gal == 0) return SPS_OK;
    if (!params || !z || !gbar || !grad_out) return set_error(SPS_E_INVAL, "null array");
    if (path == SPS_PATH_APPROX) {
        if (c->k.n_z == 0) return set_error(SPS_E_STATE, "build the z table first (sps_build_ztable)");
        return launch_approx(c, (hipStream_t)stream, n_gal, sfh, MODE_VJP, params, z, gbar, nullptr, nullptr,
                             nullptr, nullptr, nullptr, nullptr, grad_out);
    }
    if (prec != SPS_F32 && prec != SPS_BF16X)
        return set_error(SPS_E_INVAL, "exact-path vector-Jacobian products run in SPS_F32 or SPS_BF16X");
    if (!(c->prec_mask & (1u << prec))) return set_error(SPS_E_STATE, "this precision's SSP table was not uploaded");
    return launch_exact(c, (hipStream_t)stream, n_gal, sfh, prec, params, z, nullptr, gbar, nullptr, nullptr,
                        nullptr, grad_out, false, true);
}

int sps_logpost_grad(sps_ctx *c, void *stream, int n_gal, int sfh, const float *x, const float *z,
                     const float *obs, const float *sigma, const uint8_t *band_mask, const float *bounds,
                     const float *prior, float *logp_out, float *grad_out) {
    int rc = enter(c);
    if (rc) return rc;
    if ((rc = check_gal(c, n_gal, sfh))) return rc;
    if (c->k.n_z == 0) return set_error(SPS_E_STATE, "build the z table first (sps_build_ztable)");
    if (n_gal == 0) return SPS_OK;
    if (!x || !z || !obs || !sigma || !band_mask || !bounds || !prior || !logp_out || !grad_out)
        return set_error(SPS_E_INVAL, "null array");
    return launch_approx(c, (hipStream_t)stream, n_gal, sfh, MODE_LOGPOST_GRAD, x, z, obs, sigma, band_mask,
                         bounds, prior, nullptr, logp_out, grad_out);
}

int sps_hmc_run(sps_ctx *c, void *stream, const sps_hmc_cfg *cfg, int n_gal, int sfh, const float *z,
                const float *obs, const float *sigma, const uint8_t *band_mask, const float *bounds,
                const float *prior, const float *theta0, float *samples, float *post_mean, float *post_sd,
                float *rhat, float *accept, float *step, float *inv_metric, void *state_inout) {
    int rc = enter(c);
    if (rc) return rc;
    if (!cfg) return set_error(SPS_E_INVAL, "null config");
    if ((rc = check_gal(c, n_gal, sfh))) return rc;
    if (cfg->n_chain < 1 || cfg->n_chain > 64 || cfg->n_leapfrog < 1 || cfg->n_warmup < 0 || cfg->n_sample < 2)
        return set_error(SPS_E_INVAL, "need 1 <= n_chain <= 64, n_leapfrog >= 1, n_warmup >= 0, n_sample >= 2");
    if (!(cfg->init_step > 0.0f) || !(cfg->target_accept > 0.0f && cfg->target_accept < 1.0f))
        return set_error(SPS_E_INVAL, "need init_step > 0 and 0 < target_accept < 1");
    if (cfg->adapt_metric != 0 && cfg->adapt_metric != 1) return set_error(SPS_E_INVAL, "adapt_metric must be 0 or 1");
    if ((long long)n_gal * cfg->n_chain > (long long)c->max_gal)
        return set_error(SPS_E_INVAL, "n_gal * n_chain exceeds the reserved workspace (call sps_reserve)");
    const int nit = cfg->n_warmup + cfg->n_sample;
    const int it1 = cfg->it_end > 0 ? cfg->it_end : nit;
    if (cfg->it_begin < 0 || cfg->it_end < 0 || it1 > nit || cfg->it_begin >= it1)
        return set_error(SPS_E_INVAL, "need 0 <= it_begin < it_end <= n_warmup + n_sample (it_end 0 = to the end)");
    if ((cfg->it_begin > 0 || it1 < nit) && !state_inout)
        return set_error(SPS_E_INVAL, "a run split over calls needs state_inout");
    if (cfg->path == SPS_PATH_EXACT && (long long)n_gal * cfg->n_chain > (long long)c->max_exact)
        return set_error(SPS_E_STATE, "n_gal * n_chain exceeds the reserved exact rows (call sps_reserve_exact)");
    if (cfg->path != SPS_PATH_APPROX && cfg->path != SPS_PATH_EXACT) return set_error(SPS_E_INVAL, "bad path");
    if (cfg->path == SPS_PATH_APPROX && c->k.n_z == 0)
        return set_error(SPS_E_STATE, "build the z table first (sps_build_ztable)");
    if (cfg->path == SPS_PATH_EXACT) {
        if (cfg->prec != SPS_F32 && cfg->prec != SPS_BF16X)
            return set_error(SPS_E_INVAL, "exact-path HMC runs in SPS_F32 or SPS_BF16X");
        if (!(c->prec_mask & (1u << cfg->prec)))
            return set_error(SPS_E_STATE, "this precision's SSP table was not uploaded");
    }
    if (n_gal == 0) return SPS_OK;
    if (!z || !obs || !sigma || !band_mask || !bounds || !prior)
        return set_error(SPS_E_INVAL, "null array");
    if (it1 == nit && (!post_mean || !post_sd || !rhat || !accept || !step))
        return set_error(SPS_E_INVAL, "null summary array (required from the call that ends the run)");
    return launch_hmc(c, (hipStream_t)stream, cfg, n_gal, sfh, z, obs, sigma, band_mask, bounds, prior, theta0,
                      samples, post_mean, post_sd, rhat, accept, step, inv_metric, state_inout);
}

int sps_loglike_grad_static(sps_ctx *c, void *stream, int n_gal, int sfh, const float *params, const float *z,
                            const float *obs, const float *sigma, const uint8_t *band_mask, float *logl_out,
                            float *grad_out) {
    int rc = enter(c);
    if (rc) return rc;
    if (n_gal < 0 || n_gal > SPS_STATIC_MAX_GAL)
        return set_error(SPS_E_INVAL, "n_gal must be 0.." + std::to_string(SPS_STATIC_MAX_GAL) +
                                          " for sps_loglike_grad_static");
    if (sfh != SPS_SFH_LOGNORMAL && sfh != SPS_SFH_DPL) return set_error(SPS_E_INVAL, "bad sfh kind");
    if (c->k.n_z == 0) return set_error(SPS_E_STATE, "build the z table first (sps_build_ztable)");
    if (n_gal == 0) return SPS_OK;
    if (!params || !z || !obs || !sigma || !band_mask || !logl_out) return set_error(SPS_E_INVAL, "null array");
    char *base = g_scratch[c->device];   // set by sps_create for this device
    if (!base) return set_error(SPS_E_STATE, "no static scratch on this device");
    const ApproxWs ws{(int *)(base + ST_PERM), (int *)(base + ST_HIST), (float *)(base + ST_REC)};
    return launch_approx_ws(c, (hipStream_t)stream, ws, n_gal, sfh, grad_out ? MODE_LOGL_GRAD : MODE_LOGL, params, z,
                            obs, sigma, band_mask, nullptr, nullptr, nullptr, logl_out, grad_out);
}

int sps_nuts_run(sps_ctx *c, void *stream, const sps_nuts_cfg *cfg, int n_gal, int sfh, const float *z,
                 const float *obs, const float *sigma, const uint8_t *band_mask, const float *bounds,
                 const float *prior, const float *theta0, float *samples, float *post_mean, float *post_sd,
                 float *rhat, float *accept, float *step, float *inv_metric, int *depth, int *n_leaf,
                 unsigned long long *lockstep) {
    int rc = enter(c);
    if (rc) return rc;
    if (!cfg) return set_error(SPS_E_INVAL, "null config");
    if ((rc = check_gal(c, n_gal, sfh))) return rc;
    if (cfg->n_chain < 1 || cfg->n_chain > 64 || cfg->max_depth < 1 || cfg->max_depth > 12 || cfg->n_warmup < 0 ||
        cfg->n_sample < 2)
        return set_error(SPS_E_INVAL, "need 1 <= n_chain <= 64, 1 <= max_depth <= 12, n_warmup >= 0, n_sample >= 2");
    if (!(cfg->init_step > 0.0f) || !(cfg->target_accept > 0.0f && cfg->target_accept < 1.0f))
        return set_error(SPS_E_INVAL, "need init_step > 0 and 0 < target_accept < 1");
    if (cfg->adapt_metric != 0 && cfg->adapt_metric != 1) return set_error(SPS_E_INVAL, "adapt_metric must be 0 or 1");
    if (cfg->sync_iterations != 0 && cfg->sync_iterations != 1)
        return set_error(SPS_E_INVAL, "sync_iterations must be 0 or 1");
    if ((long long)n_gal * cfg->n_chain > (long long)c->max_gal)
        return set_error(SPS_E_INVAL, "n_gal * n_chain exceeds the reserved workspace (call sps_reserve_nuts)");
    if (c->k.n_z == 0) return set_error(SPS_E_STATE, "build the z table first (sps_build_ztable)");
    if (n_gal == 0) return SPS_OK;
    if (!z || !obs || !sigma || !band_mask || !bounds || !prior || !post_mean || !post_sd || !rhat || !accept || !step)
        return set_error(SPS_E_INVAL, "null array");
    return launch_nuts(c, (hipStream_t)stream, cfg, n_gal, sfh, z, obs, sigma, band_mask, bounds, prior, theta0,
                       samples, post_mean, post_sd, rhat, accept, step, inv_metric, depth, n_leaf, lockstep);
}

}  // extern "C"
