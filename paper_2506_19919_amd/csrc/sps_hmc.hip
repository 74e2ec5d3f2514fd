// Batched HMC on the unbounded parameters (Sec. 4; App. C, D.2).  Two adjacent lanes per
// chain (HG); the n_chain chains of a galaxy sit in adjacent lane pairs and galaxies are in
// z-bucket order, so a wave shares its z-table slices.  Each launch advances all chains by a
// block of iterations; chain state lives in HBM between launches.
//
// Per iteration: momentum p ~ N(0, M) from Philox4x32-10 (Box-Muller, scaled by
// M^1/2), n_leapfrog leapfrog steps (half kick, drift by M^-1 p, half kick; one
// value+gradient each), H = -log p + p^T M^-1 p / 2 summed in FP64, Metropolis test
// log u < H0 - H1 in FP64, divergence (non-finite H1 or H1 - H0 > 1000) = reject.
// Warm-up: dual averaging of log step size (Hoffman & Gelman 2014: mu = log(10 eps0),
// gamma = 0.05, t0 = 10, kappa = 0.75); afterwards the averaged step size is kept.
// Optional diagonal M (identity otherwise): Welford variance of the unbounded
// parameters over slow warm-up windows; at a window's end M^-1 = n/(n+5) var +
// 1e-3 * 5/(n+5) and dual averaging restarts at mu = log(10 eps).
// Sampling: Welford mean / M2 of the physical parameters per chain (FP64); the same
// state arrays hold the window statistics during warm-up.
#include "sps_eval.h"

namespace sps {

__device__ inline void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// uniform on (0, 1): (w + 1/2) / 2^32
__device__ inline float u01f(uint32_t w) { return fmaf((float)w, 2.3283064365386963e-10f, 1.1641532182693481e-10f); }
__device__ inline double u01d(uint32_t w) { return ((double)w + 0.5) * 2.3283064365386963e-10; }

// Unbounded starting point drawn from the skew-normal prior of every parameter (App. C, Eq.
// SkewNormPrior) by the half-normal representation: with U0, U1 standard normals and
// delta = s / sqrt(1 + s^2), xi + omega (delta |U0| + sqrt(1 - delta^2) U1) is skew-normal.
// (U0, U1) of parameter p is the Box-Muller pair of words 2p, 2p + 1 of the Philox blocks
// (blk, 0, chain id, 1), blk = 0..4 (the momentum draws use counter word 3 = 0).
__device__ __noinline__ void prior_draw(const float *prior, uint32_t key0, uint32_t key1, uint32_t chain_id,
                                        float (&x)[SPS_NPARAM]) {
    uint32_t w[20];
#pragma unroll
    for (int blk = 0; blk < 5; ++blk) {
        uint32_t c4[4] = {(uint32_t)blk, 0u, chain_id, 1u};
        philox4x32_10(c4, key0, key1);
#pragma unroll
        for (int t = 0; t < 4; ++t) w[4 * blk + t] = c4[t];
    }
#pragma unroll
    for (int p = 0; p < SPS_NPARAM; ++p) {
        const float r = sqrtf(-2.0f * logf(u01f(w[2 * p])));
        float sn, cs;
        sincosf(6.283185307179586f * u01f(w[2 * p + 1]), &sn, &cs);
        const float sk = prior[3 * p + 2], inv = 1.0f / sqrtf(1.0f + sk * sk);   // sqrt(1 - delta^2)
        x[p] = prior[3 * p] + prior[3 * p + 1] * (sk * inv * fabsf(r * cs) + inv * (r * sn));
    }
}

constexpr int MAX_WIN = 24;

// Chain state carried from one iteration to the next, SoA [quantity][slot]: the state of a run
// that a resume blob (sps_hmc_run's state_inout) holds between calls.
struct ChainState {
    float *x, *gr, *minv;               // [NP][slot]
    float *eps, *mu, *hbar, *lebar;     // [slot]
    int *nacc, *da0;                    // [slot]
    double *lp, *wmean, *wm2;           // [slot], [NP][slot], [NP][slot]
};
// floats, ints and doubles per chain slot
constexpr int CS_F = 3 * SPS_NPARAM + 4, CS_I = 2, CS_D = 1 + 2 * SPS_NPARAM;
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t chain_state_bytes(int nslot) {
    return align256((size_t)nslot * CS_F * 4) + align256((size_t)nslot * CS_I * 4) + align256((size_t)nslot * CS_D * 8);
}
// the quantities laid out from base for nslot slots
static ChainState chain_state_at(void *base, int nslot) {
    ChainState cs;
    char *b = (char *)base;
    float *f = (float *)b;
    cs.x = f;
    cs.gr = f + (size_t)SPS_NPARAM * nslot;
    cs.minv = f + (size_t)2 * SPS_NPARAM * nslot;
    cs.eps = f + (size_t)3 * SPS_NPARAM * nslot;
    cs.mu = cs.eps + nslot;
    cs.hbar = cs.mu + nslot;
    cs.lebar = cs.hbar + nslot;
    int *ip = (int *)(b + align256((size_t)nslot * CS_F * 4));
    cs.nacc = ip;
    cs.da0 = ip + nslot;
    double *d = (double *)(b + align256((size_t)nslot * CS_F * 4) + align256((size_t)nslot * CS_I * 4));
    cs.lp = d;
    cs.wmean = d + nslot;
    cs.wm2 = d + (size_t)(1 + SPS_NPARAM) * nslot;
    return cs;
}

// Resume blob: a 256-byte header (HMC_HDR_WORDS ints) and then the chain state of every chain
// in the canonical order q = chain * n_gal + galaxy (the Philox chain id).
constexpr int HMC_MAGIC = 0x48535053, HMC_VERSION = 1, HMC_HDR_WORDS = 12;
struct HmcHeader {
    int w[HMC_HDR_WORDS];   // magic, version, n_gal, n_chain, n_warmup, n_sample, iterations done,
                            // adapt_metric, seed low, seed high, n_leapfrog, 0
};

// Copies the chain state between the working layout (slot = rank * C + chain, galaxies ranked
// by perm) and the blob's canonical layout.  to_blob = 0: blob -> workspace (the header must
// describe this run with it_done = the iterations already run, else STATUS_HMC_STATE); 1:
// workspace -> blob, header written with it_done.
__global__ void __launch_bounds__(256) k_state_move(ChainState ws, ChainState bl, int n_gal, int C,
                                                    const int *__restrict__ perm, int to_blob, HmcHeader hdr,
                                                    int *__restrict__ hdr_dev, int *__restrict__ status) {
    const int nslot = n_gal * C, s = blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < HMC_HDR_WORDS) {
        const int t = threadIdx.x;
        if (to_blob) hdr_dev[t] = hdr.w[t];
        else if (hdr_dev[t] != hdr.w[t]) atomicOr(status, STATUS_HMC_STATE);
    }
    if (s >= nslot) return;
    const int ch = s % C, g = perm ? perm[s / C] : s / C, q = ch * n_gal + g;
    const int src = to_blob ? s : q, dst = to_blob ? q : s;
    const ChainState &from = to_blob ? ws : bl, &to = to_blob ? bl : ws;
#pragma unroll
    for (int p = 0; p < SPS_NPARAM; ++p) {
        const size_t a = (size_t)p * nslot;
        to.x[a + dst] = from.x[a + src];
        to.gr[a + dst] = from.gr[a + src];
        to.minv[a + dst] = from.minv[a + src];
        to.wmean[a + dst] = from.wmean[a + src];
        to.wm2[a + dst] = from.wm2[a + src];
    }
    to.eps[dst] = from.eps[src];
    to.mu[dst] = from.mu[src];
    to.hbar[dst] = from.hbar[src];
    to.lebar[dst] = from.lebar[src];
    to.nacc[dst] = from.nacc[src];
    to.da0[dst] = from.da0[src];
    to.lp[dst] = from.lp[src];
}

static HmcHeader hmc_header(const sps_hmc_cfg *cfg, int n_gal, int it_done) {
    HmcHeader h{};
    h.w[0] = HMC_MAGIC;
    h.w[1] = HMC_VERSION;
    h.w[2] = n_gal;
    h.w[3] = cfg->n_chain;
    h.w[4] = cfg->n_warmup;
    h.w[5] = cfg->n_sample;
    h.w[6] = it_done;
    h.w[7] = cfg->adapt_metric;
    h.w[8] = (int)(uint32_t)(cfg->seed & 0xffffffffull);
    h.w[9] = (int)(uint32_t)(cfg->seed >> 32);
    h.w[10] = cfg->n_leapfrog;
    return h;
}

// blob -> workspace (to_blob = 0, header checked against it_done) or workspace -> blob
static int move_state(sps_ctx *c, hipStream_t s, const ChainState &ws, void *blob, const sps_hmc_cfg *cfg,
                      int n_gal, const int *perm, int to_blob, int it_done) {
    const int nslot = n_gal * cfg->n_chain;
    const ChainState bl = chain_state_at((char *)blob + 256, nslot);
    hipLaunchKernelGGL(k_state_move, dim3((nslot + 255) / 256), dim3(256), 0, s, ws, bl, n_gal, cfg->n_chain,
                       perm, to_blob, hmc_header(cfg, n_gal, it_done), (int *)blob, c->d_status);
    SPS_HIP(hipGetLastError());
    return SPS_OK;
}

// lanes per chain: two adjacent lanes share a chain's model evaluations (each takes half of
// the age bins and bands), so the 65,536 chains of a 16,384-galaxy batch make 2,048 waves,
// two per SIMD.  Both lanes carry the whole chain state, bit for bit the same (every shared
// sum is formed symmetrically), and both write it: each lane only reads back its own writes.
constexpr int HG = 2;

struct HmcArgs {
    int n_gal, C, L, NW, NS, it0, it1, sfh;
    int n_win;                               // slow metric windows (0 = identity metric)
    int win_s[MAX_WIN], win_e[MAX_WIN];      // window w = iterations [win_s, win_e)
    float target, init_step;
    uint32_t key0, key1;
    const float *z, *obs, *sigma;
    const uint8_t *mask;
    const float *bounds, *prior, *theta0;
    const int *perm;
    const uint16_t *qf, *qa;
    float *samples;
    // chain state, indexed by slot = rank * C + chain
    float *x, *gr, *eps, *hbar, *lebar, *mu, *minv;
    int *nacc, *da0;
    double *lp, *wmean, *wm2;
    // trajectory scratch (momentum, position) per lane of the grid, [p][ntmp]: the model
    // evaluation runs with these in memory instead of registers
    float *pm, *xt;
    int ntmp;
};

struct LaneCtx {
    int kk, kmin, kmax;
    float zf, f;
    double t_obs, m0base;
    const float *obs_g, *sig_g;
    uint32_t mask;
};

// The FP64 pieces of an iteration (the prior and the Metropolis test) are out-of-line calls:
// inlined, their constants would be hoisted out of the iteration loop and held in registers
// across the model evaluations.
__device__ __noinline__ double log_prior_all(const float *prior, const float (&x)[NP], float (&dlp)[NP]) {
    double lp = 0.0;
#pragma unroll
    for (int p = 0; p < NP; ++p) lp += log_prior_skewnorm(prior + 3 * p, x[p], dlp[p]);
    return lp;
}
// the same from the constants staged in LDS (stage_prior)
__device__ __noinline__ double log_prior_all_pc(const PriorC *pc, const float (&x)[NP], float (&dlp)[NP]) {
    double lp = 0.0;
#pragma unroll
    for (int p = 0; p < NP; ++p) lp += log_prior_pc(pc[p], x[p], dlp[p]);
    return lp;
}

// Metropolis test of a proposal with energy change dH (FP64) against the uniform word w;
// alpha = min(1, exp(-dH)), 0 for a divergent proposal (non-finite H1 or dH > 1000).
__device__ __noinline__ bool metropolis(double H1, double dH, uint32_t w, float &alpha) {
    const bool divergent = !isfinite(H1) || dH > 1000.0;
    alpha = divergent ? 0.0f : (float)fmin(1.0, exp(-dH));
    return !divergent && log(u01d(w)) < -dH;
}

// Inlined at its one call site per kernel: as an out-of-line call the model would reach the
// kernel-argument constants through a stack copy.
// element p of this lane's trajectory scratch
#define TMP(arr, p) (arr)[(size_t)(p) * a.ntmp + opaque((int)(blockIdx.x * 64 + threadIdx.x))]

// log posterior and its gradient at the position held in the lane's trajectory scratch
template <int SFH>
__device__ __forceinline__ double logpost(const DevConsts &k, const float *ledge, const PriorC *pc, const HmcArgs &a,
                                          const LaneCtx &lc0, const ApproxLds &L, float (&g)[NP]) {
    float x[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) x[p] = TMP(a.xt, p);
    LaneCtx lc = lc0;
    lc.zf = opaque(lc0.zf);
    lc.f = opaque(lc0.f);
    lc.t_obs = opaque(lc0.t_obs);
    lc.m0base = opaque(lc0.m0base);
    float th[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        float dth;
        bound_param(a.bounds + 4 * p, x[p], th[p], dth);
    }
    const double m0 = lc.m0base - 2.5 * (double)th[0];
    double logl;
    float mags[NB_MAX];
    approx_eval<MODE_LOGL_GRAD, false, HG>(k, ledge, SFH, a.qf, a.qa, L, th, lc.zf, lc.kk, lc.f, lc.t_obs, m0, lc.kmin,
                                lc.kmax, lc.obs_g, lc.sig_g, lc.mask, mags, logl, g);
    asm volatile("" ::: "memory");   // the position is read again, not held through the model
#pragma unroll
    for (int p = 0; p < NP; ++p) x[p] = TMP(a.xt, p);
    float dlp[NP];
    const double lp = logl + log_prior_all_pc(pc, x, dlp);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        float t, dth;
        bound_param(a.bounds + 4 * p, x[p], t, dth);   // recomputed: not kept live across the model
        g[p] = fmaf(g[p], dth, dlp[p]);
    }
    return lp;
}

// Chain slot of this lane (slot = rank * C + chain; ranks in z-bucket order) and the
// per-galaxy constants of the model evaluation.
struct SlotInfo {
    int nslot, sl, ch, g;
    bool valid;
    uint32_t chain_id;
};

__device__ inline SlotInfo slot_info(const HmcArgs &a) {
    SlotInfo si;
    si.nslot = a.n_gal * a.C;
    const int slot = (blockIdx.x * 64 + (int)threadIdx.x) / HG;
    si.valid = slot < si.nslot;
    si.sl = si.valid ? slot : si.nslot - 1;
    const int rank = si.sl / a.C;
    si.ch = si.sl % a.C;
    si.g = a.perm[rank];
    si.chain_id = (uint32_t)(si.ch * a.n_gal + si.g);
    return si;
}

__device__ inline LaneCtx lane_ctx(const DevConsts &k, const HmcArgs &a, const SlotInfo &si) {
    LaneCtx lc;
    lc.zf = a.z[si.g];
    lc.kk = z_bucket(k, lc.zf, &lc.f);
    if (!si.valid) lc.kk = -1;
    lc.t_obs = age_universe_gyr(k, (double)lc.zf);
    lc.m0base = mag_offset(k, (double)lc.zf);
    lc.kmin = wave_min_i(lc.kk < 0 ? 1 << 30 : lc.kk);
    lc.kmax = wave_max_i(lc.kk);
    lc.obs_g = a.obs + (size_t)si.g * k.n_band;
    lc.sig_g = a.sigma + (size_t)si.g * k.n_band;
    lc.mask = a.mask[si.g];
    return lc;
}

// element p of the lane's slot in a state array; the slot index is made opaque at each use so
// that the addresses are formed where they are used, not hoisted and held across the loop
#define ST(arr, p) (arr)[(size_t)(p) * si.nslot + opaque(si.sl)]

// Chain start: log posterior and gradient at the initial point, unit metric, step-size
// adaptation state.
template <int SFH>
__global__ void __launch_bounds__(64) k_hmc_init(DevConsts k, HmcArgs a) {
    extern __shared__ __attribute__((aligned(16))) char lds_dyn[];   // approx_lds_bytes(n_band, false, HG)
    const ApproxLds lds = approx_lds(lds_dyn, k.n_band, false, HG);
    __shared__ float ledge[NA + 1];
    stage_log_age_edges(k, ledge);
    __shared__ PriorC pcs[NP];
    stage_prior(a.prior, pcs);
    const SlotInfo si = slot_info(a);
    const LaneCtx lc = lane_ctx(k, a, si);
    float x[NP], gr[NP];
    if (a.theta0) {
#pragma unroll
        for (int p = 0; p < NP; ++p) x[p] = a.theta0[((size_t)si.ch * NP + p) * a.n_gal + si.g];
    } else {
        prior_draw(a.prior, a.key0, a.key1, si.chain_id, x);
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) TMP(a.xt, p) = x[p];
    const double lp = logpost<SFH>(k, ledge, pcs, a, lc, lds, gr);
    if (!si.valid) return;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        ST(a.x, p) = x[p];
        ST(a.gr, p) = gr[p];
        ST(a.minv, p) = 1.0f;
        ST(a.wmean, p) = 0.0;
        ST(a.wm2, p) = 0.0;
    }
    a.lp[si.sl] = lp;
    a.eps[si.sl] = a.init_step;
    a.mu[si.sl] = logf(10.0f * a.init_step);
    a.hbar[si.sl] = 0.0f;
    a.lebar[si.sl] = 0.0f;
    a.nacc[si.sl] = 0;
    a.da0[si.sl] = 0;
}

// Iterations [it0, it1) of every chain.  Chain state lives in HBM (SoA [quantity][slot],
// coalesced across the wave) and is read where it is used, so that only the trajectory
// (x, p, M^-1 and the scalars of the step-size adaptation) stays in registers across the
// model evaluations.
template <int SFH>
__global__ void __launch_bounds__(64, 2) k_hmc(DevConsts k, HmcArgs a) {
    extern __shared__ __attribute__((aligned(16))) char lds_dyn[];   // approx_lds_bytes(n_band, false, HG)
    const ApproxLds lds = approx_lds(lds_dyn, k.n_band, false, HG);
    __shared__ float ledge[NA + 1];
    stage_log_age_edges(k, ledge);
    __shared__ PriorC pcs[NP];
    stage_prior(a.prior, pcs);
    const SlotInfo si = slot_info(a);
    const LaneCtx lc = lane_ctx(k, a, si);
    const bool valid = si.valid;
    const int ch = si.ch, g = si.g, sl = si.sl;
    const uint32_t chain_id = si.chain_id;

    double lp = a.lp[sl];
    float eps = a.eps[sl], mu = a.mu[sl], hbar = a.hbar[sl], lebar = a.lebar[sl];
    int nacc = a.nacc[sl], da0 = a.da0[sl];

    for (int it = a.it0; it < a.it1; ++it) {
        float p[NP], xn[NP], gn[NP];
        {
            uint32_t w[NP];
#pragma unroll
            for (int blk = 0; blk < 3; ++blk) {
                uint32_t c4[4] = {(uint32_t)blk, (uint32_t)it, chain_id, 0u};
                philox4x32_10(c4, a.key0, a.key1);
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (4 * blk + t < NP) w[4 * blk + t] = c4[t];
            }
#pragma unroll
            for (int t = 0; t < NP / 2; ++t) {
                const float r = sqrtf(-2.0f * logf(u01f(w[2 * t])));
                float sn, cs;
                sincosf(6.283185307179586f * u01f(w[2 * t + 1]), &sn, &cs);
                p[2 * t] = r * cs / sqrtf(ST(a.minv, 2 * t));
                p[2 * t + 1] = r * sn / sqrtf(ST(a.minv, 2 * t + 1));
            }
        }
        double H0 = -lp;
#pragma unroll
        for (int t = 0; t < NP; ++t) {
            H0 += 0.5 * (double)ST(a.minv, t) * (double)p[t] * (double)p[t];
            TMP(a.xt, t) = ST(a.x, t);
            gn[t] = ST(a.gr, t);
        }
        double lpn = lp;
        for (int l = 0; l < a.L; ++l) {
            // half kick and drift; momentum and position go to the trajectory scratch for the
            // model evaluation
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                p[t] = fmaf(0.5f * eps, gn[t], p[t]);
                TMP(a.pm, t) = p[t];
                TMP(a.xt, t) = fmaf(eps * ST(a.minv, t), p[t], TMP(a.xt, t));
            }
            asm volatile("" ::: "memory");
            lpn = logpost<SFH>(k, ledge, pcs, a, lc, lds, gn);
            asm volatile("" ::: "memory");
#pragma unroll
            for (int t = 0; t < NP; ++t) p[t] = fmaf(0.5f * eps, gn[t], TMP(a.pm, t));
        }
#pragma unroll
        for (int t = 0; t < NP; ++t) xn[t] = TMP(a.xt, t);
        double H1 = -lpn;
#pragma unroll
        for (int t = 0; t < NP; ++t) H1 += 0.5 * (double)ST(a.minv, t) * (double)p[t] * (double)p[t];
        uint32_t c4[4] = {2u, (uint32_t)it, chain_id, 0u};   // the accept draw: word 2 of block 2
        philox4x32_10(c4, a.key0, a.key1);
        float alpha;
        const bool acc = metropolis(H1, H1 - H0, c4[2], alpha);
        // xn now holds the chain's position after this iteration
        if (acc) {
            lp = lpn;
            if (valid) {
#pragma unroll
                for (int t = 0; t < NP; ++t) {
                    ST(a.x, t) = xn[t];
                    ST(a.gr, t) = gn[t];
                }
            }
        } else {
#pragma unroll
            for (int t = 0; t < NP; ++t) xn[t] = ST(a.x, t);
        }
        if (it < a.NW) {
            const float m = (float)(it - da0 + 1), eta = 1.0f / (m + 10.0f);
            hbar = (1.0f - eta) * hbar + eta * (a.target - alpha);
            const float leps = mu - sqrtf(m) / 0.05f * hbar, wk = powf(m, -0.75f);
            lebar = wk * leps + (1.0f - wk) * lebar;
            eps = expf(it == a.NW - 1 ? lebar : leps);
            // slow metric window holding iteration it (uniform across the grid)
            int wi = -1;
            for (int q = 0; q < a.n_win; ++q)
                if (it >= a.win_s[q] && it < a.win_e[q]) wi = q;
            if (wi >= 0) {
                const double nn = (double)(it - a.win_s[wi] + 1);
                const bool last = (it == a.win_e[wi] - 1);
#pragma unroll
                for (int t = 0; t < NP; ++t) {
                    double wmean = ST(a.wmean, t), wm2 = ST(a.wm2, t);
                    const double d = (double)xn[t] - wmean;
                    wmean += d / nn;
                    wm2 += d * ((double)xn[t] - wmean);
                    if (last) {
                        if (valid) ST(a.minv, t) = (float)(nn / (nn + 5.0) * (wm2 / (nn - 1.0)) + 1e-3 * 5.0 / (nn + 5.0));
                        wmean = wm2 = 0.0;
                    }
                    if (valid) {
                        ST(a.wmean, t) = wmean;
                        ST(a.wm2, t) = wm2;
                    }
                }
                if (last) {
                    mu = logf(10.0f * eps);
                    hbar = lebar = 0.0f;
                    da0 = it + 1;
                }
            }
        } else {
            nacc += acc ? 1 : 0;
            const double nrec = (double)(it - a.NW + 1);
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                float th, dth;
                bound_param(a.bounds + 4 * t, xn[t], th, dth);
                double wmean = ST(a.wmean, t), wm2 = ST(a.wm2, t);
                const double d = (double)th - wmean;
                wmean += d / nrec;
                wm2 += d * ((double)th - wmean);
                if (valid) {
                    ST(a.wmean, t) = wmean;
                    ST(a.wm2, t) = wm2;
                    if (a.samples) a.samples[(((size_t)(it - a.NW) * a.C + ch) * NP + t) * a.n_gal + g] = th;
                }
            }
        }
    }
    if (!valid) return;
    a.lp[sl] = lp;
    a.eps[sl] = eps;
    a.mu[sl] = mu;
    a.hbar[sl] = hbar;
    a.lebar[sl] = lebar;
    a.nacc[sl] = nacc;
    a.da0[sl] = da0;
}
#undef ST

// pooled posterior mean / sd, classic Gelman-Rubin R-hat and acceptance per galaxy; slot
// r * C + c holds chain c of galaxy perm[r] (of galaxy r if perm is null).  Acceptance: the
// accepted count nacc, or (nacc null) the summed acceptance statistic accsum, over C x NS.
__global__ void k_hmc_summary(int n_gal, int C, int NS, const int *__restrict__ perm,
                              const double *__restrict__ wmean, const double *__restrict__ wm2,
                              const int *__restrict__ nacc, const double *__restrict__ accsum,
                              const float *__restrict__ eps, const float *__restrict__ minv, float *post_mean,
                              float *post_sd, float *rhat, float *accept, float *step, float *inv_metric) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_gal) return;
    const int g = perm ? perm[r] : r, nslot = n_gal * C;
    double acc = 0.0;
    for (int c = 0; c < C; ++c) {
        acc += nacc ? (double)nacc[r * C + c] : accsum[r * C + c];
        step[(size_t)c * n_gal + g] = eps[r * C + c];
        if (inv_metric)
            for (int p = 0; p < NP; ++p)
                inv_metric[((size_t)c * NP + p) * n_gal + g] = minv[(size_t)p * nslot + r * C + c];
    }
    accept[g] = (float)(acc / ((double)C * NS));
    for (int p = 0; p < NP; ++p) {
        double gm = 0.0, W = 0.0, B = 0.0, ss = 0.0;
        for (int c = 0; c < C; ++c) {
            const size_t o = (size_t)p * nslot + r * C + c;
            gm += wmean[o];
            W += wm2[o] / (NS - 1);
        }
        gm /= C;
        W /= C;
        for (int c = 0; c < C; ++c) {
            const size_t o = (size_t)p * nslot + r * C + c;
            const double d = wmean[o] - gm;
            B += d * d;
            ss += wm2[o] + NS * d * d;
        }
        const double Bn = (C > 1) ? B / (C - 1) : 0.0;
        const double V = (NS - 1.0) / NS * W + Bn;
        post_mean[(size_t)p * n_gal + g] = (float)gm;
        post_sd[(size_t)p * n_gal + g] = (float)sqrt(ss / ((double)C * NS - 1.0));
        rhat[(size_t)p * n_gal + g] = (C > 1) ? (float)sqrt(V / W) : __int_as_float(0x7fc00000);
    }
}

// ------------------------------------------------------------------ NUTS
// The No-U-Turn Sampler (Sec. 4 and App. D.2 run it beside HMC): Hoffman & Gelman (2014),
// Algorithm 3 (slice variable, trajectory doubling in a random direction, a new subtree's
// proposal taken with probability min(1, n'/n)) with the dual averaging of their Algorithm 6
// (acceptance statistic: the mean of min(1, exp(H0 - H)) over the final tree's leaves).  The
// recursive tree building is run leaf by leaf as a per-chain state machine: after each leaf
// the U-turn test runs on every dyadic block of the subtree that ends there (innermost
// first), and a divergent leaf (log u >= 1000 - H) or a turned block ends the subtree.  Inside
// a subtree the proposal is a uniform choice among its slice-valid leaves (reservoir
// sampling, the distribution the recursion's pairwise choices give).  Diagonal metric: the
// U-turn test uses the velocities M^-1 p.
//
// Lock-step: the chains of a wave evaluate the model together (the contractions are
// wave-wide), so every leaf step costs the whole wave and a chain whose tree is done waits
// for the wave's slowest.  With sync = 1 the chains of a wave also start every iteration
// together (the vectorised-over-chains form, where each iteration lasts as long as the
// wave's deepest tree); with sync = 0 a chain whose tree is done begins its next iteration at
// once, so the wave's cost is the slowest chain's total over the launch's iterations, not
// the sum of per-iteration maxima.  The draws do not depend on it.
//
// Philox draws (chain id = c * n_gal + g): momentum and slice (blk 0..2, it, chain, 0:
// words 0..9 the momentum as in HMC, word 10 the slice uniform), per doubling j (j, it,
// chain, 2: word 0 the direction, word 1 the subtree's acceptance), per leaf (leaf index in
// the iteration, it, chain, 3: word 0 the reservoir uniform).
constexpr int NUTS_MAX_DEPTH = 12;

struct NutsArgs : HmcArgs {
    int D;                    // maximum tree depth: at most 2^D - 1 leaves per iteration
    int sync;                 // 1: a wave's chains start each iteration together
    // tree state per slot, [quantity][slot]: the two ends (position, momentum, gradient), the
    // proposal, the current subtree's proposal, the dyadic-block checkpoints [D][2][NP][slot]
    float *xl, *pl, *gl, *xr, *pr, *grr, *xm, *gm, *xs, *gs, *ck;
    double *lpl, *lpr, *lpm, *lps, *asum_it, *accsum;   // [slot]
    int *nleaf;               // [slot] leapfrog steps over the run
    int *depth_out;           // [n_it][C][n_gal] tree depth per iteration, or null
    unsigned long long *lockstep;   // [2]: chain leapfrog steps, wave leaf steps x chains per wave
};

// no U-turn between two forward-time ends of a stretch (both dot products >= 0); the first
// end at xa/pa (SoA, slot s), the second in registers
__device__ inline bool no_uturn_at(const float *xa, const float *pa, size_t ns, int s, const float (&xb)[NP],
                                   const float (&pb)[NP], const float *minv_s, int dirn) {
    float da = 0.0f, db = 0.0f;
#pragma unroll
    for (int t = 0; t < NP; ++t) {
        const float mi = minv_s[(size_t)t * ns];
        const float dx = (float)dirn * (xb[t] - xa[(size_t)t * ns + s]);
        da = fmaf(dx * mi, pa[(size_t)t * ns + s], da);
        db = fmaf(dx * mi, pb[t], db);
    }
    return da >= 0.0f && db >= 0.0f;
}

#define NS_(arr, p) (arr)[(size_t)(p) * si.nslot + opaque(si.sl)]
#define ST(arr, p) (arr)[(size_t)(p) * si.nslot + opaque(si.sl)]

enum { NU_START = 0, NU_SUB = 1, NU_LEAF = 2 };

template <int SFH>
__global__ void __launch_bounds__(64, 2) k_nuts(DevConsts k, NutsArgs a) {
    extern __shared__ __attribute__((aligned(16))) char lds_dyn[];   // approx_lds_bytes(n_band, false, HG)
    const ApproxLds lds = approx_lds(lds_dyn, k.n_band, false, HG);
    __shared__ float ledge[NA + 1];
    stage_log_age_edges(k, ledge);
    __shared__ PriorC pcs[NP];
    stage_prior(a.prior, pcs);
    const SlotInfo si = slot_info(a);
    const LaneCtx lc = lane_ctx(k, a, si);
    const uint32_t chain_id = si.chain_id;
    const int D = a.D;
#pragma unroll
    for (int p = 0; p < NP; ++p) TMP(a.xt, p) = ST(a.x, p);

    int it = a.it0, phase = NU_START, j = 0, kk = 0, dirn = 1, n = 1, nsub = 0, leaf = 0;
    bool done = !si.valid || it >= a.it1, s_sub = true;
    double logu = 0.0, H0 = 0.0, asum = 0.0;
    float eps = a.eps[si.sl];
    unsigned long long wave_steps = 0, my_leaves = 0;

    while (__any(!done)) {
        // wave-wide, so taken by every lane before any branch: are all unfinished chains
        // between iterations?
        const bool all_between = __all(done || phase == NU_START);
        bool act = !done;
        if (a.sync && phase == NU_START && !all_between) act = false;
        if (act && phase == NU_START) {   // a new iteration: momentum, slice, the one-leaf tree
            uint32_t w[12];
#pragma unroll
            for (int blk = 0; blk < 3; ++blk) {
                uint32_t c4[4] = {(uint32_t)blk, (uint32_t)it, chain_id, 0u};
                philox4x32_10(c4, a.key0, a.key1);
#pragma unroll
                for (int t = 0; t < 4; ++t) w[4 * blk + t] = c4[t];
            }
            double kin = 0.0;
#pragma unroll
            for (int t = 0; t < NP / 2; ++t) {
                const float r = sqrtf(-2.0f * logf(u01f(w[2 * t])));
                float sn, cs;
                sincosf(6.283185307179586f * u01f(w[2 * t + 1]), &sn, &cs);
                const float m0 = ST(a.minv, 2 * t), m1 = ST(a.minv, 2 * t + 1);
                const float p0 = r * cs / sqrtf(m0), p1 = r * sn / sqrtf(m1);
                kin += 0.5 * (double)m0 * (double)p0 * (double)p0 + 0.5 * (double)m1 * (double)p1 * (double)p1;
                NS_(a.pl, 2 * t) = p0;
                NS_(a.pr, 2 * t) = p0;
                NS_(a.pl, 2 * t + 1) = p1;
                NS_(a.pr, 2 * t + 1) = p1;
            }
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                const float x = ST(a.x, t), g = ST(a.gr, t);
                NS_(a.xl, t) = x;
                NS_(a.xr, t) = x;
                NS_(a.xm, t) = x;
                NS_(a.gl, t) = g;
                NS_(a.grr, t) = g;
                NS_(a.gm, t) = g;
            }
            const double lp = a.lp[si.sl];
            a.lpl[si.sl] = lp;
            a.lpr[si.sl] = lp;
            a.lpm[si.sl] = lp;
            H0 = -lp + kin;
            logu = log(u01d(w[10])) - H0;
            n = 1;
            j = 0;
            leaf = 0;
            asum = 0.0;
            eps = a.eps[si.sl];
            phase = NU_SUB;
        }
        if (act && phase == NU_SUB) {   // a new subtree of 2^j leaves in a random direction
            uint32_t c4[4] = {(uint32_t)j, (uint32_t)it, chain_id, 2u};
            philox4x32_10(c4, a.key0, a.key1);
            dirn = u01d(c4[0]) < 0.5 ? -1 : 1;
            nsub = 0;
            s_sub = true;
            kk = 0;
            phase = NU_LEAF;
        }
        // one leapfrog step from the growing end (every lane evaluates the model; only the
        // active ones keep the result)
        float *ex = dirn < 0 ? a.xl : a.xr, *ep = dirn < 0 ? a.pl : a.pr, *eg = dirn < 0 ? a.gl : a.grr;
        const float e = (float)dirn * eps;
        if (act) {
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                const float p = fmaf(0.5f * e, NS_(eg, t), NS_(ep, t));
                NS_(ep, t) = p;
                const float x = fmaf(e * ST(a.minv, t), p, NS_(ex, t));
                NS_(ex, t) = x;
                TMP(a.xt, t) = x;
            }
        }
        asm volatile("" ::: "memory");
        float ge[NP];
        const double lpe = logpost<SFH>(k, ledge, pcs, a, lc, lds, ge);
        asm volatile("" ::: "memory");
        ++wave_steps;
        if (!act) continue;
        float xe[NP], pe[NP];
        double kin = 0.0;
#pragma unroll
        for (int t = 0; t < NP; ++t) {
            xe[t] = NS_(ex, t);
            pe[t] = fmaf(0.5f * e, ge[t], NS_(ep, t));
            NS_(ep, t) = pe[t];
            NS_(eg, t) = ge[t];
            kin += 0.5 * (double)ST(a.minv, t) * (double)pe[t] * (double)pe[t];
        }
        (dirn < 0 ? a.lpl : a.lpr)[si.sl] = lpe;
        const double H = -lpe + kin;
        asum += isfinite(H) ? fmin(1.0, exp(H0 - H)) : 0.0;
        ++leaf;
        if (logu <= -H) {   // a slice-valid leaf: the subtree's proposal with probability 1 / nsub
            ++nsub;
            uint32_t c4[4] = {(uint32_t)(leaf - 1), (uint32_t)it, chain_id, 3u};
            philox4x32_10(c4, a.key0, a.key1);
            if (u01d(c4[0]) * (double)nsub < 1.0) {
#pragma unroll
                for (int t = 0; t < NP; ++t) {
                    NS_(a.xs, t) = xe[t];
                    NS_(a.gs, t) = ge[t];
                }
                a.lps[si.sl] = lpe;
            }
        }
        if (!(logu < 1000.0 - H)) s_sub = false;   // divergence (or a non-finite H)
        const size_t cstride = (size_t)2 * NP * si.nslot;
        for (int l = 1; l <= j; ++l)   // the first leaf of every dyadic block starting here
            if ((kk & ((1 << l) - 1)) == 0) {
                float *cx = a.ck + (size_t)(l - 1) * cstride, *cp = cx + (size_t)NP * si.nslot;
#pragma unroll
                for (int t = 0; t < NP; ++t) {
                    NS_(cx, t) = xe[t];
                    NS_(cp, t) = pe[t];
                }
            }
        for (int l = 1; l <= j && s_sub; ++l)   // every block ending here, innermost first
            if (((kk + 1) & ((1 << l) - 1)) == 0) {
                const float *cx = a.ck + (size_t)(l - 1) * cstride, *cp = cx + (size_t)NP * si.nslot;
                if (!no_uturn_at(cx, cp, si.nslot, opaque(si.sl), xe, pe, a.minv + opaque(si.sl), dirn))
                    s_sub = false;
            }
        ++kk;
        if (kk < (1 << j) && s_sub) continue;
        // the subtree is done: its proposal replaces the tree's with probability min(1, nsub / n)
        {
            uint32_t c4[4] = {(uint32_t)j, (uint32_t)it, chain_id, 2u};
            philox4x32_10(c4, a.key0, a.key1);
            if (s_sub && nsub > 0 && u01d(c4[1]) * (double)n < (double)nsub) {
#pragma unroll
                for (int t = 0; t < NP; ++t) {
                    NS_(a.xm, t) = NS_(a.xs, t);
                    NS_(a.gm, t) = NS_(a.gs, t);
                }
                a.lpm[si.sl] = a.lps[si.sl];
            }
        }
        n += nsub;
        bool s_tree = s_sub;
        if (s_tree) {
            float xb[NP], pb[NP];
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                xb[t] = NS_(a.xr, t);
                pb[t] = NS_(a.pr, t);
            }
            s_tree = no_uturn_at(a.xl, a.pl, si.nslot, opaque(si.sl), xb, pb, a.minv + opaque(si.sl), 1);
        }
        ++j;
        if (s_tree && j < D) {
            phase = NU_SUB;
            continue;
        }
        // the iteration is done: the proposal becomes the chain's state
        float xn[NP];
#pragma unroll
        for (int t = 0; t < NP; ++t) {
            xn[t] = NS_(a.xm, t);
            ST(a.x, t) = xn[t];
            ST(a.gr, t) = NS_(a.gm, t);
        }
        a.lp[si.sl] = a.lpm[si.sl];
        const float alpha = (float)(asum / (double)leaf);
        my_leaves += (unsigned long long)leaf;
        a.nleaf[si.sl] += leaf;
        if (a.depth_out) a.depth_out[((size_t)it * a.C + si.ch) * a.n_gal + si.g] = j;
        if (it < a.NW) {   // dual averaging and the metric windows, as in HMC
            int da0 = a.da0[si.sl];
            const float m = (float)(it - da0 + 1), eta = 1.0f / (m + 10.0f);
            float hbar = (1.0f - eta) * a.hbar[si.sl] + eta * (a.target - alpha);
            const float leps = a.mu[si.sl] - sqrtf(m) / 0.05f * hbar, wk = powf(m, -0.75f);
            float lebar = wk * leps + (1.0f - wk) * a.lebar[si.sl];
            eps = expf(it == a.NW - 1 ? lebar : leps);
            int wi = -1;
            for (int q = 0; q < a.n_win; ++q)
                if (it >= a.win_s[q] && it < a.win_e[q]) wi = q;
            if (wi >= 0) {
                const double nn = (double)(it - a.win_s[wi] + 1);
                const bool wlast = (it == a.win_e[wi] - 1);
#pragma unroll
                for (int t = 0; t < NP; ++t) {
                    double wmean = ST(a.wmean, t), wm2 = ST(a.wm2, t);
                    const double d = (double)xn[t] - wmean;
                    wmean += d / nn;
                    wm2 += d * ((double)xn[t] - wmean);
                    if (wlast) {
                        ST(a.minv, t) = (float)(nn / (nn + 5.0) * (wm2 / (nn - 1.0)) + 1e-3 * 5.0 / (nn + 5.0));
                        wmean = wm2 = 0.0;
                    }
                    ST(a.wmean, t) = wmean;
                    ST(a.wm2, t) = wm2;
                }
                if (wlast) {
                    a.mu[si.sl] = logf(10.0f * eps);
                    hbar = lebar = 0.0f;
                    a.da0[si.sl] = it + 1;
                }
            }
            a.hbar[si.sl] = hbar;
            a.lebar[si.sl] = lebar;
            a.eps[si.sl] = eps;
        } else {
            a.accsum[si.sl] += (double)alpha;
            const double nrec = (double)(it - a.NW + 1);
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                float th, dth;
                bound_param(a.bounds + 4 * t, xn[t], th, dth);
                double wmean = ST(a.wmean, t), wm2 = ST(a.wm2, t);
                const double d = (double)th - wmean;
                wmean += d / nrec;
                wm2 += d * ((double)th - wmean);
                ST(a.wmean, t) = wmean;
                ST(a.wm2, t) = wm2;
                if (a.samples) a.samples[(((size_t)(it - a.NW) * a.C + si.ch) * NP + t) * a.n_gal + si.g] = th;
            }
        }
        ++it;
        phase = NU_START;
        if (it >= a.it1) done = true;
    }
    if (a.lockstep) {   // one lane per chain counts its steps; lane 0 the wave's
        const bool own = si.valid && (threadIdx.x % HG) == 0;
        unsigned long long chains = own ? 1ull : 0ull, mine = own ? my_leaves : 0ull;
#pragma unroll
        for (int o = 1; o < WAVE; o <<= 1) {
            chains += __shfl_xor(chains, o, WAVE);
            mine += __shfl_xor(mine, o, WAVE);
        }
        if (threadIdx.x == 0) {
            atomicAdd(&a.lockstep[0], mine);
            atomicAdd(&a.lockstep[1], wave_steps * chains);
        }
    }
}
#undef NS_
#undef ST

__global__ void k_zero_words(uint32_t *__restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// per-slot leapfrog counts to the caller's [n_chain][n_gal] order
__global__ void k_nuts_leaves(int n_gal, int C, const int *__restrict__ perm, const int *__restrict__ nl,
                              int *__restrict__ out) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n_gal * C) return;
    out[(size_t)(s % C) * n_gal + perm[s / C]] = nl[s];
}

static int metric_windows(int nw, int *ws, int *we);

// the NUTS workspace: the HMC chain state and trajectory scratch, then the tree state
struct NutsLayout {
    size_t o_tree, o_ck, o_d, o_i, bytes;
};
static NutsLayout nuts_layout(int nslot, int D) {
    NutsLayout L{};
    size_t off = hmc_state_bytes(nslot);
    L.o_tree = off;
    off += align256((size_t)10 * NP * nslot * sizeof(float));
    L.o_ck = off;
    off += align256((size_t)D * 2 * NP * nslot * sizeof(float));
    L.o_d = off;
    off += align256((size_t)6 * nslot * sizeof(double));
    L.o_i = off;
    off += align256((size_t)nslot * sizeof(int));
    L.bytes = off;
    return L;
}
size_t nuts_state_bytes(int nslot, int max_depth) { return nuts_layout(nslot, max_depth).bytes; }

int launch_nuts(sps_ctx *c, hipStream_t s, const sps_nuts_cfg *cfg, int n_gal, int sfh, const float *z,
                const float *obs, const float *sigma, const uint8_t *mask, const float *bounds, const float *prior,
                const float *theta0, float *samples, float *post_mean, float *post_sd, float *rhat, float *accept,
                float *step, float *inv_metric, int *depth, int *n_leaf, unsigned long long *lockstep) {
    const int C = cfg->n_chain, nslot = n_gal * C, D = cfg->max_depth;
    const NutsLayout L = nuts_layout(nslot, D);
    if (c->nwork_bytes < L.bytes)
        return set_error(SPS_E_STATE, "the NUTS workspace needs n_gal * n_chain chains at this max_depth "
                                      "(call sps_reserve_nuts)");
    NutsArgs a{};
    a.n_win = 0;
    if (cfg->adapt_metric) {
        a.n_win = metric_windows(cfg->n_warmup, a.win_s, a.win_e);
        if (a.n_win < 0) return set_error(SPS_E_INVAL, "n_warmup too long for the metric-window table");
    }
    int rc = launch_bucket_sort(c, s, n_gal, z);
    if (rc) return rc;
    char *W = (char *)c->d_nwork;
    const ChainState cs = chain_state_at(W, nslot);
    a.n_gal = n_gal;
    a.C = C;
    a.L = 0;
    a.NW = cfg->n_warmup;
    a.NS = cfg->n_sample;
    a.sfh = sfh;
    a.target = cfg->target_accept;
    a.init_step = cfg->init_step;
    a.key0 = (uint32_t)(cfg->seed & 0xffffffffull);
    a.key1 = (uint32_t)(cfg->seed >> 32);
    a.z = z;
    a.obs = obs;
    a.sigma = sigma;
    a.mask = mask;
    a.bounds = bounds;
    a.prior = prior;
    a.theta0 = theta0;
    a.perm = c->d_perm;
    a.qf = c->d_qf;
    a.qa = c->d_qa;
    a.samples = samples;
    a.x = cs.x;
    a.gr = cs.gr;
    a.minv = cs.minv;
    a.eps = cs.eps;
    a.mu = cs.mu;
    a.hbar = cs.hbar;
    a.lebar = cs.lebar;
    a.nacc = cs.nacc;
    a.da0 = cs.da0;
    a.lp = cs.lp;
    a.wmean = cs.wmean;
    a.wm2 = cs.wm2;
    const int ntmp = (nslot * HG + 63) / 64 * 64;
    a.pm = (float *)(W + chain_state_bytes(nslot));
    a.xt = a.pm + (size_t)NP * ntmp;
    a.ntmp = ntmp;
    a.D = D;
    a.sync = cfg->sync_iterations;
    float *tf = (float *)(W + L.o_tree);
    float **tq[10] = {&a.xl, &a.pl, &a.gl, &a.xr, &a.pr, &a.grr, &a.xm, &a.gm, &a.xs, &a.gs};
    for (int q = 0; q < 10; ++q) *tq[q] = tf + (size_t)q * NP * nslot;
    a.ck = (float *)(W + L.o_ck);
    double *td = (double *)(W + L.o_d);
    double **dq[6] = {&a.lpl, &a.lpr, &a.lpm, &a.lps, &a.asum_it, &a.accsum};
    for (int q = 0; q < 6; ++q) *dq[q] = td + (size_t)q * nslot;
    a.nleaf = (int *)(W + L.o_i);
    a.depth_out = depth;
    a.lockstep = lockstep;
    // counters start at zero (fill kernels rather than memset nodes, so the sequence can be
    // captured in a graph)
    hipLaunchKernelGGL(k_zero_words, dim3((2 * nslot + 255) / 256), dim3(256), 0, s, (uint32_t *)a.accsum,
                       (size_t)2 * nslot);
    hipLaunchKernelGGL(k_zero_words, dim3((nslot + 255) / 256), dim3(256), 0, s, (uint32_t *)a.nleaf, (size_t)nslot);
    if (lockstep) hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, (uint32_t *)lockstep, (size_t)4);
    dim3 grid((nslot * HG + 63) / 64), block(64);
    const bool dpl = (sfh == SPS_SFH_DPL);
    const size_t lds_bytes = approx_lds_bytes(c->n_band, false, HG);
    const HmcArgs &ha = a;
    if (dpl) hipLaunchKernelGGL(k_hmc_init<SPS_SFH_DPL>, grid, block, lds_bytes, s, c->k, ha);
    else hipLaunchKernelGGL(k_hmc_init<SPS_SFH_LOGNORMAL>, grid, block, lds_bytes, s, c->k, ha);
    const int nit = cfg->n_warmup + cfg->n_sample, blk_it = c->launch.nuts_block_iters;
    for (int b0 = 0; b0 < nit; b0 += blk_it) {
        a.it0 = b0;
        a.it1 = b0 + blk_it < nit ? b0 + blk_it : nit;
        if (dpl) hipLaunchKernelGGL(k_nuts<SPS_SFH_DPL>, grid, block, lds_bytes, s, c->k, a);
        else hipLaunchKernelGGL(k_nuts<SPS_SFH_LOGNORMAL>, grid, block, lds_bytes, s, c->k, a);
    }
    hipLaunchKernelGGL(k_hmc_summary, dim3((n_gal + 255) / 256), dim3(256), 0, s, n_gal, C, cfg->n_sample, c->d_perm,
                       a.wmean, a.wm2, (const int *)nullptr, a.accsum, a.eps, a.minv, post_mean, post_sd, rhat,
                       accept, step, inv_metric);
    if (n_leaf)
        hipLaunchKernelGGL(k_nuts_leaves, dim3((nslot + 255) / 256), dim3(256), 0, s, n_gal, C, c->d_perm, a.nleaf,
                           n_leaf);
    SPS_HIP(hipGetLastError());
    return SPS_OK;
}

// ------------------------------------------------------------------ exact-path HMC
// With exact photometry the model is a GEMM over all chains at once (Sec. 3), so the
// leapfrog runs as a host loop: each step is one exact value+gradient call over every chain
// (the likelihood entry point's own kernels), with small per-chain kernels around it for
// the kicks, the drift and the end of the iteration.  Slot = rank * C + chain with the
// galaxies ranked by z (the z table's buckets, or z_sort_grid's without a table), so a
// 128-row tile of the GEMMs spans a narrow z range and skips the wavelengths outside its
// filters' support.  Chain ids, Philox counters, the FP32 trajectory arithmetic, the FP64
// Hamiltonian and the adaptation are those of the fused approximate-path kernel.
struct HmcxArgs {
    int n_gal, C, nslot, nb, NW, NS;
    int n_win;
    int win_s[MAX_WIN], win_e[MAX_WIN];
    float target, init_step;
    uint32_t key0, key1;
    const float *z, *obs, *sigma;
    const uint8_t *mask;
    const float *bounds, *prior, *theta0;
    const int *perm;           // galaxy of each rank (z order)
    float *samples;
    // chain state, [quantity][slot]
    float *x, *gr, *minv, *eps, *mu, *hbar, *lebar;
    int *nacc, *da0;
    double *lp, *h0, *wmean, *wm2;
    // trajectory (momentum, position), the physical parameters of the model call and its
    // outputs (log L, gradient w.r.t. the physical parameters)
    float *pm, *xt, *th, *logl, *grad;
    // per-slot copies of the galaxy's inputs, the layout the exact path reads
    float *zs, *obs_s, *sig_s;
    uint8_t *mask_s;
    // iteration index in device memory (a captured iteration reads it there), or null: the
    // kernels' own argument
    int *itp;
};

#define XS(arr, p) (arr)[(size_t)(p) * a.nslot + s]

// per-slot inputs and (start = 1) the starting point
__global__ void __launch_bounds__(256) k_hmcx_setup(HmcxArgs a, int start) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= a.nslot) return;
    const int g = a.perm[s / a.C], ch = s % a.C;
    a.zs[s] = a.z[g];
    for (int b = 0; b < a.nb; ++b) {
        a.obs_s[(size_t)s * a.nb + b] = a.obs[(size_t)g * a.nb + b];
        a.sig_s[(size_t)s * a.nb + b] = a.sigma[(size_t)g * a.nb + b];
    }
    a.mask_s[s] = a.mask[g];
    if (!start) return;   // a resumed run: the chain state comes from the blob
    float x[NP];
    if (a.theta0) {
#pragma unroll
        for (int p = 0; p < NP; ++p) x[p] = a.theta0[((size_t)ch * NP + p) * a.n_gal + g];
    } else {
        prior_draw(a.prior, a.key0, a.key1, (uint32_t)(ch * a.n_gal + g), x);
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        float th, dth;
        bound_param(a.bounds + 4 * p, x[p], th, dth);
        XS(a.xt, p) = x[p];
        XS(a.th, p) = th;
    }
}

// log posterior on the unbounded parameters at the trajectory position from the model
// call's log L and physical-parameter gradient: prior added, chain rule through F_B
__device__ inline double hmcx_logpost(const HmcxArgs &a, int s, float (&x)[NP], float (&g)[NP]) {
#pragma unroll
    for (int p = 0; p < NP; ++p) x[p] = XS(a.xt, p);
    float dlp[NP];
    const double lp = (double)a.logl[s] + log_prior_all(a.prior, x, dlp);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        float th, dth;
        bound_param(a.bounds + 4 * p, x[p], th, dth);
        g[p] = fmaf(XS(a.grad, p), dth, dlp[p]);
    }
    return lp;
}

__global__ void __launch_bounds__(256) k_hmcx_init(HmcxArgs a) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= a.nslot) return;
    float x[NP], g[NP];
    const double lp = hmcx_logpost(a, s, x, g);
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        XS(a.x, p) = x[p];
        XS(a.gr, p) = g[p];
        XS(a.minv, p) = 1.0f;
        XS(a.wmean, p) = 0.0;
        XS(a.wm2, p) = 0.0;
    }
    a.lp[s] = lp;
    a.eps[s] = a.init_step;
    a.mu[s] = logf(10.0f * a.init_step);
    a.hbar[s] = 0.0f;
    a.lebar[s] = 0.0f;
    a.nacc[s] = 0;
    a.da0[s] = 0;
}

__global__ void k_hmcx_set_it(int *itp, int v) {
    if (threadIdx.x == 0) *itp = v;
}
__global__ void k_hmcx_next_it(int *itp) {
    if (threadIdx.x == 0) *itp += 1;
}

// iteration it begins: momentum draw, H0, the first half kick and drift
__global__ void __launch_bounds__(256) k_hmcx_start(HmcxArgs a, int it_arg) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= a.nslot) return;
    const int it = a.itp ? *a.itp : it_arg;
    const int g = a.perm[s / a.C], ch = s % a.C;
    const uint32_t chain_id = (uint32_t)(ch * a.n_gal + g);
    uint32_t w[NP];
#pragma unroll
    for (int blk = 0; blk < 3; ++blk) {
        uint32_t c4[4] = {(uint32_t)blk, (uint32_t)it, chain_id, 0u};
        philox4x32_10(c4, a.key0, a.key1);
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (4 * blk + t < NP) w[4 * blk + t] = c4[t];
    }
    float p[NP];
#pragma unroll
    for (int t = 0; t < NP / 2; ++t) {
        const float r = sqrtf(-2.0f * logf(u01f(w[2 * t])));
        float sn, cs;
        sincosf(6.283185307179586f * u01f(w[2 * t + 1]), &sn, &cs);
        p[2 * t] = r * cs / sqrtf(XS(a.minv, 2 * t));
        p[2 * t + 1] = r * sn / sqrtf(XS(a.minv, 2 * t + 1));
    }
    double H0 = -a.lp[s];
    const float eps = a.eps[s];
#pragma unroll
    for (int t = 0; t < NP; ++t) {
        const float mi = XS(a.minv, t);
        H0 += 0.5 * (double)mi * (double)p[t] * (double)p[t];
        p[t] = fmaf(0.5f * eps, XS(a.gr, t), p[t]);
        XS(a.pm, t) = p[t];
        const float xt = fmaf(eps * mi, p[t], XS(a.x, t));
        float th, dth;
        bound_param(a.bounds + 4 * t, xt, th, dth);
        XS(a.xt, t) = xt;
        XS(a.th, t) = th;
    }
    a.h0[s] = H0;
}

// after the model call of a leapfrog step: the closing half kick; then either the next
// step's half kick and drift, or (last step) the Metropolis test, the step-size and metric
// adaptation and the sample statistics
__global__ void __launch_bounds__(256) k_hmcx_step(HmcxArgs a, int it_arg, int last) {
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= a.nslot) return;
    const int it = a.itp ? *a.itp : it_arg;
    const int g = a.perm[s / a.C], ch = s % a.C;
    float x[NP], gn[NP], p[NP];
    const double lpn = hmcx_logpost(a, s, x, gn);
    const float eps = a.eps[s];
#pragma unroll
    for (int t = 0; t < NP; ++t) p[t] = fmaf(0.5f * eps, gn[t], XS(a.pm, t));
    if (!last) {
#pragma unroll
        for (int t = 0; t < NP; ++t) {
            p[t] = fmaf(0.5f * eps, gn[t], p[t]);
            XS(a.pm, t) = p[t];
            const float xt = fmaf(eps * XS(a.minv, t), p[t], x[t]);
            float th, dth;
            bound_param(a.bounds + 4 * t, xt, th, dth);
            XS(a.xt, t) = xt;
            XS(a.th, t) = th;
        }
        return;
    }
    double H1 = -lpn;
#pragma unroll
    for (int t = 0; t < NP; ++t) H1 += 0.5 * (double)XS(a.minv, t) * (double)p[t] * (double)p[t];
    const uint32_t chain_id = (uint32_t)(ch * a.n_gal + g);
    uint32_t c4[4] = {2u, (uint32_t)it, chain_id, 0u};   // the accept draw: word 2 of block 2
    philox4x32_10(c4, a.key0, a.key1);
    float alpha;
    const bool acc = metropolis(H1, H1 - a.h0[s], c4[2], alpha);
    float xn[NP];
    if (acc) {
        a.lp[s] = lpn;
#pragma unroll
        for (int t = 0; t < NP; ++t) {
            xn[t] = x[t];
            XS(a.x, t) = x[t];
            XS(a.gr, t) = gn[t];
        }
    } else {
#pragma unroll
        for (int t = 0; t < NP; ++t) xn[t] = XS(a.x, t);
    }
    if (it < a.NW) {
        const int da0 = a.da0[s];
        const float m = (float)(it - da0 + 1), eta = 1.0f / (m + 10.0f);
        float hbar = (1.0f - eta) * a.hbar[s] + eta * (a.target - alpha);
        const float leps = a.mu[s] - sqrtf(m) / 0.05f * hbar, wk = powf(m, -0.75f);
        float lebar = wk * leps + (1.0f - wk) * a.lebar[s];
        float e = expf(it == a.NW - 1 ? lebar : leps);
        int wi = -1;
        for (int q = 0; q < a.n_win; ++q)
            if (it >= a.win_s[q] && it < a.win_e[q]) wi = q;
        if (wi >= 0) {
            const double nn = (double)(it - a.win_s[wi] + 1);
            const bool wlast = (it == a.win_e[wi] - 1);
#pragma unroll
            for (int t = 0; t < NP; ++t) {
                double wmean = XS(a.wmean, t), wm2 = XS(a.wm2, t);
                const double d = (double)xn[t] - wmean;
                wmean += d / nn;
                wm2 += d * ((double)xn[t] - wmean);
                if (wlast) {
                    XS(a.minv, t) = (float)(nn / (nn + 5.0) * (wm2 / (nn - 1.0)) + 1e-3 * 5.0 / (nn + 5.0));
                    wmean = wm2 = 0.0;
                }
                XS(a.wmean, t) = wmean;
                XS(a.wm2, t) = wm2;
            }
            if (wlast) {
                a.mu[s] = logf(10.0f * e);
                hbar = lebar = 0.0f;
                a.da0[s] = it + 1;
            }
        }
        a.hbar[s] = hbar;
        a.lebar[s] = lebar;
        a.eps[s] = e;
    } else {
        a.nacc[s] += acc ? 1 : 0;
        const double nrec = (double)(it - a.NW + 1);
#pragma unroll
        for (int t = 0; t < NP; ++t) {
            float th, dth;
            bound_param(a.bounds + 4 * t, xn[t], th, dth);
            double wmean = XS(a.wmean, t), wm2 = XS(a.wm2, t);
            const double d = (double)th - wmean;
            wmean += d / nrec;
            wm2 += d * ((double)th - wmean);
            XS(a.wmean, t) = wmean;
            XS(a.wm2, t) = wm2;
            if (a.samples) a.samples[(((size_t)(it - a.NW) * a.C + ch) * NP + t) * a.n_gal + g] = th;
        }
    }
}
#undef XS

// Slow windows of the metric adaptation over nw warm-up iterations.  Defaults: fast
// buffers of 75 (first) and 50 (last) iterations around windows of 25, 50, 100, ...;
// if 75 + 25 + 50 exceeds nw, the buffers are 15 % and 10 % of nw and the first window
// the rest.  A window that would leave less than twice its length (the next window's
// size) before the last buffer absorbs that remainder.  Returns the count, or -1 if it
// exceeds MAX_WIN.  No windows below 20 warm-up iterations.
static int metric_windows(int nw, int *ws, int *we) {
    if (nw < 20) return 0;
    int first = 75, last = 50, len = 25;
    if (first + len + last > nw) {
        first = (int)(0.15 * nw);
        last = (int)(0.1 * nw);
        len = nw - first - last;
    }
    const int stop = nw - last;
    int n = 0;
    for (int at = first; at < stop; len *= 2) {
        if (n == MAX_WIN) return -1;
        const int end = (at + 3 * len > stop) ? stop : at + len;
        ws[n] = at;
        we[n] = end;
        ++n;
        at = end;
    }
    return n;
}

size_t chain_state_bytes_public(int nslot) { return chain_state_bytes(nslot); }

size_t hmc_state_bytes(int nslot) {
    const size_t ntmp = ((size_t)nslot * HG + 63) / 64 * 64;   // trajectory scratch: every lane of the grid
    return chain_state_bytes(nslot) + align256((size_t)2 * NP * ntmp * sizeof(float));
}

// the exact-path HMC's per-slot arrays besides the chain state: floats pm, xt, th, grad [NP] +
// logl, zs + obs_s, sig_s [nb]; double h0; bytes mask_s
struct HmcxLayout {
    size_t o_f, o_d, o_m, o_it, bytes;
};
static HmcxLayout hmcx_layout(int nslot, int nb) {
    HmcxLayout L{};
    size_t off = chain_state_bytes(nslot);
    L.o_f = off;
    off += align256((size_t)nslot * (4 * NP + 2 + 2 * nb) * sizeof(float));
    L.o_d = off;
    off += align256((size_t)nslot * sizeof(double));
    L.o_m = off;
    off += align256((size_t)nslot);
    L.o_it = off;
    off += 256;
    L.bytes = off;
    return L;
}

int release_graph(sps_ctx *c) {
    if (!c->graph_exec) return SPS_OK;
    SPS_HIP(hipEventSynchronize(c->graph_done));
    (void)hipGraphExecDestroy(c->graph_exec);
    (void)hipGraphDestroy(c->graph);
    c->graph_exec = nullptr;
    c->graph = nullptr;
    return SPS_OK;
}
size_t hmcx_state_bytes(const sps_ctx *c, int nslot) { return hmcx_layout(nslot, c->n_band).bytes; }

static int launch_hmc_exact(sps_ctx *c, hipStream_t s, const sps_hmc_cfg *cfg, int n_gal, int sfh, const float *z,
                            const float *obs, const float *sigma, const uint8_t *mask, const float *bounds,
                            const float *prior, const float *theta0, float *samples, float *post_mean,
                            float *post_sd, float *rhat, float *accept, float *step, float *inv_metric,
                            int n_win, const int *win_s, const int *win_e, void *state) {
    const int C = cfg->n_chain, nslot = n_gal * C, nb = c->n_band;
    const int nit = cfg->n_warmup + cfg->n_sample;
    const int it0 = cfg->it_begin, it1 = cfg->it_end > 0 ? cfg->it_end : nit;
    HmcxArgs a{};
    a.n_win = n_win;
    for (int w = 0; w < n_win; ++w) {
        a.win_s[w] = win_s[w];
        a.win_e[w] = win_e[w];
    }
    const HmcxLayout L = hmcx_layout(nslot, nb);
    if (c->hwork_bytes < L.bytes || nslot > c->max_exact)
        return set_error(SPS_E_STATE, "the exact-path HMC needs " + std::to_string(nslot) +
                                          " reserved exact rows (call sps_reserve_exact)");
    char *W = (char *)c->d_hwork;
    const ChainState cs = chain_state_at(W, nslot);
    a.x = cs.x;
    a.gr = cs.gr;
    a.minv = cs.minv;
    a.eps = cs.eps;
    a.mu = cs.mu;
    a.hbar = cs.hbar;
    a.lebar = cs.lebar;
    a.nacc = cs.nacc;
    a.da0 = cs.da0;
    a.lp = cs.lp;
    a.wmean = cs.wmean;
    a.wm2 = cs.wm2;
    float *fp = (float *)(W + L.o_f);
    auto fq = [&](int count) { float *r = fp; fp += (size_t)count * nslot; return r; };
    a.pm = fq(NP);
    a.xt = fq(NP);
    a.th = fq(NP);
    a.grad = fq(NP);
    a.logl = fq(1);
    a.zs = fq(1);
    a.obs_s = fq(nb);
    a.sig_s = fq(nb);
    a.h0 = (double *)(W + L.o_d);
    a.mask_s = (uint8_t *)(W + L.o_m);
    a.n_gal = n_gal;
    a.C = C;
    a.nslot = nslot;
    a.nb = nb;
    a.NW = cfg->n_warmup;
    a.NS = cfg->n_sample;
    a.target = cfg->target_accept;
    a.init_step = cfg->init_step;
    a.key0 = (uint32_t)(cfg->seed & 0xffffffffull);
    a.key1 = (uint32_t)(cfg->seed >> 32);
    a.z = z;
    a.obs = obs;
    a.sigma = sigma;
    a.mask = mask;
    a.bounds = bounds;
    a.prior = prior;
    a.theta0 = theta0;
    a.samples = samples;
    {   // rank the galaxies by z
        const DevConsts grid = z_sort_grid(c);
        int rc0 = launch_bucket_sort(c, s, n_gal, z, nullptr, &grid);
        if (rc0) return rc0;
        a.perm = c->d_perm;
    }
    const dim3 grid((nslot + 255) / 256), block(256);
    // one exact value+gradient over every chain at the positions in a.th (the start)
    auto model = [&]() {
        return launch_exact(c, s, nslot, sfh, cfg->prec, a.th, a.zs, nullptr, a.obs_s, a.sig_s, a.mask_s, a.logl,
                            a.grad, true);
    };
    int rc;
    hipLaunchKernelGGL(k_hmcx_setup, grid, block, 0, s, a, (int)(it0 == 0));
    if (it0 == 0) {
        if ((rc = model())) return rc;
        hipLaunchKernelGGL(k_hmcx_init, grid, block, 0, s, a);
    } else if ((rc = move_state(c, s, cs, state, cfg, n_gal, a.perm, 0, it0))) {
        return rc;
    }
    // one iteration: the momentum draw and first half step, then per leapfrog step the exact
    // value+gradient over every chain and the per-chain closing kick / drift / end of iteration
    auto iteration = [&](hipStream_t st, int it) -> int {
        hipLaunchKernelGGL(k_hmcx_start, grid, block, 0, st, a, it);
        for (int l = 0; l < cfg->n_leapfrog; ++l) {
            const int r = launch_exact(c, st, nslot, sfh, cfg->prec, a.th, a.zs, nullptr, a.obs_s, a.sig_s,
                                       a.mask_s, a.logl, a.grad, true);
            if (r) return r;
            hipLaunchKernelGGL(k_hmcx_step, grid, block, 0, st, a, it, (int)(l == cfg->n_leapfrog - 1));
        }
        if (a.itp) hipLaunchKernelGGL(k_hmcx_next_it, dim3(1), dim3(64), 0, st, a.itp);
        return SPS_OK;
    };
    if (c->launch.hmcx_graph && it1 - it0 >= 2) {
        // capture one iteration on the context's capture stream (the iteration index lives in
        // device memory and the captured iteration advances it), then replay it on s
        if ((rc = release_graph(c))) return rc;
        a.itp = (int *)(W + L.o_it);
        hipLaunchKernelGGL(k_hmcx_set_it, dim3(1), dim3(64), 0, s, a.itp, it0);
        SPS_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        rc = iteration(c->cap_stream, it0);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
        if (rc || ec != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return rc ? rc : hip_check(ec, "hipStreamEndCapture");
        }
        hipGraphExec_t ge = nullptr;
        const hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (ei != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_check(ei, "hipGraphInstantiate");
        }
        c->graph = g;
        c->graph_exec = ge;
        for (int it = it0; it < it1; ++it) SPS_HIP(hipGraphLaunch(ge, s));
        SPS_HIP(hipEventRecord(c->graph_done, s));
        a.itp = nullptr;
    } else {
        for (int it = it0; it < it1; ++it)
            if ((rc = iteration(s, it))) return rc;
    }
    if (state && (rc = move_state(c, s, cs, state, cfg, n_gal, a.perm, 1, it1))) return rc;
    if (it1 == nit)
        hipLaunchKernelGGL(k_hmc_summary, dim3((n_gal + 255) / 256), dim3(256), 0, s, n_gal, C, cfg->n_sample,
                           a.perm, a.wmean, a.wm2, a.nacc, nullptr, a.eps, a.minv, post_mean, post_sd, rhat, accept, step,
                           inv_metric);
    SPS_HIP(hipGetLastError());
    return SPS_OK;
}

int launch_hmc(sps_ctx *c, hipStream_t s, const sps_hmc_cfg *cfg, int n_gal, int sfh, const float *z,
               const float *obs, const float *sigma, const uint8_t *mask, const float *bounds, const float *prior,
               const float *theta0, float *samples, float *post_mean, float *post_sd, float *rhat, float *accept,
               float *step, float *inv_metric, void *state) {
    const int C = cfg->n_chain, nslot = n_gal * C;
    HmcArgs a{};
    a.n_win = 0;
    if (cfg->adapt_metric) {
        a.n_win = metric_windows(cfg->n_warmup, a.win_s, a.win_e);
        if (a.n_win < 0) return set_error(SPS_E_INVAL, "n_warmup too long for the metric-window table");
    }
    if (cfg->path == SPS_PATH_EXACT)
        return launch_hmc_exact(c, s, cfg, n_gal, sfh, z, obs, sigma, mask, bounds, prior, theta0, samples,
                                post_mean, post_sd, rhat, accept, step, inv_metric, a.n_win, a.win_s, a.win_e, state);
    const int nit = cfg->n_warmup + cfg->n_sample;
    const int it0 = cfg->it_begin, it1 = cfg->it_end > 0 ? cfg->it_end : nit;
    if (c->hstate_bytes < hmc_state_bytes(nslot))
        return set_error(SPS_E_STATE, "the HMC chain state needs n_gal * n_chain reserved galaxies (call sps_reserve)");
    int rc = launch_bucket_sort(c, s, n_gal, z);
    if (rc) return rc;
    const ChainState cs = chain_state_at(c->d_hstate, nslot);
    a.n_gal = n_gal;
    a.C = C;
    a.L = cfg->n_leapfrog;
    a.NW = cfg->n_warmup;
    a.NS = cfg->n_sample;
    a.sfh = sfh;
    a.target = cfg->target_accept;
    a.init_step = cfg->init_step;
    a.key0 = (uint32_t)(cfg->seed & 0xffffffffull);
    a.key1 = (uint32_t)(cfg->seed >> 32);
    a.z = z;
    a.obs = obs;
    a.sigma = sigma;
    a.mask = mask;
    a.bounds = bounds;
    a.prior = prior;
    a.theta0 = theta0;
    a.perm = c->d_perm;
    a.qf = c->d_qf;
    a.qa = c->d_qa;
    a.samples = samples;
    a.x = cs.x;
    a.gr = cs.gr;
    a.minv = cs.minv;
    a.eps = cs.eps;
    a.mu = cs.mu;
    a.hbar = cs.hbar;
    a.lebar = cs.lebar;
    a.nacc = cs.nacc;
    a.da0 = cs.da0;
    a.lp = cs.lp;
    a.wmean = cs.wmean;
    a.wm2 = cs.wm2;
    const int ntmp = (nslot * HG + 63) / 64 * 64;   // every lane of the grid
    a.pm = (float *)((char *)c->d_hstate + chain_state_bytes(nslot));
    a.xt = a.pm + (size_t)NP * ntmp;
    a.ntmp = ntmp;
    const int blk_it = c->launch.hmc_block_iters;
    dim3 grid((nslot * HG + 63) / 64), block(64);
    const bool dpl = (sfh == SPS_SFH_DPL);
    const size_t lds_bytes = approx_lds_bytes(c->n_band, false, HG);
    if (it0 == 0) {
        if (dpl) hipLaunchKernelGGL(k_hmc_init<SPS_SFH_DPL>, grid, block, lds_bytes, s, c->k, a);
        else hipLaunchKernelGGL(k_hmc_init<SPS_SFH_LOGNORMAL>, grid, block, lds_bytes, s, c->k, a);
    } else if ((rc = move_state(c, s, cs, state, cfg, n_gal, c->d_perm, 0, it0))) {
        return rc;
    }
    for (int b0 = it0; b0 < it1; b0 += blk_it) {
        a.it0 = b0;
        a.it1 = b0 + blk_it < it1 ? b0 + blk_it : it1;
        if (dpl) hipLaunchKernelGGL(k_hmc<SPS_SFH_DPL>, grid, block, lds_bytes, s, c->k, a);
        else hipLaunchKernelGGL(k_hmc<SPS_SFH_LOGNORMAL>, grid, block, lds_bytes, s, c->k, a);
    }
    if (state && (rc = move_state(c, s, cs, state, cfg, n_gal, c->d_perm, 1, it1))) return rc;
    if (it1 == nit)
        hipLaunchKernelGGL(k_hmc_summary, dim3((n_gal + 255) / 256), dim3(256), 0, s, n_gal, C, cfg->n_sample,
                           c->d_perm, a.wmean, a.wm2, a.nacc, nullptr, a.eps, a.minv, post_mean, post_sd, rhat, accept, step,
                           inv_metric);
    SPS_HIP(hipGetLastError());
    return SPS_OK;
}

}  // namespace sps
