// Per-lane evaluation of the approximate-path model and its adjoint, shared by
// the one-shot kernels and the HMC kernel.
#pragma once
#include "sps_model.h"

namespace sps {

typedef const float __attribute__((address_space(4))) cfloat;

constexpr int WAVE = 64;
constexpr int LDS_SLOTS = (NA > NB_MAX * NZ + NB_MAX) ? NA : NB_MAX * NZ + NB_MAX;

// ------------------------------------------------------------------ bucket sort
// bucket of a galaxy: interval k of the z table, or n_z - 1 for z outside the table
__device__ inline int z_bucket(const DevConsts &k, float z, float *frac) {
    const double u = ((double)z - (double)k.z_lo) / (double)k.dz;
    const double top = (double)(k.n_z - 1);
    if (!(u >= 0.0 && u <= top)) {
        *frac = 0.0f;
        return -1;
    }
    int kk = (int)floor(u);
    kk = min(kk, k.n_z - 2);
    *frac = (float)(u - (double)kk);
    return kk;
}

// ------------------------------------------------------------------ per-lane LDS column
struct LdsCol {
    float *base;  // &lds[lane]; slot s at base[s * WAVE]
    __device__ float &operator[](int s) const { return base[s * WAVE]; }
};

// ------------------------------------------------------------------ forward weights
// Leaves P_age in registers (pa), P_Z in registers (pz); returns the burst
// normaliser and the total smooth mass (needed by the adjoint).
struct WeightsState {
    double S;      // total smooth mass (FP64 running sum)
    float Zb;      // burst normaliser (1 unless clipped at t_obs)
    float l_obs;   // log10 t_obs [yr]
    int i0;        // first age bin of the burst window
};

__device__ inline void forward_weights(const DevConsts &k, int sfh, const float *th, double t_obs,
                                       LdsCol col, float (&pa)[NA], float (&pz)[NZ], WeightsState &ws) {
    const float t_obs_f = (float)t_obs;
    double S = 0.0;
    if (sfh == SPS_SFH_DPL) {
        const Dpl p = make_dpl(th[1], th[2], th[3]);
        for (int i = 0; i < NA; ++i) {
            float m, a, b, c;
            dpl_bin<false>(k, i, t_obs_f, p, m, a, b, c);
            col[i] = m;
            S += (double)m;
        }
    } else {
        for (int i = 0; i < NA; ++i) {
            double m, a, b;
            logn_bin<false>(k, i, t_obs, (double)th[1], (double)th[2], m, a, b);
            col[i] = (float)m;
            S += m;
        }
    }
    // burst: only the bins the triweight window [mu - 3 sigma, mu + 3 sigma] touches
    const float l_obs = (float)log10(t_obs * 1e9), mu = th[5], inv_s3 = 1.0f / (3.0f * k.burst_sig);
    const int i0 = first_bin_above(k, mu - 3.0f * k.burst_sig);
    float Zb = 0.0f;
    for (int t = 0; t < k.burst_nbins; ++t) {
        float p, dp;
        if (i0 + t < NA) burst_bin(k, i0 + t, l_obs, mu, inv_s3, p, dp);
        else p = 0.0f;
        Zb += p;
    }
    const float fb = th[4], sm = (1.0f - fb) * (float)(1.0 / S), bz = (Zb > 0.0f) ? fb / Zb : 0.0f;
    for (int i = 0; i < NA; ++i) col[i] = col[i] * sm;
    for (int t = 0; t < k.burst_nbins; ++t) {
        if (i0 + t >= NA) break;
        float p, dp;
        burst_bin(k, i0 + t, l_obs, mu, inv_s3, p, dp);
        col[i0 + t] = fmaf(bz, p, col[i0 + t]);
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) pa[i] = col[i];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        float dp;
        met_bin(k, j, th[6], pz[j], dp);
    }
    ws.S = S;
    ws.Zb = Zb;
    ws.l_obs = l_obs;
    ws.i0 = i0;
}

// gradient of the weights: given dP_age (LDS column, slots 0..NA) and dP_Z,
// accumulate d/d(theta_1..6)
__device__ inline void adjoint_weights(const DevConsts &k, int sfh, const float *th, double t_obs,
                                       const WeightsState &ws, LdsCol col, const float (&pzbar)[NZ],
                                       float *g) {
    const float t_obs_f = (float)t_obs, fb = th[4];
    const float invS = (float)(1.0 / ws.S), invZ = (ws.Zb > 0.0f) ? 1.0f / ws.Zb : 0.0f;
    float fbar = 0.0f, cbar = 0.0f, e1 = 0.0f, e2 = 0.0f, e3 = 0.0f;
    float A0 = 0.f, A1 = 0.f, A2 = 0.f, B0 = 0.f, B1 = 0.f, B2 = 0.f;
    double dA0 = 0.0, dA1 = 0.0, dB0 = 0.0, dB1 = 0.0;
    Dpl p;
    if (sfh == SPS_SFH_DPL) p = make_dpl(th[1], th[2], th[3]);
    // smooth part: dP_age/dF_burst = P_burst - P_smooth; the P_burst term is added below
    for (int i = 0; i < NA; ++i) {
        const float gbar = col[i];
        float ps;
        float m, mt, ma, mb;
        double dm, dmt, dmw;
        if (sfh == SPS_SFH_DPL) {
            dpl_bin<true>(k, i, t_obs_f, p, m, mt, ma, mb);
            ps = m * invS;
        } else {
            logn_bin<true>(k, i, t_obs, (double)th[1], (double)th[2], dm, dmt, dmw);
            ps = (float)(dm / ws.S);
        }
        fbar = fmaf(-gbar, ps, fbar);
        const float psbar = (1.0f - fb) * gbar;
        cbar = fmaf(psbar, ps, cbar);
        if (sfh == SPS_SFH_DPL) {
            A0 = fmaf(psbar, mt, A0); A1 = fmaf(psbar, ma, A1); A2 = fmaf(psbar, mb, A2);
            B0 += mt; B1 += ma; B2 += mb;
        } else {
            dA0 += (double)psbar * dmt; dA1 += (double)psbar * dmw;
            dB0 += dmt; dB1 += dmw;
        }
    }
    // burst part over the triweight window
    const float inv_s3 = 1.0f / (3.0f * k.burst_sig);
    for (int t = 0; t < k.burst_nbins; ++t) {
        const int i = ws.i0 + t;
        if (i >= NA) break;
        const float gbar = col[i];
        float pbr, dpb;
        burst_bin(k, i, ws.l_obs, th[5], inv_s3, pbr, dpb);
        const float pb = pbr * invZ, pbbar = fb * gbar;
        fbar = fmaf(gbar, pb, fbar);
        e1 = fmaf(pbbar, dpb, e1);
        e2 = fmaf(pbbar, pb, e2);
        e3 += dpb;
    }
    if (sfh == SPS_SFH_DPL) {
        g[1] += (A0 - cbar * B0) * invS;
        g[2] += (A1 - cbar * B1) * invS;
        g[3] += (A2 - cbar * B2) * invS;
    } else {
        g[1] += (float)((dA0 - (double)cbar * dB0) / ws.S);
        g[2] += (float)((dA1 - (double)cbar * dB1) / ws.S);
    }
    g[4] += fbar;
    g[5] += (e1 - e2 * e3) * invZ;
    float mbar = 0.0f;
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        float pzj, dpz;
        met_bin(k, j, th[6], pzj, dpz);
        mbar = fmaf(pzbar[j], dpz, mbar);
    }
    g[6] += mbar;
}


// ------------------------------------------------------------------ one evaluation
// Magnitudes (MODE_MAGS) or log-likelihood with its gradient w.r.t. the physical
// parameters (MODE_LOGL_GRAD) for the lane's galaxy.  Every lane of the wave
// must call it (the z-bucket loop is wave-uniform); lanes with kk < 0 take part
// without contributing.  kmin/kmax: wave-uniform range of the lanes' buckets.
template <int MODE>
__device__ inline void approx_eval(const DevConsts &k, int sfh, cfloat *qc, LdsCol col, const float (&th)[NP],
                                   float zf, int kk, float f, double t_obs, double m0, int kmin, int kmax,
                                   const float *obs_g, const float *sig_g, uint32_t mask, float *mag_out,
                                   double &logl, float (&gr)[NP]) {
    const int nb = k.n_band;
    float pa[NA], pz[NZ];
    WeightsState ws;
    forward_weights(k, sfh, th, t_obs, col, pa, pz, ws);

    // ---- contraction: T[b][j] = sum_i P_age(i) Qz[b][j][i]
    const int rows = nb * NZ;
    for (int kb = kmin; kb <= kmax; ++kb) {
        const bool act = (kk == kb);
        if (__builtin_amdgcn_readfirstlane(__ballot(act) != 0ull) == 0) continue;
        cfloat *q0 = qc + (size_t)kb * rows * NA;
        cfloat *q1 = q0 + (size_t)rows * NA;
        for (int r = 0; r < rows; ++r) {
            cfloat *r0 = q0 + r * NA;
            cfloat *r1 = q1 + r * NA;
            float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
#pragma unroll
            for (int i = 0; i + 3 < NA; i += 4) {
                a0 = fmaf(pa[i], r0[i], a0); c0 = fmaf(pa[i], r1[i], c0);
                a1 = fmaf(pa[i + 1], r0[i + 1], a1); c1 = fmaf(pa[i + 1], r1[i + 1], c1);
                a2 = fmaf(pa[i + 2], r0[i + 2], a2); c2 = fmaf(pa[i + 2], r1[i + 2], c2);
                a3 = fmaf(pa[i + 3], r0[i + 3], a3); c3 = fmaf(pa[i + 3], r1[i + 3], c3);
            }
#pragma unroll
            for (int i = NA & ~3; i < NA; ++i) {
                a0 = fmaf(pa[i], r0[i], a0);
                c0 = fmaf(pa[i], r1[i], c0);
            }
            const float t = (1.0f - f) * ((a0 + a1) + (a2 + a3)) + f * ((c0 + c1) + (c2 + c3));
            if (act) col[r] = t;
        }
    }

    // ---- magnitudes, likelihood.  The band sums, magnitudes and residuals are formed in
    // FP64 from the FP32 row sums: an FP32 magnitude near 25 carries ~2e-6 of rounding,
    // which the likelihood gradient amplifies by 1/sigma^2.
    const float tauv = th[7], delta = th[8], ffl = th[9];
    const float opz = 1.0f + zf;
    double logl_d = 0.0;
#pragma unroll
    for (int p = 0; p < NP; ++p) gr[p] = 0.0f;
    float sbar[NB_MAX];
#pragma unroll
    for (int b = 0; b < NB_MAX; ++b) {
        sbar[b] = 0.0f;
        if (b >= nb) continue;
        double sb = 0.0;
#pragma unroll
        for (int j = 0; j < NZ; ++j) sb += (double)pz[j] * (double)col[b * NZ + j];
        const DustVal d = dust_at(k.lam_eff[b] / (opz * 5500.0f), tauv, delta, ffl);
        const double mag = m0 - 2.5 * log10((double)d.F * sb);
        if (MODE == MODE_MAGS) {
            mag_out[b] = (float)mag;
            continue;
        }
        if ((mask >> b) & 1u) {
            const double s = sig_g[b];
            const double r = (mag - (double)obs_g[b]) / s;
            logl_d += -0.5 * r * r - log(s * 2.5066282746310002);
            if (MODE != MODE_LOGL) {
                const float gm = (float)(-r / s);            // d logL / d m_b
                const float c = gm * (-2.5f / LN10F);        // d logL / d ln(F S)
                sbar[b] = (float)(c / sb);
                const float fbar = c / d.F;
                gr[0] += -2.5f * gm;
                gr[7] = fmaf(fbar, d.dF_tauv, gr[7]);
                gr[8] = fmaf(fbar, d.dF_delta, gr[8]);
                gr[9] = fmaf(fbar, d.dF_floor, gr[9]);
            }
        }
    }
    logl = logl_d;
    if (MODE != MODE_LOGL_GRAD) return;

    // dP_Z and the row coefficients of the adjoint contraction
    float pzbar[NZ];
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        float s = 0.0f;
#pragma unroll
        for (int b = 0; b < NB_MAX; ++b)
            if (b < nb) s = fmaf(sbar[b], col[b * NZ + j], s);
        pzbar[j] = s;
    }
#pragma unroll
    for (int b = 0; b < NB_MAX; ++b)
        if (b < nb) {
#pragma unroll
            for (int j = 0; j < NZ; ++j) col[b * NZ + j] = sbar[b] * pz[j];
        }
    // dP_age(i) = sum_{b,j} sbar_b P_Z(j) Qz[b][j][i]
    float pbar[NA];
#pragma unroll
    for (int i = 0; i < NA; ++i) pbar[i] = 0.0f;
    for (int kb = kmin; kb <= kmax; ++kb) {
        const bool act = (kk == kb);
        if (__builtin_amdgcn_readfirstlane(__ballot(act) != 0ull) == 0) continue;
        cfloat *q0 = qc + (size_t)kb * rows * NA;
        cfloat *q1 = q0 + (size_t)rows * NA;
        for (int r = 0; r < rows; ++r) {
            cfloat *r0 = q0 + r * NA;
            cfloat *r1 = q1 + r * NA;
            const float c = act ? col[r] : 0.0f;
            const float c0 = (1.0f - f) * c, c1 = f * c;
#pragma unroll
            for (int i = 0; i < NA; ++i) pbar[i] = fmaf(c0, r0[i], fmaf(c1, r1[i], pbar[i]));
        }
    }
#pragma unroll
    for (int i = 0; i < NA; ++i) col[i] = pbar[i];
    adjoint_weights(k, sfh, th, t_obs, ws, col, pzbar, gr);
}

// bounding function (App. C): theta = lo + (hi - lo) sigmoid(k (x - x0)) and d theta / d x
__device__ inline void bound_param(const float *bnd, float x, float &th, float &dth) {
    const float lo = bnd[0], hi = bnd[1], kk = bnd[2], x0 = bnd[3];
    const float s = 1.0f / (1.0f + expf(-kk * (x - x0)));
    th = lo + (hi - lo) * s;
    dth = kk * (hi - lo) * s * (1.0f - s);
}

// skew-normal log prior on the unbounded value (App. C) and its derivative
__device__ inline double log_prior_skewnorm(const float *pri, float x, float &dlp) {
    const double xi = pri[0], om = pri[1], sk = pri[2];
    const double y = ((double)x - xi) / om, v = sk * y;
    double lphi, ratio;
    if (v < -5.0) {  // scaled complementary error function keeps log Phi finite in the far tail
        const double e = erfcx(-v * 0.7071067811865475);
        lphi = log(0.5 * e) - 0.5 * v * v;
        ratio = 0.7978845608028654 / e;
    } else {
        const double P = Phi_d(v);
        lphi = log(P);
        ratio = phi_d(v) / P;
    }
    dlp = (float)((-y + sk * ratio) / om);
    return log(2.0 / om) - 0.9189385332046727 - 0.5 * y * y + lphi;
}

}  // namespace sps
