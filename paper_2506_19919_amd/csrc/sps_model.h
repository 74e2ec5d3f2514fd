// Device-side forward model, one galaxy (or chain) per lane.
//
// SFH bin masses (App. A.1, Eqs. totalMstarFormed, SFRsmooth, smoothPsfh):
//   double power law: bin integrals by Gauss-Legendre-4 panels in X = ln(t/tau)
//   (one 2-point panel for bins narrower than 1/4 of the panel width, the midpoint for bins
//   whose older edge lies within 2^-7 of t_obs),
//   where the integrand tau / (e^{(alpha-1)X} + e^{-(beta+1)X}) is analytic with
//   poles at distance pi/(alpha+beta) from the real axis.  Panel width
//   min(0.56, 2.8/(alpha+beta), 1.68/(beta+1)); in the oldest bin the panels reach down
//   to 4/(alpha+beta) below min(X_hi, 0) and the rest of the tail is integrated term by
//   term from a four-term series in e^{(alpha+beta)X} (TAIL_CUT, TAIL_TERMS).  Node
//   values in FP32, the running total mass in FP64.  Against the exact integrals this
//   keeps the total mass within ~4e-6 and the tau, alpha, beta derivatives within ~8e-5
//   over tau 0.1-14 Gyr, alpha, beta 0.1-8, z 0.1-3.
//   log-normal SFH: Gauss-Legendre quadrature of the normal density over each bin in FP32
//   (closed-form normal-CDF differences in FP64 on the FP64 exact path).
// Burst (Eq. triweight): closed-form triweight CDF differences in log age.
// Metallicity (App. A.2): normal-CDF differences on the midpoint bins.
// Dust (App. A.3, Eq. DustAtt with k0 = 4.05, D = 0, plus the unobscured floor).
#pragma once
#include "sps_internal.h"

namespace sps {

// 4-point Gauss-Legendre rule: nodes +-sqrt(3/7 -+ (2/7) sqrt(6/5)), weights (18 +- sqrt(30))/36
__device__ constexpr float GL4X[4] = {-0.86113631159405258f, -0.33998104358485626f,
                                      0.33998104358485626f, 0.86113631159405258f};
__device__ constexpr float GL4W[4] = {0.34785484513745386f, 0.65214515486254614f,
                                      0.65214515486254614f, 0.34785484513745386f};

constexpr float LN10F = 2.302585092994046f;
constexpr double PI_D = 3.14159265358979323846;

// ------------------------------------------------------------------ cosmology (FP64)
__device__ inline double age_universe_gyr(const DevConsts &k, double z) {
    double ol = 1.0 - k.om, a15 = pow(1.0 + z, -1.5);
    if (ol > 0.0) return 2.0 / (3.0 * k.h0_gyr * sqrt(ol)) * asinh(sqrt(ol / k.om) * a15);
    return 2.0 / (3.0 * k.h0_gyr) * a15;
}

__device__ inline double lum_distance_cm(const DevConsts &k, double z) {
    double ol = 1.0 - k.om, h = 0.5 * z, s = 0.0;
#pragma unroll
    for (int i = 0; i < NGL_DL; ++i) {
        double zp = h + h * k.gl_x[i], zm = h - h * k.gl_x[i];
        double ep = 1.0 + zp, em = 1.0 + zm;
        s += k.gl_w[i] * (1.0 / sqrt(k.om * ep * ep * ep + ol) + 1.0 / sqrt(k.om * em * em * em + ol));
    }
    return (1.0 + z) * k.dh_cm * h * s;
}

// -2.5 log10 K(z):  K = (1+z) Lsun / (4 pi D_L^2 c 3631 Jy)
__device__ inline double mag_offset(const DevConsts &k, double z) {
    double dl = lum_distance_cm(k, z);
    return -2.5 * log10((1.0 + z) * k.kfac) + 5.0 * log10(dl);
}

// d t_obs / dz = -1 / ((1 + z) H(z)) and d mag_offset / dz = (2.5 / ln 10) / (1 + z) +
// (5 / ln 10) / (E(z) chi(z)), chi the comoving distance in Hubble lengths
__device__ inline void cosmo_derivs(const DevConsts &k, double z, double dl_cm, double &dt, double &dm) {
    const double ep = 1.0 + z, e = sqrt(k.om * ep * ep * ep + (1.0 - k.om));
    dt = -1.0 / (ep * k.h0_gyr * e);
    const double chi = dl_cm / (ep * k.dh_cm);
    dm = 1.0857362047581294 / ep + 2.1714724095162588 / (e * chi);
}

// t_obs and mag_offset at z: cubic Hermite interpolation in the cosmology table inside the
// z table's range (|error| < 1e-10 Gyr and 1e-7 mag), the direct evaluation outside it
__device__ inline void cosmo_at(const DevConsts &k, double z, double &t_obs, double &m0) {
    const double u = (z - k.ct_lo) * k.ct_inv_dz;
    if (k.ctab && u >= 0.0 && u <= (double)(CT_N - 1)) {
        const int i = min((int)u, CT_N - 2);
        const double s = u - (double)i, s2 = s * s, r = 1.0 - s;
        const double h00 = (1.0 + 2.0 * s) * r * r, h10 = s * r * r * k.ct_dz;
        const double h01 = s2 * (3.0 - 2.0 * s), h11 = -s2 * r * k.ct_dz;
        const double *a = k.ctab + 4 * i, *b = a + 4;
        t_obs = h00 * a[0] + h10 * a[1] + h01 * b[0] + h11 * b[1];
        m0 = h00 * a[2] + h10 * a[3] + h01 * b[2] + h11 * b[3];
    } else {
        t_obs = age_universe_gyr(k, z);
        m0 = mag_offset(k, z);
    }
}

// ------------------------------------------------------------------ helpers
__device__ inline float phi_f(float x) { return 0.3989422804014327f * expf(-0.5f * x * x); }
__device__ inline float Phi_f(float x) { return 0.5f * erfcf(-0.7071067811865475f * x); }
__device__ inline double Phi_d(double x) { return 0.5 * erfc(-0.7071067811865475 * x); }
__device__ inline double Phic_d(double x) { return 0.5 * erfc(0.7071067811865475 * x); }
__device__ inline double phi_d(double x) { return 0.3989422804014327 * exp(-0.5 * x * x); }

// triweight CDF in u = x/3 (closed-form antiderivative of (35/32)(1-u^2)^3) and its slope
__device__ inline float tri_cdf(float u) {
    u = fminf(fmaxf(u, -1.0f), 1.0f);
    float u2 = u * u;
    return 0.5f + 1.09375f * u * (1.0f - u2 + u2 * u2 * (0.6f - u2 * (1.0f / 7.0f)));
}
__device__ inline float tri_dcdf(float u) {
    float v = 1.0f - u * u;
    return (v > 0.0f) ? 1.09375f * v * v * v : 0.0f;
}

// ------------------------------------------------------------------ double power law
struct Dpl {
    float tau, bp1, ltau, inv_w;
    float s_l2, b_l2;   // (alpha + beta) log2(e), (beta + 1) log2(e)
    float alpha, ab;         // alpha, alpha + beta
    float x_obs, inv_tobs;   // ln(t_obs / tau), 1 / t_obs: set by dpl_at_obs
};

// the observation-time constants of a galaxy's DPL evaluation
__device__ inline void dpl_at_obs(Dpl &d, float t_obs) {
    d.x_obs = __builtin_amdgcn_logf(t_obs) * 0.69314718055994531f - d.ltau;
    d.inv_tobs = __builtin_amdgcn_rcpf(t_obs);
}

// ln(1 + x) for |x| <= 2^-7 by its series to x^4 (relative error below 3e-10)
__device__ inline float log1p_small(float x) {
    return x * fmaf(x, fmaf(x, fmaf(x, -0.25f, 0.33333333f), -0.5f), 1.0f);
}
__device__ inline Dpl make_dpl(float tau, float al, float be) {
    Dpl d;
    d.tau = tau;
    d.bp1 = be + 1.0f;
    d.ltau = logf(tau);
    float w = fminf(0.56f, fminf(2.8f / (al + be), 1.68f / d.bp1));
    d.inv_w = 1.0f / w;
    d.s_l2 = (al + be) * 1.4426950408889634f;
    d.b_l2 = d.bp1 * 1.4426950408889634f;
    d.alpha = al;
    d.ab = al + be;
    return d;
}

// 2-point Gauss-Legendre node 1/sqrt(3) (weights 1): bins narrower than 1/4 of the panel
// width, where the 4-point panel rule would be wasted.  Panel width and this cut keep the
// bin masses within ~4e-6 of the exact integral in total and their tau/alpha/beta
// derivatives within ~8e-5, over tau 0.1-14 Gyr, alpha, beta 0.1-8, z 0.1-3
constexpr float GL2X = 0.57735026918962576f;

// oldest age bin: quadrature panels cover X down to TAIL_CUT / (alpha + beta) below
// min(X_obs, 0); the series below that cut takes TAIL_TERMS terms
constexpr float TAIL_CUT = 4.0f;
constexpr int TAIL_TERMS = 4;

// integrand h = tau g(X), g = 1 / (e^{(alpha-1)X} + e^{-(beta+1)X}), at X with weight wg.
// Written without overflow as g = fB e^{(beta+1)X}, fB = 1 / (1 + e^{(alpha+beta)X}), and
// with fA = 1 - fB:
//   dh/dtau = g (alpha - (alpha+beta) fB)   (X = ln(t/tau) moves with tau),
//   dh/dalpha = -tau g X (1 - fB),  dh/dbeta = tau g X fB,
// so four sums carry the derivatives: s = sum w g, sf = sum w g fB, sa = sum w g X fA and
// sb = sum w g X fB (tau is applied once per bin; fA is formed as e fB, not 1 - fB, which
// would lose its relative precision where it is small).
template <bool DERIV>
__device__ inline void dpl_node(const Dpl &p, float X, float wg, float &s, float &sf, float &sa, float &sb) {
    const float ed = __builtin_amdgcn_exp2f(p.s_l2 * X);
    const float eb = __builtin_amdgcn_exp2f(p.b_l2 * X);
    const float fB = __builtin_amdgcn_rcpf(1.0f + ed);
    const float t = wg * fB * eb;
    s += t;
    if (DERIV) {
        const float tx = t * X, fA = (ed < 3.0e38f) ? ed * fB : 1.0f;
        sf = fmaf(t, fB, sf);
        sa = fmaf(tx, fA, sa);
        sb = fmaf(tx, fB, sb);
    }
}

// Mass formed in the age bin [a_lo, a_hi) (rate amplitude 1) and, if DERIV, its derivatives
// w.r.t. (tau, alpha, beta).
// The age edges of the bins i = q, q + G, ... in turn, each bin's edges read one bin ahead of their
// use (the bins are contiguous: the upper edge of bin i is the lower edge of bin i + 1, so with
// G = 1 each step reads one edge)
template <int G>
struct AgeEdges {
    const DevConsts &k;
    float lo, hi;
    __device__ AgeEdges(const DevConsts &k_, int q) : k(k_), lo(k_.age_lo[q]), hi(k_.age_hi[q]) {}
    // the edges of bin i, then those of bin i + G prefetched
    __device__ void step(int i, float &a_lo, float &a_hi) {
        a_lo = lo;
        a_hi = hi;
        const int in = min(i + G, NA - 1);
        lo = (G == 1) ? hi : k.age_lo[in];
        hi = k.age_hi[in];
    }
};

template <bool DERIV>
__device__ inline void dpl_bin(float a_lo, float a_hi, float t_obs, const Dpl &p, float &m, float &d_tau,
                               float &d_al, float &d_be) {
    m = d_tau = d_al = d_be = 0.0f;
    if (!(a_lo < t_obs)) return;
    // span W of the bin in X is formed directly as log1p of the age-edge ratio (young bins
    // are ~1e-5 wide at |X| ~ 1, where xhi - xlo would cancel in FP32)
    float xhi, span, tail = 0.0f, tail_t = 0.0f, tail_a = 0.0f, tail_b = 0.0f;
    if (a_hi <= 0.0078125f * t_obs) {
        // young bin (older edge within 2^-7 of t_obs): X_hi = X_obs + ln(1 - a_lo / t_obs) and
        // W = ln(1 + d) by series, no transcendental beyond one reciprocal
        xhi = p.x_obs + log1p_small(-a_lo * p.inv_tobs);
        span = log1p_small((a_hi - a_lo) * __builtin_amdgcn_rcpf(t_obs - a_hi));
    } else if (a_hi < t_obs) {
        // hardware log2 / reciprocal: ~1 ulp, shifting every node of the bin alike by < 3e-7;
        // log1p(d) as log(u) d / (u - 1) with u = 1 + d, which absorbs the rounding of u
        xhi = __builtin_amdgcn_logf(t_obs - a_lo) * 0.69314718055994531f - p.ltau;
        const float d = (a_hi - a_lo) * __builtin_amdgcn_rcpf(t_obs - a_hi);
        const float u = 1.0f + d;
        span = (u == 1.0f) ? d : __builtin_amdgcn_logf(u) * 0.69314718055994531f * (d * __builtin_amdgcn_rcpf(u - 1.0f));
    } else {
        xhi = __builtin_amdgcn_logf(t_obs - a_lo) * 0.69314718055994531f - p.ltau;
        // oldest bin: panels down to the cut xc, where u = e^{(alpha+beta) X} <= e^-4; below
        // it g = e^{(beta+1) X} sum_n (-1)^n u^n integrates term by term, with k_n =
        // beta + 1 + n (alpha + beta):  int e^{kX} = e^{k xc} / k,  int X e^{kX} =
        // (e^{k xc} / k) (xc - 1 / k);  g fB carries the factor n + 1 and g fA the factor
        // -n.  Four terms leave < 1e-7 of the tail.
        const float xc = fminf(xhi, 0.0f) - TAIL_CUT * __builtin_amdgcn_rcpf(p.ab);
        span = xhi - xc;
        const float u = __builtin_amdgcn_exp2f(p.s_l2 * xc);
        float term = __builtin_amdgcn_exp2f(p.b_l2 * xc), sv = 0.0f, st = 0.0f, sa = 0.0f, sb = 0.0f;
#pragma unroll
        for (int n = 0; n < TAIL_TERMS; ++n) {
            const float ik = __builtin_amdgcn_rcpf(p.bp1 + (float)n * p.ab);
            const float I = ((n & 1) ? -term : term) * ik, g1 = xc - ik;
            sv += I;
            if (DERIV) {
                st = fmaf(I, p.alpha - p.ab * (float)(n + 1), st);
                sa = fmaf(-(float)n * I, g1, sa);
                sb = fmaf((float)(n + 1) * I, g1, sb);
            }
            term *= u;
        }
        tail = p.tau * sv;
        if (DERIV) {
            tail_t = st;
            tail_a = -p.tau * sa;
            tail_b = p.tau * sb;
        }
    }
    float s = 0.0f, sf = 0.0f, sa = 0.0f, sb = 0.0f, hw;
    const float npan = span * p.inv_w;
    if (a_hi <= 0.0078125f * t_obs) {
        // young bin: its span in X is below 9e-4, so the midpoint rule's relative error,
        // span^2 |g''/g| / 24 with |g''/g| <= (beta+1)^2 + (alpha+beta)^2 / 4 + ..., stays
        // below 5e-6 over alpha, beta <= 8 (typically below 1e-7)
        hw = 0.5f * span;
        dpl_node<DERIV>(p, xhi - hw, 2.0f, s, sf, sa, sb);
    } else if (npan <= 0.25f) {
        hw = 0.5f * span;
        const float c = xhi - hw, d = hw * GL2X;
        dpl_node<DERIV>(p, c - d, 1.0f, s, sf, sa, sb);
        dpl_node<DERIV>(p, c + d, 1.0f, s, sf, sa, sb);
    } else {
        int n = (int)ceilf(npan);
        n = min(max(n, 1), 64);
        hw = 0.5f * span * __builtin_amdgcn_rcpf((float)n);   // n is a small integer
        const float xlo = xhi - span;
        for (int q = 0; q < n; ++q) {
            const float c = xlo + (float)(2 * q + 1) * hw;
#pragma unroll
            for (int g = 0; g < 4; ++g) dpl_node<DERIV>(p, fmaf(hw, GL4X[g], c), GL4W[g], s, sf, sa, sb);
        }
    }
    const float th = p.tau * hw;
    m = fmaf(s, th, tail);
    if (DERIV) {
        d_tau = fmaf(hw, p.alpha * s - p.ab * sf, tail_t);
        d_al = fmaf(-th, sa, tail_a);
        d_be = fmaf(sb, th, tail_b);
    }
}

// FP64 variant (exact FP64 path): 8-point Gauss-Legendre panels of half the
// FP32 width, FP64 nodes; value only.
__device__ inline double dpl_bin_f64(const DevConsts &k, double a_lo, double a_hi, double t_obs, double tau,
                                     double al, double be) {
    if (!(a_lo < t_obs)) return 0.0;
    const double am1 = al - 1.0, bp1 = be + 1.0, ltau = log(tau);
    const double w = 0.5 * fmin(0.4, fmin(2.0 / (al + be), 1.2 / bp1));
    const double xhi = log(t_obs - a_lo) - ltau;
    double span, tail = 0.0;
    if (a_hi < t_obs) {
        span = log1p((a_hi - a_lo) / (t_obs - a_hi));
    } else {
        const double xlo = fmin(xhi, 0.0) - 40.0 / bp1;
        span = xhi - xlo;
        tail = tau * exp(bp1 * xlo) / bp1;
    }
    int n = (int)ceil(span / w);
    n = min(max(n, 1), 256);
    const double hw = 0.5 * span / n;
    const double xlo = xhi - span;
    double s = 0.0;
    for (int q = 0; q < n; ++q) {
        const double c = xlo + (2 * q + 1) * hw;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const double d = hw * k.gl8_x[g];
            const double X1 = c + d, X2 = c - d;
            s += k.gl8_w[g] * (tau / (exp(am1 * X1) + exp(-bp1 * X1)) + tau / (exp(am1 * X2) + exp(-bp1 * X2)));
        }
    }
    return s * hw + tail;
}

// ------------------------------------------------------------------ log-normal SFH (FP64)
// mass in bin i up to the common factor t_p w sqrt(2 pi) e^{w^2/2}, which cancels in the weights
template <bool DERIV>
__device__ inline void logn_bin_e(double a_lo, double a_hi, double t_obs, double tp, double w, double &m,
                                  double &d_tp, double &d_w) {
    m = d_tp = d_w = 0.0;
    if (!(a_lo < t_obs)) return;
    const double t_hi = t_obs - a_lo;
    const double l_hi = log(t_hi / tp), x_hi = l_hi / w - w;
    if (a_hi < t_obs) {
        const double t_lo = t_obs - a_hi;
        const double l_lo = log(t_lo / tp), x_lo = l_lo / w - w;
        m = (x_lo > 0.0) ? Phic_d(x_lo) - Phic_d(x_hi) : Phi_d(x_hi) - Phi_d(x_lo);
        if (DERIV) {
            const double f_hi = phi_d(x_hi), f_lo = phi_d(x_lo);
            d_tp = (f_lo - f_hi) / (tp * w);
            d_w = f_hi * (-l_hi / (w * w) - 1.0) - f_lo * (-l_lo / (w * w) - 1.0);
        }
    } else {
        m = Phi_d(x_hi);
        if (DERIV) {
            const double f_hi = phi_d(x_hi);
            d_tp = -f_hi / (tp * w);
            d_w = f_hi * (-l_hi / (w * w) - 1.0);
        }
    }
}

// FP32 form for the approximate and FP32 / BF16X exact paths.  A bin's mass is the integral of
// phi(x) over its span in x = ln(t / t_p) / w - w (the same common factor as above), taken by
// Gauss-Legendre quadrature of phi rather than as a difference of two normal CDFs, which in
// FP32 would cancel in the narrow young bins.  The span comes from log1p of the age-edge ratio.
// The same nodes give the derivatives: d/dt_p = (1 / (t_p w)) int x phi and, with
// dx/dw = -x/w - 2 at both edges, d/dw = int phi (x^2 / w + 2 x - 1 / w).  Rule, on the span
// h measured in units of phi's local scale, h max(1, |x|): the midpoint up to 0.01, 2 points up
// to 0.15, else 4-point panels of at most 0.5 (against FP64 normal-CDF differences over t_p
// 0.5-13 Gyr, w 0.15-2, t_obs 2-12 Gyr: bin masses within 1e-5 relative, where FP32 x itself
// limits far tails, and the derivatives within 5e-7 of their sum over the bins).  The oldest
// bin, open to t = 0, is the normal CDF at its upper edge (a tail value: no cancellation).
struct Logn {
    float w, inv_w, ltp, inv_tpw;   // width, 1 / w, ln t_p, 1 / (t_p w)
};
__device__ inline Logn make_logn(float tp, float w) {
    Logn p;
    p.w = w;
    p.inv_w = 1.0f / w;
    p.ltp = logf(tp);
    p.inv_tpw = 1.0f / (tp * w);
    return p;
}

template <bool DERIV>
__device__ inline void logn_bin(float a_lo, float a_hi, float t_obs, const Logn &p, float &m, float &d_tp,
                                float &d_w) {
    m = d_tp = d_w = 0.0f;
    if (!(a_lo < t_obs)) return;
    const float x_hi = (__builtin_amdgcn_logf(t_obs - a_lo) * 0.69314718055994531f - p.ltp) * p.inv_w - p.w;
    if (!(a_hi < t_obs)) {
        m = Phi_f(x_hi);
        if (DERIV) {
            const float f = phi_f(x_hi);
            d_tp = -f * p.inv_tpw;
            d_w = f * (-x_hi * p.inv_w - 2.0f);
        }
        return;
    }
    const float d = (a_hi - a_lo) * __builtin_amdgcn_rcpf(t_obs - a_hi), u = 1.0f + d;
    const float dl = (u == 1.0f) ? d : __builtin_amdgcn_logf(u) * 0.69314718055994531f * (d * __builtin_amdgcn_rcpf(u - 1.0f));
    const float span = dl * p.inv_w;
    // phi changes over 1 / |x| in its tails: the rule is chosen on the span in those units
    const float heff = span * fmaxf(1.0f, fmaxf(fabsf(x_hi), fabsf(x_hi - span)));
    float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, hw;
    auto node = [&](float x, float wg) {
        const float f = wg * __builtin_amdgcn_exp2f(-0.72134752044448170f * x * x);   // e^{-x^2/2}
        s0 += f;
        if (DERIV) {
            s1 = fmaf(f, x, s1);
            s2 = fmaf(f * x, x, s2);
        }
    };
    if (heff <= 0.01f) {
        hw = 0.5f * span;
        node(x_hi - hw, 2.0f);
    } else if (heff <= 0.15f) {
        hw = 0.5f * span;
        const float c = x_hi - hw, dd = hw * GL2X;
        node(c - dd, 1.0f);
        node(c + dd, 1.0f);
    } else {
        int n = (int)ceilf(heff * 2.0f);
        n = min(max(n, 1), 256);
        hw = 0.5f * span * __builtin_amdgcn_rcpf((float)n);
        const float xlo = x_hi - span;
        for (int q = 0; q < n; ++q) {
            const float c = xlo + (float)(2 * q + 1) * hw;
#pragma unroll
            for (int g = 0; g < 4; ++g) node(fmaf(hw, GL4X[g], c), GL4W[g]);
        }
    }
    const float h = 0.3989422804014327f * hw;   // 1 / sqrt(2 pi) and the panel half-width
    m = h * s0;
    if (DERIV) {
        d_tp = h * s1 * p.inv_tpw;
        d_w = h * fmaf(s2 - s0, p.inv_w, 2.0f * s1);
    }
}

// ------------------------------------------------------------------ burst (triweight)
// unnormalised probability of bin i and its derivative w.r.t. mu = log10 T_peak
// (inv_s3 = 1 / (3 sigma_burst))
// The burst and its window use the log-age bin edges e_0 .. e_NA (bin i spans [e_i, e_i+1];
// -inf and +inf at the ends), read at lane-dependent bins: the kernels keep a copy in LDS.
__device__ inline void stage_log_age_edges(const DevConsts &k, float *ledge) {
    for (int i = threadIdx.x; i <= NA; i += blockDim.x) ledge[i] = (i < NA) ? k.lage_lo[i] : k.lage_hi[NA - 1];
    __syncthreads();
}

// The window is walked edge by edge: an edge at standardised log age u keeps the tail value
// C(-|u|) (no difference near 1 cancels) and, if DERIV, the density C'(u); each edge serves
// the two bins it bounds.  Edges are clipped to log10 t_obs, so bins past t_obs (and past
// the last bin) come out empty.
struct BurstEdge {
    float u, tail, d;
};
// an edge at log age le
template <bool DERIV>
__device__ inline BurstEdge burst_edge_at(float le, float l_obs, float mu, float inv_s3) {
    BurstEdge r;
    r.u = (fminf(le, l_obs) - mu) * inv_s3;
    r.tail = tri_cdf(-fabsf(r.u));
    r.d = DERIV ? tri_dcdf(r.u) : 0.0f;
    return r;
}
template <bool DERIV>
__device__ inline BurstEdge burst_edge(const float *ledge, int e, float l_obs, float mu, float inv_s3) {
    return burst_edge_at<DERIV>(ledge[min(e, NA)], l_obs, mu, inv_s3);
}
// profile mass between two edges (the derivative w.r.t. mu is (lo.d - hi.d) / (3 sigma))
__device__ inline float burst_mass(const BurstEdge &lo, const BurstEdge &hi) {
    return (lo.u > 0.0f) ? lo.tail - hi.tail : ((hi.u <= 0.0f) ? hi.tail - lo.tail : 1.0f - hi.tail - lo.tail);
}

// first age bin whose upper log-age edge exceeds v (edges increasing, last = +inf)
__device__ inline int first_bin_above(const float *ledge, float v) {
    int a = 0, b = NA - 1;
    while (a < b) {
        const int c = (a + b) >> 1;
        if (ledge[c + 1] > v) b = c;
        else a = c + 1;
    }
    return a;
}

// ------------------------------------------------------------------ metallicity
// All NZ metallicity weights (normal CDF differences over the bin edges) and, if DERIV, their
// derivatives w.r.t. mu; each interior edge is evaluated once.  An edge at standardised
// x carries the tail value T = 0.5 erfc(|x| / sqrt 2) (Phi(x) for x <= 0, 1 - Phi(x) for
// x > 0) so that no bin difference cancels against 1.
template <bool DERIV>
__device__ inline void met_weights(const DevConsts &k, float mu, float (&pz)[NZ], float (&dpz)[NZ]) {
    const float inv_s = 1.0f / k.sigma_logz;
    float xp = -INFINITY, tp = 0.0f, dp = 0.0f;   // the open lower edge
#pragma unroll
    for (int j = 0; j < NZ; ++j) {
        float x = INFINITY, t = 0.0f, d = 0.0f;    // the open upper edge of the last bin
        if (j < NZ - 1) {
            x = (k.met_hi[j] - mu) * inv_s;
            t = 0.5f * erfcf(0.7071067811865475f * fabsf(x));
            d = phi_f(x);
        }
        pz[j] = (xp > 0.0f) ? tp - t : ((x <= 0.0f) ? t - tp : 1.0f - tp - t);
        if (DERIV) dpz[j] = (dp - d) * inv_s;
        xp = x;
        tp = t;
        dp = d;
    }
}

// ------------------------------------------------------------------ dust at one wavelength
// x = lambda_rest / 5500 A;  F = F_floor + (1 - F_floor) exp(-tau_V x^delta)
struct DustVal {
    float F, dF_tauv, dF_delta, dF_floor;
};
__device__ inline DustVal dust_at(float x, float tauv, float delta, float ffloor) {
    DustVal d;
    const float lx = logf(x), xd = expf(delta * lx), e = expf(-tauv * xd);
    d.F = fmaf(1.0f - ffloor, e, ffloor);
    d.dF_floor = 1.0f - e;
    d.dF_tauv = -(1.0f - ffloor) * xd * e;
    d.dF_delta = d.dF_tauv * tauv * lx;
    return d;
}

// ------------------------------------------------------------------ wave helpers
__device__ inline int wave_min_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
    return __builtin_amdgcn_readfirstlane(v);
}
__device__ inline int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

}  // namespace sps
