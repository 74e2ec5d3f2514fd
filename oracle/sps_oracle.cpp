/*
 * SPS hot-path ORACLE -- test infrastructure only (tests, smoke check, CPU
 * baseline).  Plain FP64, written step by step from the paper:
 *
 *   composite SED            Sec. 2 / App. A, Eq. (galSEDdef), separable weights Eq. (Pssp)
 *   total mass formed        App. A.1, Eq. (totalMstarFormed)
 *   smooth SFH (double PL)   App. A.1, Eq. (SFRsmooth); bin weights Eq. (smoothPsfh)
 *   burst mixture            App. A.1, Eq. (composite age weights) + triweight Eq. (triweight)
 *   metallicity (lognormal)  App. A.2
 *   dust attenuation         App. A.3, Eq. (DustAtt) + unobscured floor
 *   exact photometry         Sec. 3, Eq. (photo integral exact)
 *   effective wavelength     Sec. 3, Eq. (lambda_eff)
 *   approximate photometry   Sec. 3, Eq. (photo integral approx) with a c_SSP(z) lookup table
 *   bounding function        App. C, Eq. (BoundingFunction)
 *   skew-normal prior        App. C, Eq. (SkewNormPrior)
 *   Gaussian likelihood      App. D.1 (diagonal covariance)
 *   HMC + leapfrog           Sec. 4 / App. D.2 (fixed-length trajectories; step size
 *                            and, optionally, a diagonal mass matrix adapted in a
 *                            warm-up phase)
 *
 * Readings where the paper is silent or garbled are restated next to the code
 * they govern.  No blocking, fusion or reordering:
 * each quantity is computed from its definition.  Derivatives come from
 * forward-mode dual numbers carried through the same code.
 */
#include "sps_oracle.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

namespace {

constexpr int NP = ORC_NPARAM;
constexpr double PI = 3.14159265358979323846264338327950288;
constexpr double LN10 = 2.30258509299404568401799145468436421;
constexpr double C_KMS = 299792.458;                 // km/s
constexpr double C_ANGS = 2.99792458e18;             // A/s
constexpr double MPC_CM = 3.0856775814913673e24;
constexpr double MPC_KM = 3.0856775814913673e19;
constexpr double GYR_S = 3.15576e16;                 // Julian Gyr
constexpr double LSUN = 3.828e33;                    // erg/s (IAU nominal)
constexpr double AB_FNU0 = 3631.0e-23;               // erg/s/cm^2/Hz
constexpr double LAMBDA_V = 5500.0;                  // A
constexpr double INF = std::numeric_limits<double>::infinity();
constexpr double NaN = std::numeric_limits<double>::quiet_NaN();

// ------------------------------------------------------------------------
// forward-mode dual numbers: value + NP partial derivatives
// ------------------------------------------------------------------------
struct Dual {
    double v;
    double d[NP];
    Dual() : v(0.0) { for (int i = 0; i < NP; ++i) d[i] = 0.0; }
    Dual(double x) : v(x) { for (int i = 0; i < NP; ++i) d[i] = 0.0; }  // NOLINT
};
inline double val(double x) { return x; }
inline double val(const Dual &x) { return x.v; }

inline Dual operator+(const Dual &a, const Dual &b) { Dual r; r.v = a.v + b.v; for (int i = 0; i < NP; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual &a, const Dual &b) { Dual r; r.v = a.v - b.v; for (int i = 0; i < NP; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator*(const Dual &a, const Dual &b) { Dual r; r.v = a.v * b.v; for (int i = 0; i < NP; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator/(const Dual &a, const Dual &b) { Dual r; r.v = a.v / b.v; double ib = 1.0 / b.v; for (int i = 0; i < NP; ++i) r.d[i] = (a.d[i] - r.v * b.d[i]) * ib; return r; }
inline Dual operator-(const Dual &a) { Dual r; r.v = -a.v; for (int i = 0; i < NP; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator+(const Dual &a, double b) { Dual r = a; r.v += b; return r; }
inline Dual operator+(double a, const Dual &b) { return b + a; }
inline Dual operator-(const Dual &a, double b) { Dual r = a; r.v -= b; return r; }
inline Dual operator-(double a, const Dual &b) { Dual r = -b; r.v += a; return r; }
inline Dual operator*(const Dual &a, double b) { Dual r; r.v = a.v * b; for (int i = 0; i < NP; ++i) r.d[i] = a.d[i] * b; return r; }
inline Dual operator*(double a, const Dual &b) { return b * a; }
inline Dual operator/(const Dual &a, double b) { return a * (1.0 / b); }
inline Dual operator/(double a, const Dual &b) { Dual r; r.v = a / b.v; double s = -r.v / b.v; for (int i = 0; i < NP; ++i) r.d[i] = s * b.d[i]; return r; }
inline Dual &operator+=(Dual &a, const Dual &b) { a = a + b; return a; }
inline Dual &operator-=(Dual &a, const Dual &b) { a = a - b; return a; }
inline Dual &operator*=(Dual &a, const Dual &b) { a = a * b; return a; }
inline Dual &operator/=(Dual &a, const Dual &b) { a = a / b; return a; }

inline Dual chain(const Dual &a, double f, double df) {  // f(a) with f' = df
    Dual r; r.v = f; for (int i = 0; i < NP; ++i) r.d[i] = df * a.d[i]; return r;
}
inline Dual exp(const Dual &a) { double e = std::exp(a.v); return chain(a, e, e); }
inline Dual log(const Dual &a) { return chain(a, std::log(a.v), 1.0 / a.v); }
inline Dual sqrt(const Dual &a) { double s = std::sqrt(a.v); return chain(a, s, 0.5 / s); }
inline Dual pow(const Dual &a, const Dual &b) { return exp(b * log(a)); }
inline Dual pow(double a, const Dual &b) { double r = std::pow(a, b.v); return chain(b, r, r * std::log(a)); }
inline Dual pow(const Dual &a, double b) { double r = std::pow(a.v, b); return chain(a, r, b * std::pow(a.v, b - 1.0)); }

// standard normal CDF, from erfc (no cancellation in the lower tail)
inline double Phi(double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); }
inline double phi(double x) { return std::exp(-0.5 * x * x) / std::sqrt(2.0 * PI); }
inline Dual Phi(const Dual &x) { return chain(x, Phi(x.v), phi(x.v)); }

using std::exp;
using std::log;
using std::pow;
using std::sqrt;

// ------------------------------------------------------------------------
// Gauss-Legendre nodes by the Golub-Welsch method, and adaptive bisection
// ------------------------------------------------------------------------
// The n-point rule's nodes are the eigenvalues of the symmetric tridiagonal Jacobi matrix of
// the Legendre three-term recurrence (zero diagonal, off-diagonal k / sqrt(4k^2 - 1)), and each
// weight is 2 (the integral of the weight function) times the squared first component of the
// node's unit eigenvector (Golub & Welsch 1969).  The eigenproblem is solved by cyclic Jacobi
// rotations, which for n <= 16 converge to rounding in a handful of sweeps.
struct GaussLegendre {
    int n;
    double x[16], w[16];
    explicit GaussLegendre(int n_) : n(n_) {
        long double a[16][16] = {{0.0L}}, v[16][16] = {{0.0L}};   // extended precision, rounded at the end
        for (int i = 0; i < n; ++i) v[i][i] = 1.0;
        for (int k = 1; k < n; ++k) a[k - 1][k] = a[k][k - 1] = k / std::sqrt(4.0L * k * k - 1.0L);
        for (int sweep = 0; sweep < 50; ++sweep) {
            long double off = 0.0L;
            for (int i = 0; i < n; ++i)
                for (int j = i + 1; j < n; ++j) off += a[i][j] * a[i][j];
            if (off < 1e-4000L) break;
            for (int pi = 0; pi < n; ++pi)
                for (int qi = pi + 1; qi < n; ++qi) {
                    if (a[pi][qi] == 0.0L) continue;
                    // rotation in the (pi, qi) plane that zeroes a[pi][qi]
                    const long double th = (a[qi][qi] - a[pi][pi]) / (2.0L * a[pi][qi]);
                    const long double t = (th >= 0.0L ? 1.0L : -1.0L) / (std::fabs(th) + std::sqrt(th * th + 1.0L));
                    const long double c = 1.0L / std::sqrt(t * t + 1.0L), sn = t * c;
                    for (int r = 0; r < n; ++r) {   // A <- A G (columns pi, qi)
                        const long double ap = a[r][pi], aq = a[r][qi];
                        a[r][pi] = c * ap - sn * aq;
                        a[r][qi] = sn * ap + c * aq;
                    }
                    for (int r = 0; r < n; ++r) {   // A <- G^T A (rows pi, qi)
                        const long double ap = a[pi][r], aq = a[qi][r];
                        a[pi][r] = c * ap - sn * aq;
                        a[qi][r] = sn * ap + c * aq;
                    }
                    for (int r = 0; r < n; ++r) {   // eigenvectors: V <- V G
                        const long double vp = v[r][pi], vq = v[r][qi];
                        v[r][pi] = c * vp - sn * vq;
                        v[r][qi] = sn * vp + c * vq;
                    }
                }
        }
        // nodes in increasing order with their weights
        int idx[16];
        for (int i = 0; i < n; ++i) idx[i] = i;
        std::sort(idx, idx + n, [&](int i, int j) { return a[i][i] < a[j][j]; });
        long double xl[16], wl[16];
        for (int i = 0; i < n; ++i) {
            xl[i] = a[idx[i]][idx[i]];
            wl[i] = 2.0L * v[0][idx[i]] * v[0][idx[i]];
        }
        // the rule is symmetric: average the mirrored pairs (and put the middle node of an odd
        // rule exactly at 0)
        for (int i = 0; i < n / 2; ++i) {
            const long double xs = 0.5L * (xl[n - 1 - i] - xl[i]), ws = 0.5L * (wl[i] + wl[n - 1 - i]);
            x[i] = (double)-xs;
            x[n - 1 - i] = (double)xs;
            w[i] = w[n - 1 - i] = (double)ws;
        }
        if (n % 2) {
            x[n / 2] = 0.0;
            w[n / 2] = (double)wl[n / 2];
        }
    }
};
const GaussLegendre GL10(10);

template <class T, class F>
T gl_rule(const F &f, double a, double b) {
    double h = 0.5 * (b - a), m = 0.5 * (a + b);
    T s(0.0);
    for (int k = 0; k < GL10.n; ++k) s += GL10.w[k] * f(m + h * GL10.x[k]);
    return s * h;
}

template <class T, class F>
T adapt(const F &f, double a, double b, const T &whole, double tol, int depth, int &budget) {
    double m = 0.5 * (a + b);
    T l = gl_rule<T>(f, a, m), r = gl_rule<T>(f, m, b);
    T lr = l + r;
    budget -= 1;
    double e = std::fabs(val(lr) - val(whole));
    // stop on convergence, on non-finite values, at the depth limit, or when the
    // subdivision budget of this integral is spent
    if (!(e > tol) || !std::isfinite(val(lr)) || depth >= 60 || budget <= 0) return lr;
    return adapt<T>(f, a, m, l, tol, depth + 1, budget) + adapt<T>(f, m, b, r, tol, depth + 1, budget);
}

// integral of f over [a, b] to relative accuracy ~rel (value part drives refinement)
template <class T, class F>
T integrate(const F &f, double a, double b, double rel = 1e-13) {
    if (!(b > a)) return T(0.0);
    const int n0 = 8;
    T parts[n0];
    double scale = 0.0;
    for (int p = 0; p < n0; ++p) {
        double lo = a + (b - a) * p / n0, hi = (p == n0 - 1) ? b : a + (b - a) * (p + 1) / n0;
        parts[p] = gl_rule<T>(f, lo, hi);
        scale += std::fabs(val(parts[p]));
    }
    // absolute floor far below anything that matters, so underflowing tails converge
    double tol = std::max(rel * scale, 1e-290);
    int budget = 4000;
    T s(0.0);
    for (int p = 0; p < n0; ++p) {
        double lo = a + (b - a) * p / n0, hi = (p == n0 - 1) ? b : a + (b - a) * (p + 1) / n0;
        s += adapt<T>(f, lo, hi, parts[p], tol / n0, 0, budget);
    }
    return s;
}

// ------------------------------------------------------------------------
// cosmology: flat LCDM with matter + Lambda (reading: H0 = 70, Om = 0.3)
// ------------------------------------------------------------------------
double hubble_per_gyr(const orc_cosmo &c) { return c.H0 / MPC_KM * GYR_S; }

// t(z) = int_0^{a} da' / (a' H(a')),  a = 1/(1+z);  substitute a' = s^2 so the
// integrand 2 s^2 / (H0 sqrt(Om + OL s^6)) is smooth at the big bang.
double age_universe(const orc_cosmo &c, double z) {
    double H = hubble_per_gyr(c), OL = 1.0 - c.Om;
    auto f = [&](double s) { return 2.0 * s * s / (H * std::sqrt(c.Om + OL * std::pow(s, 6))); };
    return integrate<double>(f, 0.0, std::sqrt(1.0 / (1.0 + z)), 1e-15);
}

// D_L = (1+z) (c/H0) int_0^z dz'/E(z'),  E = sqrt(Om (1+z)^3 + OL)
double lum_distance_mpc(const orc_cosmo &c, double z) {
    double OL = 1.0 - c.Om;
    auto f = [&](double zz) { return 1.0 / std::sqrt(c.Om * std::pow(1.0 + zz, 3) + OL); };
    return (1.0 + z) * (C_KMS / c.H0) * integrate<double>(f, 0.0, z, 1e-15);
}

// ------------------------------------------------------------------------
// grids: bin edges at midpoints of the (log) grid, open-ended at both ends
// ------------------------------------------------------------------------
struct Grid {
    const orc_ssp *s;
    std::vector<double> met_edge;     // [n_met+1], -inf .. +inf (log10 Z)
    std::vector<double> lage_edge;    // [n_age+1], -inf .. +inf (log10 yr)
    std::vector<double> age_edge;     // [n_age+1], 0 .. inf (Gyr)
    std::vector<double> trap;         // [n_wave] trapezoid weights on the wavelength grid
    explicit Grid(const orc_ssp *s_) : s(s_) {
        int nm = s->n_met, na = s->n_age, nw = s->n_wave;
        met_edge.assign(nm + 1, 0.0);
        met_edge[0] = -INF;
        met_edge[nm] = INF;
        for (int j = 1; j < nm; ++j) met_edge[j] = 0.5 * (s->log10_met[j - 1] + s->log10_met[j]);
        lage_edge.assign(na + 1, 0.0);
        age_edge.assign(na + 1, 0.0);
        lage_edge[0] = -INF;
        lage_edge[na] = INF;
        for (int i = 1; i < na; ++i) lage_edge[i] = 0.5 * (s->log10_age_yr[i - 1] + s->log10_age_yr[i]);
        for (int i = 0; i <= na; ++i) age_edge[i] = (i == 0) ? 0.0 : (i == na ? INF : std::pow(10.0, lage_edge[i]) * 1e-9);
        trap.assign(nw, 0.0);
        for (int k = 0; k < nw; ++k) {
            double lo = (k == 0) ? s->wave_A[0] : s->wave_A[k - 1];
            double hi = (k == nw - 1) ? s->wave_A[nw - 1] : s->wave_A[k + 1];
            trap[k] = 0.5 * (hi - lo);
        }
    }
    double L(int j, int i, int k) const { return s->lum[((size_t)j * s->n_age + i) * s->n_wave + k]; }
};

// ------------------------------------------------------------------------
// star-formation history
// ------------------------------------------------------------------------
// Smooth SFR at cosmic time t [Gyr] (amplitude 1: only the shape matters, the
// mass normalisation is 10^theta[0] = total mass formed by t_obs).
//   double power law (Eq. SFRsmooth): 1 / ((t/tau)^alpha + (t/tau)^-beta)
//   log-normal in cosmic time:        exp(-(ln(t/t_peak))^2 / (2 w^2))
template <class T>
T sfr(int sfh, const T *th, double t) {
    if (!(t > 0.0)) return T(0.0);
    if (sfh == 0) {
        T x = log(t / th[1]) / th[2];
        return exp(-0.5 * (x * x));
    }
    T u = t / th[1];
    return 1.0 / (pow(u, th[2]) + pow(u, -th[3]));
}

// Mass formed in each age bin (Eq. smoothPsfh, reading: bin i spans the
// stellar ages between the midpoint edges, i.e. formation times
// [t_obs - age_hi, t_obs - age_lo] clipped to [0, t_obs]).  The integral is
// taken over stellar age a, with formation time t = t_obs - a.
template <class T>
void smooth_bin_mass(const Grid &G, int sfh, const T *th, double t_obs, T *mass) {
    for (int i = 0; i < G.s->n_age; ++i) {
        double a_lo = G.age_edge[i], a_hi = std::min(G.age_edge[i + 1], t_obs);
        if (a_lo >= t_obs) { mass[i] = T(0.0); continue; }
        auto f = [&](double a) { return sfr<T>(sfh, th, t_obs - a); };
        mass[i] = integrate<T>(f, a_lo, a_hi);
    }
}

// triweight kernel (Eq. triweight)
template <class T>
T triweight(const T &x) {
    if (std::fabs(val(x)) > 3.0) return T(0.0);
    T u = x / 3.0;
    T v = 1.0 - u * u;
    return (35.0 / 96.0) * (v * v * v);
}

// Burst age PDF: probability of each log-age bin under the triweight in
// x = (log10 age - log10 T_peak) / sigma, sigma = (log10 T_max - log10 T_peak)/3.
// Bins are clipped to ages below t_obs and the weights renormalised.  The
// integral of the degree-6 polynomial on [-3, 3] is exact with 10-point Gauss.
template <class T>
void burst_weights(const Grid &G, const orc_model &M, const T *th, double t_obs, T *p) {
    const int na = G.s->n_age;
    const double sig = M.burst_dlogt / 3.0;
    const double l_obs = std::log10(t_obs * 1e9);
    T tot(0.0);
    for (int i = 0; i < na; ++i) {
        double lo = G.lage_edge[i], hi = std::min(G.lage_edge[i + 1], l_obs);
        p[i] = T(0.0);
        if (lo >= l_obs) continue;
        T xlo = (lo - th[5]) / sig, xhi = (hi - th[5]) / sig;
        if (!(val(xlo) > -3.0)) xlo = T(-3.0);
        if (!(val(xhi) < 3.0)) xhi = T(3.0);
        if (!(val(xhi) > val(xlo))) continue;
        T mid = 0.5 * (xlo + xhi), half = 0.5 * (xhi - xlo);
        T s(0.0);
        for (int k = 0; k < GL10.n; ++k) s += GL10.w[k] * triweight<T>(mid + half * GL10.x[k]);
        p[i] = s * half;
        tot += p[i];
    }
    if (val(tot) > 0.0)
        for (int i = 0; i < na; ++i) p[i] = p[i] / tot;
}

// Age weights: P_SFH = (1 - F_burst) P_smooth + F_burst P_burst (Eq. composite age weights)
template <class T>
void age_weights(const Grid &G, const orc_model &M, int sfh, const T *th, double t_obs,
                 T *p_age, T *p_smooth, T *p_burst) {
    const int na = G.s->n_age;
    smooth_bin_mass<T>(G, sfh, th, t_obs, p_smooth);
    T tot(0.0);
    for (int i = 0; i < na; ++i) tot += p_smooth[i];
    for (int i = 0; i < na; ++i) p_smooth[i] = p_smooth[i] / tot;
    burst_weights<T>(G, M, th, t_obs, p_burst);
    for (int i = 0; i < na; ++i) p_age[i] = (1.0 - th[4]) * p_smooth[i] + th[4] * p_burst[i];
}

// Metallicity weights: Gaussian in log10 Z with median mu and width sigma_logZ,
// integrated over the midpoint bins of the Z grid (open-ended at both ends).
template <class T>
void met_weights(const Grid &G, const orc_model &M, const T *th, T *p) {
    for (int j = 0; j < G.s->n_met; ++j) {
        double lo = G.met_edge[j], hi = G.met_edge[j + 1];
        T c_hi = std::isinf(hi) ? T(1.0) : Phi((hi - th[6]) / M.sigma_logz);
        T c_lo = std::isinf(lo) ? T(0.0) : Phi((lo - th[6]) / M.sigma_logz);
        p[j] = c_hi - c_lo;
    }
}

// Attenuation (Eq. DustAtt with k0 = 4.05, D = 0, A_V = 2.5 log10(e) tau_V) and the
// unobscured floor:  F = F_floor + (1 - F_floor) exp(-tau_V (lambda/5500)^delta)
template <class T>
T dust_att(const T *th, double lam_rest) {
    return th[9] + (1.0 - th[9]) * exp(-th[7] * pow(lam_rest / LAMBDA_V, th[8]));
}

// AB normalisation: flux ratio = K(z) * sum(...) with
// K = (1+z) Lsun / (4 pi D_L^2 c 3631 Jy)   [photon-counting AB, rest-frame integral]
double k_dist(const orc_cosmo &c, double z) {
    double dl = lum_distance_mpc(c, z) * MPC_CM;
    return (1.0 + z) * LSUN / (4.0 * PI * dl * dl * C_ANGS * AB_FNU0);
}

double gauss_t(const orc_filters &f, int b, double lam_obs) {
    double x = (lam_obs - f.center_A[b]) / f.sigma_A[b];
    return std::exp(-0.5 * x * x);
}

// lambda_eff = int lambda T / int T over the observed-frame filter (Eq. lambda_eff)
double lambda_eff(const orc_filters &f, int b) {
    double c = f.center_A[b], s = f.sigma_A[b];
    double lo = std::max(0.0, c - 40.0 * s), hi = c + 40.0 * s;
    auto num = [&](double l) { return l * gauss_t(f, b, l); };
    auto den = [&](double l) { return gauss_t(f, b, l); };
    return integrate<double>(num, lo, hi, 1e-15) / integrate<double>(den, lo, hi, 1e-15);
}

// band normalisation on the SSP wavelength nodes: N_b(z) = sum_k T_b((1+z) l_k) q_k / l_k
double band_norm(const Grid &G, const orc_filters &f, int b, double z) {
    double n = 0.0;
    for (int k = 0; k < G.s->n_wave; ++k) {
        double l = G.s->wave_A[k];
        n += gauss_t(f, b, (1.0 + z) * l) * G.trap[k] / l;
    }
    return n;
}

// Exact photometry (Eq. photo integral exact): the composite SED on the SSP
// wavelength grid, attenuated, integrated against the redshifted filter with
// the trapezoid rule, photon-counting AB normalisation.
template <class T>
void mags_exact(const Grid &G, const orc_filters &f, const orc_cosmo &c, const orc_model &M,
                int sfh, const T *th, double z, T *mags) {
    const int nm = G.s->n_met, na = G.s->n_age, nw = G.s->n_wave, nb = f.n_band;
    double t_obs = age_universe(c, z), K = k_dist(c, z);
    std::vector<T> pa(na), ps(na), pb(na), pm(nm), sed(nw, T(0.0));
    age_weights<T>(G, M, sfh, th, t_obs, pa.data(), ps.data(), pb.data());
    met_weights<T>(G, M, th, pm.data());
    // SED(lambda) = sum_ij L_SSP(lambda | i, j) P(i) P(j)   (per unit mass formed)
    for (int j = 0; j < nm; ++j)
        for (int i = 0; i < na; ++i) {
            T w = pm[j] * pa[i];
            for (int k = 0; k < nw; ++k) sed[k] += w * G.L(j, i, k);
        }
    T mass = exp(LN10 * th[0]);
    for (int b = 0; b < nb; ++b) {
        T num(0.0);
        for (int k = 0; k < nw; ++k) {
            double l = G.s->wave_A[k];
            num += sed[k] * dust_att<T>(th, l) * (gauss_t(f, b, (1.0 + z) * l) * l * G.trap[k]);
        }
        T flux = K * mass * num / band_norm(G, f, b, z);
        mags[b] = -2.5 * log(flux) / LN10;
    }
}

// c_SSP on the z nodes, without the distance factor and divided by N_b(z_k)
void ztable(const Grid &G, const orc_filters &f, int n_z, double z_lo, double z_hi, double *q) {
    const int nm = G.s->n_met, na = G.s->n_age, nw = G.s->n_wave, nb = f.n_band;
#pragma omp parallel for schedule(dynamic, 1)
    for (int kb = 0; kb < n_z * nb; ++kb) {
        const int kz = kb / nb, b = kb % nb;
        double z = z_lo + (z_hi - z_lo) * kz / (n_z - 1);
        double nrm = band_norm(G, f, b, z);
        std::vector<double> tw(nw);  // T_b((1+z) l_k) l_k q_k
        for (int k = 0; k < nw; ++k) {
            double l = G.s->wave_A[k];
            tw[k] = gauss_t(f, b, (1.0 + z) * l) * l * G.trap[k];
        }
        for (int j = 0; j < nm; ++j)
            for (int i = 0; i < na; ++i) {
                double s = 0.0;
                for (int k = 0; k < nw; ++k) s += G.L(j, i, k) * tw[k];
                q[(((size_t)kz * nb + b) * nm + j) * na + i] = s / nrm;
            }
    }
}

// Approximate photometry (Eq. photo integral approx): attenuation pulled out at
// the rest-frame effective wavelength, c_SSP linearly interpolated in z (in flux).
template <class T>
bool mags_approx(const Grid &G, const orc_filters &f, const orc_cosmo &c, const orc_model &M,
                 int n_z, double z_lo, double z_hi, const double *q, int sfh, const T *th, double z,
                 T *mags) {
    const int nm = G.s->n_met, na = G.s->n_age, nb = f.n_band;
    if (!(z >= z_lo && z <= z_hi)) {
        for (int b = 0; b < nb; ++b) mags[b] = T(NaN);
        return false;
    }
    double dz = (z_hi - z_lo) / (n_z - 1), u = (z - z_lo) / dz;
    int kk = std::min((int)std::floor(u), n_z - 2);
    double fz = u - kk;
    double t_obs = age_universe(c, z), K = k_dist(c, z);
    std::vector<T> pa(na), ps(na), pb(na), pm(nm);
    age_weights<T>(G, M, sfh, th, t_obs, pa.data(), ps.data(), pb.data());
    met_weights<T>(G, M, th, pm.data());
    T mass = exp(LN10 * th[0]);
    for (int b = 0; b < nb; ++b) {
        const double *q0 = q + ((size_t)kk * nb + b) * nm * na;
        const double *q1 = q + ((size_t)(kk + 1) * nb + b) * nm * na;
        T acc(0.0);
        for (int j = 0; j < nm; ++j)
            for (int i = 0; i < na; ++i) {
                double cs = (1.0 - fz) * q0[j * na + i] + fz * q1[j * na + i];
                acc += pm[j] * pa[i] * cs;
            }
        T att = dust_att<T>(th, lambda_eff(f, b) / (1.0 + z));
        T flux = K * mass * att * acc;
        mags[b] = -2.5 * log(flux) / LN10;
    }
    return true;
}

template <class T>
T loglike(const T *mags, const double *obs, const double *sig, uint8_t mask, int nb) {
    T ll(0.0);
    for (int b = 0; b < nb; ++b) {
        if (!((mask >> b) & 1)) continue;
        T r = (mags[b] - obs[b]) / sig[b];
        ll += -0.5 * (r * r) - std::log(sig[b] * std::sqrt(2.0 * PI));
    }
    return ll;
}

// ---- bounding function (Eq. BoundingFunction) and skew-normal prior (Eq. SkewNormPrior)
template <class T>
T bound(const double *bnd, const T &x) {
    return bnd[0] + (bnd[1] - bnd[0]) / (1.0 + exp(-bnd[2] * (x - bnd[3])));
}
template <class T>
T log_Phi(const T &x) { return log(Phi(x)); }
template <class T>
T log_prior(const double *pri, const T &x) {
    T y = (x - pri[0]) / pri[1];
    return std::log(2.0 / pri[1]) - 0.5 * std::log(2.0 * PI) - 0.5 * (y * y) + log_Phi<T>(pri[2] * y);
}

struct Model {
    Grid G;
    orc_filters f;
    orc_cosmo c;
    orc_model m;
    Model(const orc_ssp *s, const orc_filters *f_, const orc_cosmo *c_, const orc_model *m_)
        : G(s), f(*f_), c(*c_), m(*m_) {}
};

bool check_common(const orc_ssp *s, const orc_filters *f) {
    if (!s || !s->lum || s->n_met < 1 || s->n_age < 2 || s->n_wave < 2) return false;
    if (f && (f->n_band < 1 || f->n_band > 8)) return false;
    return true;
}

// log posterior on unbounded parameters, value and gradient (dual numbers)
void logpost(const Model &X, int path, int n_z, double z_lo, double z_hi, const double *q, int sfh,
             const double *xu, double z, const double *obs, const double *sig, uint8_t mask,
             const double *bounds, const double *prior, double *lp, double *grad) {
    Dual x[NP], th[NP], mags[8];
    for (int p = 0; p < NP; ++p) { x[p] = Dual(xu[p]); x[p].d[p] = 1.0; }
    for (int p = 0; p < NP; ++p) th[p] = bound<Dual>(bounds + 4 * p, x[p]);
    // the magnitudes of either photometry path (Sec. 3): the z table or the full spectrum
    if (path == 0)
        mags_approx<Dual>(X.G, X.f, X.c, X.m, n_z, z_lo, z_hi, q, sfh, th, z, mags);
    else
        mags_exact<Dual>(X.G, X.f, X.c, X.m, sfh, th, z, mags);
    Dual v = loglike<Dual>(mags, obs, sig, mask, X.f.n_band);
    for (int p = 0; p < NP; ++p) v += log_prior<Dual>(prior + 3 * p, x[p]);
    *lp = v.v;
    for (int p = 0; p < NP; ++p) grad[p] = v.d[p];
}

// ---- Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011)
void philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

double u01(uint32_t w) { return (w + 0.5) * (1.0 / 4294967296.0); }

// Warm-up schedule of the windowed metric adaptation (the scheme of the Stan manual,
// which Blackjax's window adaptation also follows): a fast buffer of 75 iterations
// (step size only), slow windows that start at 25 iterations and double, a final fast
// buffer of 50.  When the three defaults do not fit, the buffers are 15 % and 10 % of
// the warm-up and one window takes the remaining 75 %.  A window is stretched to the
// end of the slow phase when the next, doubled, window would overrun it.
int hmc_windows(int nw, int max_win, int *start, int *end) {
    if (nw < 20) return 0;
    int init = 75, term = 50, base = 25;
    if (init + base + term > nw) {
        init = (int)(0.15 * nw);
        term = (int)(0.1 * nw);
        base = nw - init - term;
    }
    const int slow_end = nw - term;
    int n = 0, s = init, w = base;
    while (s < slow_end) {
        int e = s + w;
        if (e + 2 * w > slow_end) e = slow_end;
        if (n < max_win) { start[n] = s; end[n] = e; }
        ++n;
        s = e;
        w *= 2;
    }
    return n;
}

}  // namespace

// =========================================================================
// C ABI
// =========================================================================
extern "C" {

double orc_age_universe_gyr(const orc_cosmo *c, double z) { return age_universe(*c, z); }
double orc_lum_distance_mpc(const orc_cosmo *c, double z) { return lum_distance_mpc(*c, z); }

int orc_smooth_bin_mass(const orc_ssp *s, const orc_cosmo *c, int sfh, const double *theta, double z,
                        double *mass) {
    if (!check_common(s, nullptr) || !theta || !mass) return 1;
    Grid G(s);
    smooth_bin_mass<double>(G, sfh, theta, age_universe(*c, z), mass);
    return 0;
}

int orc_age_weights(const orc_ssp *s, const orc_cosmo *c, const orc_model *m, int sfh,
                    const double *theta, double z, double *p_age, double *p_smooth, double *p_burst) {
    if (!check_common(s, nullptr) || !theta) return 1;
    Grid G(s);
    int na = s->n_age;
    std::vector<double> pa(na), ps(na), pb(na);
    age_weights<double>(G, *m, sfh, theta, age_universe(*c, z), pa.data(), ps.data(), pb.data());
    if (p_age) std::memcpy(p_age, pa.data(), na * sizeof(double));
    if (p_smooth) std::memcpy(p_smooth, ps.data(), na * sizeof(double));
    if (p_burst) std::memcpy(p_burst, pb.data(), na * sizeof(double));
    return 0;
}

int orc_met_weights(const orc_ssp *s, const orc_model *m, const double *theta, double *p_met) {
    if (!check_common(s, nullptr) || !theta || !p_met) return 1;
    Grid G(s);
    met_weights<double>(G, *m, theta, p_met);
    return 0;
}

int orc_weights(const orc_ssp *s, const orc_cosmo *c, const orc_model *m, int sfh, int n_gal,
                const double *theta, const double *z, double *w) {
    if (!check_common(s, nullptr) || n_gal < 0 || (n_gal && (!theta || !z || !w))) return 1;
    Grid G(s);
    const int nm = s->n_met, na = s->n_age;
#pragma omp parallel for schedule(dynamic, 1)
    for (int g = 0; g < n_gal; ++g) {
        const double *th = theta + (size_t)g * NP;
        std::vector<double> pa(na), ps(na), pb(na), pm(nm);
        age_weights<double>(G, *m, sfh, th, age_universe(*c, z[g]), pa.data(), ps.data(), pb.data());
        met_weights<double>(G, *m, th, pm.data());
        double mass = std::pow(10.0, th[0]);
        for (int j = 0; j < nm; ++j)
            for (int i = 0; i < na; ++i) w[((size_t)g * nm + j) * na + i] = mass * pm[j] * pa[i];
    }
    return 0;
}

double orc_dust_att(const double *theta, double lam_rest_A) { return dust_att<double>(theta, lam_rest_A); }

double orc_lambda_eff(const orc_filters *f, int band) { return lambda_eff(*f, band); }

int orc_phot_exact(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                   int sfh, int n_gal, const double *theta, const double *z, double *mags) {
    if (!check_common(s, f) || n_gal < 0 || (n_gal && (!theta || !z || !mags))) return 1;
    Model X(s, f, c, m);
    const int nb = f->n_band;
#pragma omp parallel for schedule(dynamic, 1)
    for (int g = 0; g < n_gal; ++g)
        mags_exact<double>(X.G, X.f, X.c, X.m, sfh, theta + (size_t)g * NP, z[g], mags + (size_t)g * nb);
    return 0;
}

int orc_ztable(const orc_ssp *s, const orc_filters *f, int n_z, double z_lo, double z_hi, double *q) {
    if (!check_common(s, f) || n_z < 2 || !(z_hi > z_lo) || !q) return 1;
    Grid G(s);
    ztable(G, *f, n_z, z_lo, z_hi, q);
    return 0;
}

int orc_phot_approx(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                    int n_z, double z_lo, double z_hi, const double *q, int sfh, int n_gal,
                    const double *theta, const double *z, double *mags) {
    if (!check_common(s, f) || n_gal < 0 || !q || n_z < 2 || (n_gal && (!theta || !z || !mags))) return 1;
    Model X(s, f, c, m);
    const int nb = f->n_band;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int g = 0; g < n_gal; ++g)
        bad += !mags_approx<double>(X.G, X.f, X.c, X.m, n_z, z_lo, z_hi, q, sfh, theta + (size_t)g * NP,
                                    z[g], mags + (size_t)g * nb);
    return bad ? 2 : 0;
}

int orc_loglike_grad(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                     int path, int n_z, double z_lo, double z_hi, const double *q, int sfh, int n_gal,
                     const double *theta, const double *z, const double *obs, const double *sigma,
                     const uint8_t *mask, double *logl, double *grad) {
    if (!check_common(s, f) || n_gal < 0 || (path == 0 && !q)) return 1;
    if (n_gal && (!theta || !z || !obs || !sigma || !mask || !logl)) return 1;
    Model X(s, f, c, m);
    const int nb = f->n_band;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int g = 0; g < n_gal; ++g) {
        const double *thg = theta + (size_t)g * NP;
        const double *o = obs + (size_t)g * nb, *sg = sigma + (size_t)g * nb;
        if (grad) {
            Dual th[NP], mags[8];
            for (int p = 0; p < NP; ++p) { th[p] = Dual(thg[p]); th[p].d[p] = 1.0; }
            if (path == 0)
                bad += !mags_approx<Dual>(X.G, X.f, X.c, X.m, n_z, z_lo, z_hi, q, sfh, th, z[g], mags);
            else
                mags_exact<Dual>(X.G, X.f, X.c, X.m, sfh, th, z[g], mags);
            Dual ll = loglike<Dual>(mags, o, sg, mask[g], nb);
            logl[g] = ll.v;
            for (int p = 0; p < NP; ++p) grad[(size_t)g * NP + p] = ll.d[p];
        } else {
            double mags[8];
            if (path == 0)
                bad += !mags_approx<double>(X.G, X.f, X.c, X.m, n_z, z_lo, z_hi, q, sfh, thg, z[g], mags);
            else
                mags_exact<double>(X.G, X.f, X.c, X.m, sfh, thg, z[g], mags);
            logl[g] = loglike<double>(mags, o, sg, mask[g], nb);
        }
    }
    return bad ? 2 : 0;
}

int orc_mags_jacobian(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m, int path,
                      int n_z, double z_lo, double z_hi, const double *q, int sfh, int n_gal, const double *theta,
                      const double *z, double *mags, double *jac) {
    if (!check_common(s, f) || n_gal < 0 || (path == 0 && !q) || (n_gal && (!theta || !z || !mags || !jac)))
        return 1;
    Model X(s, f, c, m);
    const int nb = f->n_band;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
    for (int g = 0; g < n_gal; ++g) {
        Dual th[NP], mg[8];
        for (int p = 0; p < NP; ++p) { th[p] = Dual(theta[(size_t)g * NP + p]); th[p].d[p] = 1.0; }
        if (path == 0)
            bad += !mags_approx<Dual>(X.G, X.f, X.c, X.m, n_z, z_lo, z_hi, q, sfh, th, z[g], mg);
        else
            mags_exact<Dual>(X.G, X.f, X.c, X.m, sfh, th, z[g], mg);
        for (int b = 0; b < nb; ++b) {
            mags[(size_t)g * nb + b] = mg[b].v;
            for (int p = 0; p < NP; ++p) jac[((size_t)g * nb + b) * NP + p] = mg[b].d[p];
        }
    }
    return bad ? 2 : 0;
}

double orc_bound(const double *bnd, double x) { return bound<double>(bnd, x); }
double orc_unbound(const double *bnd, double th) {
    // inverse of the sigmoid: x0 - ln((y_hi - y_lo)/(theta - y_lo) - 1) / k
    return bnd[3] - std::log((bnd[1] - bnd[0]) / (th - bnd[0]) - 1.0) / bnd[2];
}
double orc_log_prior(const double *pri, double x) { return log_prior<double>(pri, x); }

int orc_logpost_grad(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m, int path,
                     int n_z, double z_lo, double z_hi, const double *q, int sfh, const double *theta_u,
                     double z, const double *obs, const double *sigma, uint8_t mask,
                     const double *bounds, const double *prior, double *logp, double *grad) {
    if (!check_common(s, f) || (path == 0 && !q) || !theta_u || !bounds || !prior || !logp || !grad) return 1;
    Model X(s, f, c, m);
    logpost(X, path, n_z, z_lo, z_hi, q, sfh, theta_u, z, obs, sigma, mask, bounds, prior, logp, grad);
    return 0;
}

int orc_leapfrog(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                 int n_z, double z_lo, double z_hi, const double *q, int sfh, double z, const double *obs,
                 const double *sigma, uint8_t mask, const double *bounds, const double *prior,
                 const double *gauss_prec, int n_step, double eps, double *x, double *p, double *logp) {
    if (!x || !p || !logp || n_step < 0) return 1;
    if (!gauss_prec && (!check_common(s, f) || !q || !bounds || !prior)) return 1;
    Model *X = gauss_prec ? nullptr : new Model(s, f, c, m);
    auto eval = [&](const double *xx, double *lp, double *gr) {
        if (gauss_prec) {
            double v = 0.0;
            for (int a = 0; a < NP; ++a) {
                double ax = 0.0;
                for (int b = 0; b < NP; ++b) ax += gauss_prec[a * NP + b] * xx[b];
                gr[a] = -ax;
                v += -0.5 * xx[a] * ax;
            }
            *lp = v;
        } else {
            logpost(*X, 0, n_z, z_lo, z_hi, q, sfh, xx, z, obs, sigma, mask, bounds, prior, lp, gr);
        }
    };
    double gr[NP], lp;
    eval(x, &lp, gr);
    for (int l = 0; l < n_step; ++l) {
        for (int k = 0; k < NP; ++k) p[k] += 0.5 * eps * gr[k];
        for (int k = 0; k < NP; ++k) x[k] += eps * p[k];
        eval(x, &lp, gr);
        for (int k = 0; k < NP; ++k) p[k] += 0.5 * eps * gr[k];
    }
    *logp = lp;
    delete X;
    return 0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) { philox(ctr, key, out); }

int orc_gauss_legendre(int n, double *x, double *w) {
    if (n < 1 || n > 16 || !x || !w) return 1;
    GaussLegendre g(n);
    for (int i = 0; i < n; ++i) { x[i] = g.x[i]; w[i] = g.w[i]; }
    return 0;
}

int orc_hmc_windows(int n_warmup, int max_win, int *start, int *end) {
    return hmc_windows(n_warmup, max_win, start, end);
}

double orc_rhat(int n_chain, int n, const double *x) {
    // classic Gelman-Rubin: V = (n-1)/n W + B/n, R = sqrt(V / W)
    std::vector<double> mean(n_chain, 0.0), var(n_chain, 0.0);
    for (int c = 0; c < n_chain; ++c) {
        for (int t = 0; t < n; ++t) mean[c] += x[(size_t)c * n + t];
        mean[c] /= n;
        for (int t = 0; t < n; ++t) { double d = x[(size_t)c * n + t] - mean[c]; var[c] += d * d; }
        var[c] /= (n - 1);
    }
    double W = 0.0, gm = 0.0, B = 0.0;
    for (int c = 0; c < n_chain; ++c) { W += var[c]; gm += mean[c]; }
    W /= n_chain;
    gm /= n_chain;
    for (int c = 0; c < n_chain; ++c) B += (mean[c] - gm) * (mean[c] - gm);
    B = B * n / (n_chain - 1);
    double V = (n - 1.0) / n * W + B / n;
    return std::sqrt(V / W);
}

void orc_hmc_prior_draw(const double *prior, uint64_t seed, uint32_t chain_id, double *x) {
    // A skew-normal variate (App. C, Eq. SkewNormPrior) from two independent standard normals
    // U0, U1 by the half-normal representation: Z = delta |U0| + sqrt(1 - delta^2) U1 with
    // delta = s / sqrt(1 + s^2) is SN(0, 1, s), and x = xi + omega Z.  (U0, U1) of parameter p
    // is the Box-Muller pair of uniforms 2p, 2p + 1 of the Philox blocks (blk, 0, chain id, 1),
    // blk = 0..4.
    const uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t w[20];
    for (int blk = 0; blk < 5; ++blk) {
        const uint32_t ctr[4] = {(uint32_t)blk, 0u, chain_id, 1u};
        philox(ctr, key, w + 4 * blk);
    }
    for (int p = 0; p < NP; ++p) {
        const double r = std::sqrt(-2.0 * std::log(u01(w[2 * p]))), a = 2.0 * PI * u01(w[2 * p + 1]);
        const double u0 = r * std::cos(a), u1 = r * std::sin(a);
        const double sk = prior[3 * p + 2], delta = sk / std::sqrt(1.0 + sk * sk);
        x[p] = prior[3 * p] + prior[3 * p + 1] * (delta * std::fabs(u0) + std::sqrt(1.0 - delta * delta) * u1);
    }
}

int orc_hmc_run(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                int n_z, double z_lo, double z_hi, const double *q, int sfh, const orc_hmc_cfg *cfg,
                int n_gal, const double *z, const double *obs, const double *sigma, const uint8_t *mask,
                const double *bounds, const double *prior, const double *theta0, const double *gauss_prec,
                double *post_mean, double *post_sd, double *rhat, double *accept, double *step,
                double *samples, double *trace_logp, int n_gal_total, const uint32_t *gal_id,
                double *inv_metric, double *trace_acc, double *state) {
    if (!cfg || cfg->n_chain < 1 || cfg->n_leapfrog < 1 || cfg->n_warmup < 0 || cfg->n_sample < 2) return 1;
    if (n_gal < 0) return 1;
    if (cfg->path != 0 && cfg->path != 1) return 1;
    if (!gauss_prec && (!check_common(s, f) || (cfg->path == 0 && !q) || !z || !obs || !sigma || !mask || !bounds ||
                        !prior))
        return 1;
    const int C = cfg->n_chain, L = cfg->n_leapfrog, NW = cfg->n_warmup, NS = cfg->n_sample;
    const int NIT = NW + NS;
    // iterations [it0, it1) of this call; a run split over calls carries every chain's state in
    // `state` ([chain][galaxy][ORC_HMC_STATE]) from one call to the next
    const int it0 = cfg->it_begin, it1 = cfg->it_end > 0 ? cfg->it_end : NIT;
    if (it0 < 0 || it1 > NIT || it0 >= it1 || ((it0 > 0 || it1 < NIT) && !state)) return 1;
    if (it0 == 0 && !theta0 && !prior) return 1;
    const int nb = f ? f->n_band : 0;
    Model *X = gauss_prec ? nullptr : new Model(s, f, c, m);
    std::vector<double> local;
    if (!state) {
        local.assign((size_t)C * n_gal * ORC_HMC_STATE, 0.0);
        state = local.data();
    }
    const uint32_t key[2] = {(uint32_t)(cfg->seed & 0xffffffffu), (uint32_t)(cfg->seed >> 32)};
    // dual-averaging constants (Hoffman & Gelman 2014, step-size adaptation)
    const double gamma = 0.05, t0 = 10.0, kappa = 0.75, delta = cfg->target_accept;
    int w_start[64], w_end[64];
    const int n_win = cfg->adapt_metric ? std::min(hmc_windows(NW, 64, w_start, w_end), 64) : 0;

#pragma omp parallel for schedule(dynamic, 1)
    for (long cg = 0; cg < (long)C * n_gal; ++cg) {
        const int ch = (int)(cg / n_gal), g = (int)(cg % n_gal);
        // Philox chain id = chain * (batch size) + galaxy index in the batch; a subset of a
        // larger batch passes the batch size and its galaxies' indices to reproduce its streams
        const uint32_t chain_id = gal_id ? (uint32_t)ch * (uint32_t)n_gal_total + gal_id[g] : (uint32_t)cg;
        auto eval = [&](const double *x, double *lp, double *gr) {
            if (gauss_prec) {
                double v = 0.0;
                for (int a = 0; a < NP; ++a) {
                    double ax = 0.0;
                    for (int b = 0; b < NP; ++b) ax += gauss_prec[a * NP + b] * x[b];
                    gr[a] = -ax;
                    v += -0.5 * x[a] * ax;
                }
                *lp = v;
            } else {
                logpost(*X, cfg->path, n_z, z_lo, z_hi, q, sfh, x, z[g], obs + (size_t)g * nb, sigma + (size_t)g * nb,
                        mask[g], bounds, prior, lp, gr);
            }
        };
        auto physical = [&](int p, double x) { return gauss_prec ? x : bound<double>(bounds + 4 * p, x); };
        // the chain's state, unpacked from / packed into its ORC_HMC_STATE doubles (layout in the header)
        double *S = state + (size_t)cg * ORC_HMC_STATE;
        double *x = S + 0, *gr = S + 10, *minv = S + 30, *wmu = S + 40, *wm2 = S + 50, *mean = S + 60, *m2 = S + 70;
        double(*Mi)[NP] = (double(*)[NP])(S + 100), (*Lc)[NP] = (double(*)[NP])(S + 200);
        double(*wcm)[NP] = (double(*)[NP])(S + 300);
        if (it0 == 0) {
            std::fill(S, S + ORC_HMC_STATE, 0.0);
            if (theta0) {
                for (int p = 0; p < NP; ++p) x[p] = theta0[(size_t)cg * NP + p];
            } else {
                orc_hmc_prior_draw(prior, cfg->seed, chain_id, x);
            }
            eval(x, &S[20], gr);
            S[21] = cfg->init_step;                       // eps
            S[22] = std::log(10.0 * cfg->init_step);      // mu
            // diagonal inverse mass matrix M^-1 (identity unless adapted); dense M^-1 = Lc Lc^T
            for (int k = 0; k < NP; ++k) minv[k] = Mi[k][k] = Lc[k][k] = 1.0;
        }
        double lp = S[20], eps = S[21], mu = S[22], hbar = S[23], leps_bar = S[24];
        int da_start = (int)S[25];   // iteration at which dual averaging last (re)started
        int win = (int)S[26], n_rec = (int)S[27], n_acc = (int)S[28];
        const bool dense = cfg->adapt_metric == 2;
        for (int it = it0; it < it1; ++it) {
            uint32_t w[12];
            for (int blk = 0; blk < 3; ++blk) {
                uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)it, chain_id, 0u};
                philox(ctr, key, w + 4 * blk);
            }
            // momentum p ~ N(0, M): standard normals (Box-Muller pairs) scaled by M^1/2
            double p[NP];
            for (int k = 0; k < NP / 2; ++k) {
                double r = std::sqrt(-2.0 * std::log(u01(w[2 * k]))), a = 2.0 * PI * u01(w[2 * k + 1]);
                p[2 * k] = r * std::cos(a) / std::sqrt(minv[2 * k]);
                p[2 * k + 1] = r * std::sin(a) / std::sqrt(minv[2 * k + 1]);
            }
            if (dense) {  // p = Lc^-T z solves Lc^T p = z, so that p^T Mi p = |z|^2
                double zv[NP];
                for (int k = 0; k < NP; ++k) zv[k] = p[k] * std::sqrt(minv[k]);
                for (int k = NP - 1; k >= 0; --k) {
                    double v = zv[k];
                    for (int j = k + 1; j < NP; ++j) v -= Lc[j][k] * p[j];
                    p[k] = v / Lc[k][k];
                }
            }
            auto kinetic = [&](const double *qv) {
                double e = 0.0;
                if (dense) {
                    for (int i = 0; i < NP; ++i)
                        for (int j = 0; j < NP; ++j) e += 0.5 * qv[i] * Mi[i][j] * qv[j];
                } else {
                    for (int k = 0; k < NP; ++k) e += 0.5 * minv[k] * qv[k] * qv[k];
                }
                return e;
            };
            // H = -log p(x) + p^T M^-1 p / 2
            double H0 = -lp + kinetic(p);
            double xn[NP], pn[NP], grn[NP], lpn = lp;
            for (int k = 0; k < NP; ++k) { xn[k] = x[k]; pn[k] = p[k]; grn[k] = gr[k]; }
            for (int l = 0; l < L; ++l) {  // leapfrog: half kick, drift by M^-1 p, half kick
                for (int k = 0; k < NP; ++k) pn[k] += 0.5 * eps * grn[k];
                if (dense) {
                    for (int i = 0; i < NP; ++i) {
                        double v = 0.0;
                        for (int j = 0; j < NP; ++j) v += Mi[i][j] * pn[j];
                        xn[i] += eps * v;
                    }
                } else {
                    for (int k = 0; k < NP; ++k) xn[k] += eps * minv[k] * pn[k];
                }
                eval(xn, &lpn, grn);
                for (int k = 0; k < NP; ++k) pn[k] += 0.5 * eps * grn[k];
            }
            double H1 = -lpn + kinetic(pn);
            double dH = H1 - H0;
            bool divergent = !std::isfinite(H1) || dH > 1000.0;
            double alpha = divergent ? 0.0 : std::min(1.0, std::exp(-dH));
            const double log_u = std::log(u01(w[10]));
            bool acc = !divergent && log_u < -dH;
            if (trace_acc) {
                double *t = trace_acc + (((size_t)it * C + ch) * n_gal + g) * 3;
                t[0] = alpha;
                t[1] = log_u + dH;   // accepted iff negative (and not divergent)
                t[2] = eps;
            }
            if (acc) {
                for (int k = 0; k < NP; ++k) { x[k] = xn[k]; gr[k] = grn[k]; }
                lp = lpn;
            }
            if (it < NW) {
                double mm = it - da_start + 1.0, eta = 1.0 / (mm + t0);
                hbar = (1.0 - eta) * hbar + eta * (delta - alpha);
                double leps = mu - std::sqrt(mm) / gamma * hbar, wk = std::pow(mm, -kappa);
                leps_bar = wk * leps + (1.0 - wk) * leps_bar;
                eps = std::exp(it == NW - 1 ? leps_bar : leps);
                if (win < n_win && it >= w_start[win]) {
                    // slow window: accumulate x; at its end, set M^-1 to the regularised
                    // sample variance and restart dual averaging from the current step
                    const double nn = it - w_start[win] + 1.0;
                    double d[NP];
                    for (int k = 0; k < NP; ++k) {
                        d[k] = x[k] - wmu[k];
                        wmu[k] += d[k] / nn;
                        wm2[k] += d[k] * (x[k] - wmu[k]);
                    }
                    if (dense)
                        for (int i = 0; i < NP; ++i)
                            for (int j = 0; j < NP; ++j) wcm[i][j] += d[i] * (x[j] - wmu[j]);
                    if (it == w_end[win] - 1) {
                        for (int k = 0; k < NP; ++k) {
                            minv[k] = nn / (nn + 5.0) * (wm2[k] / (nn - 1.0)) + 1e-3 * 5.0 / (nn + 5.0);
                            wmu[k] = wm2[k] = 0.0;
                        }
                        if (dense) {
                            // regularised sample covariance and its Cholesky factor
                            for (int i = 0; i < NP; ++i)
                                for (int j = 0; j < NP; ++j) {
                                    Mi[i][j] = nn / (nn + 5.0) * (wcm[i][j] / (nn - 1.0)) +
                                               (i == j ? 1e-3 * 5.0 / (nn + 5.0) : 0.0);
                                    wcm[i][j] = 0.0;
                                }
                            for (int j = 0; j < NP; ++j) {
                                double v = Mi[j][j];
                                for (int k = 0; k < j; ++k) v -= Lc[j][k] * Lc[j][k];
                                Lc[j][j] = std::sqrt(v);
                                for (int i = j + 1; i < NP; ++i) {
                                    double u = Mi[i][j];
                                    for (int k = 0; k < j; ++k) u -= Lc[i][k] * Lc[j][k];
                                    Lc[i][j] = u / Lc[j][j];
                                }
                            }
                            // the momentum scaling above then uses unit variances
                            for (int k = 0; k < NP; ++k) minv[k] = 1.0;
                        }
                        mu = std::log(10.0 * eps);
                        hbar = leps_bar = 0.0;
                        da_start = it + 1;
                        ++win;
                    }
                }
            } else {
                n_acc += acc;
                ++n_rec;
                for (int k = 0; k < NP; ++k) {
                    double th = physical(k, x[k]), d = th - mean[k];
                    mean[k] += d / n_rec;
                    m2[k] += d * (th - mean[k]);
                    if (samples) samples[(((size_t)(it - NW) * C + ch) * n_gal + g) * NP + k] = th;
                }
            }
            if (trace_logp) trace_logp[((size_t)it * C + ch) * n_gal + g] = lp;
        }
        S[20] = lp;
        S[21] = eps;
        S[22] = mu;
        S[23] = hbar;
        S[24] = leps_bar;
        S[25] = da_start;
        S[26] = win;
        S[27] = n_rec;
        S[28] = n_acc;
        if (inv_metric)
            for (int k = 0; k < NP; ++k) inv_metric[(size_t)cg * NP + k] = dense ? Mi[k][k] : minv[k];
        if (step) step[cg] = eps;
    }
    delete X;
    if (it1 < NIT) return 0;   // summaries once the run is complete
    for (int g = 0; g < n_gal; ++g) {
        int acc = 0;
        for (int ch = 0; ch < C; ++ch) acc += (int)state[((size_t)ch * n_gal + g) * ORC_HMC_STATE + 28];
        if (accept) accept[g] = (double)acc / ((double)C * NS);
        for (int k = 0; k < NP; ++k) {
            double gm = 0.0, W = 0.0, B = 0.0, ss = 0.0;
            auto cmean = [&](int ch) { return state[((size_t)ch * n_gal + g) * ORC_HMC_STATE + 60 + k]; };
            auto cm2 = [&](int ch) { return state[((size_t)ch * n_gal + g) * ORC_HMC_STATE + 70 + k]; };
            for (int ch = 0; ch < C; ++ch) {
                gm += cmean(ch);
                W += cm2(ch) / (NS - 1);
            }
            gm /= C;
            W /= C;
            for (int ch = 0; ch < C; ++ch) {
                B += (cmean(ch) - gm) * (cmean(ch) - gm);
                ss += cm2(ch) + NS * (cmean(ch) - gm) * (cmean(ch) - gm);
            }
            double Bn = (C > 1) ? B / (C - 1) : 0.0;  // = B/n in the usual notation
            double V = (NS - 1.0) / NS * W + Bn;
            if (post_mean) post_mean[(size_t)g * NP + k] = gm;
            if (post_sd) post_sd[(size_t)g * NP + k] = std::sqrt(ss / ((double)C * NS - 1.0));
            if (rhat) rhat[(size_t)g * NP + k] = (C > 1) ? std::sqrt(V / W) : NaN;
        }
    }
    return 0;
}

// ---- No-U-Turn Sampler (the paper's second gradient-based sampler, App. D.2; Sec. 4 runs it
// beside HMC).  Hoffman & Gelman (2014), Algorithm 3 (the "efficient" NUTS: slice variable,
// doubling in a random direction, a subtree's proposal taken with probability
// min(1, n'/n)) with the dual averaging of their Algorithm 6 (acceptance statistic = mean of
// min(1, exp(H0 - H)) over the leaves of the final tree).  The recursion of BuildTree is
// unrolled leaf by leaf, which builds the same leaves and makes the same U-turn checks in the
// same order: after the last leaf of every dyadic block of a subtree (innermost first), the
// block's ends are tested, and a divergent leaf ends the subtree at once.  Inside a subtree
// the proposal is a uniform choice among its valid leaves (reservoir sampling), the
// distribution the recursion's pairwise choices give.  Diagonal metric: the U-turn test uses
// the velocities M^-1 p.  Philox draws: momentum and slice (blk 0..2, it, chain, 0: words 0..9
// momentum as in HMC, word 10 the slice uniform), per doubling j (j, it, chain, 2: word 0 the
// direction, word 1 the subtree's acceptance), per leaf (leaf index in the iteration, it,
// chain, 3: word 0 the reservoir uniform).
int orc_nuts_run(const orc_ssp *s, const orc_filters *f, const orc_cosmo *c, const orc_model *m,
                 int n_z, double z_lo, double z_hi, const double *q, int sfh, const orc_nuts_cfg *cfg,
                 int n_gal, const double *z, const double *obs, const double *sigma, const uint8_t *mask,
                 const double *bounds, const double *prior, const double *theta0, const double *gauss_prec,
                 double *post_mean, double *post_sd, double *rhat, double *accept, double *step,
                 double *samples, int *trace_depth, int *trace_steps, double *trace_margin, double *inv_metric,
                 int n_gal_total, const uint32_t *gal_id) {
    if (!cfg || cfg->n_chain < 1 || cfg->max_depth < 1 || cfg->max_depth > 12 || cfg->n_warmup < 0 ||
        cfg->n_sample < 2 || n_gal < 0)
        return 1;
    if (cfg->path != 0 && cfg->path != 1) return 1;
    if (cfg->adapt_metric != 0 && cfg->adapt_metric != 1) return 1;
    if (!gauss_prec && (!check_common(s, f) || (cfg->path == 0 && !q) || !z || !obs || !sigma || !mask || !bounds ||
                        !prior))
        return 1;
    if (!theta0 && !prior) return 1;
    const int C = cfg->n_chain, NW = cfg->n_warmup, NS = cfg->n_sample, NIT = NW + NS, D = cfg->max_depth;
    const int nb = f ? f->n_band : 0;
    const double DELTA_MAX = 1000.0;
    Model *X = gauss_prec ? nullptr : new Model(s, f, c, m);
    std::vector<double> cmean((size_t)C * n_gal * NP, 0.0), cm2((size_t)C * n_gal * NP, 0.0), cacc((size_t)C * n_gal);
    const uint32_t key[2] = {(uint32_t)(cfg->seed & 0xffffffffu), (uint32_t)(cfg->seed >> 32)};
    const double gamma = 0.05, t0 = 10.0, kappa = 0.75, delta = cfg->target_accept;
    int w_start[64], w_end[64];
    const int n_win = cfg->adapt_metric ? std::min(hmc_windows(NW, 64, w_start, w_end), 64) : 0;

#pragma omp parallel for schedule(dynamic, 1)
    for (long cg = 0; cg < (long)C * n_gal; ++cg) {
        const int ch = (int)(cg / n_gal), g = (int)(cg % n_gal);
        const uint32_t chain_id = gal_id ? (uint32_t)ch * (uint32_t)n_gal_total + gal_id[g] : (uint32_t)cg;
        auto eval = [&](const double *x, double *lp, double *gr) {
            if (gauss_prec) {
                double v = 0.0;
                for (int a = 0; a < NP; ++a) {
                    double ax = 0.0;
                    for (int b = 0; b < NP; ++b) ax += gauss_prec[a * NP + b] * x[b];
                    gr[a] = -ax;
                    v += -0.5 * x[a] * ax;
                }
                *lp = v;
            } else {
                logpost(*X, cfg->path, n_z, z_lo, z_hi, q, sfh, x, z[g], obs + (size_t)g * nb, sigma + (size_t)g * nb,
                        mask[g], bounds, prior, lp, gr);
            }
        };
        auto physical = [&](int p, double x) { return gauss_prec ? x : bound<double>(bounds + 4 * p, x); };
        double x[NP], gr[NP], lp, minv[NP], wmu[NP] = {0.0}, wm2[NP] = {0.0};
        if (theta0) {
            for (int p = 0; p < NP; ++p) x[p] = theta0[(size_t)cg * NP + p];
        } else {
            orc_hmc_prior_draw(prior, cfg->seed, chain_id, x);
        }
        eval(x, &lp, gr);
        for (int k = 0; k < NP; ++k) minv[k] = 1.0;
        double eps = cfg->init_step, mu = std::log(10.0 * cfg->init_step), hbar = 0.0, leps_bar = 0.0, acc_sum = 0.0;
        int da_start = 0, win = 0, n_rec = 0;
        double *mean = &cmean[(size_t)cg * NP], *m2 = &cm2[(size_t)cg * NP];
        auto kinetic = [&](const double *pv) {
            double e = 0.0;
            for (int k = 0; k < NP; ++k) e += 0.5 * minv[k] * pv[k] * pv[k];
            return e;
        };
        // smallest distance of this iteration's decisions from their thresholds (trace only):
        // |log u + H| over the leaves, and the cosine of the angle between the stretch and the
        // velocity at its ends over the U-turn tests
        double mg_slice = INFINITY, mg_turn = INFINITY;
        // no U-turn between the forward-time ends of a stretch: (x+ - x-) . M^-1 p >= 0 at both
        auto no_uturn = [&](const double *xa, const double *pa, const double *xb, const double *pb, int dirn) {
            double da = 0.0, db = 0.0, dd = 0.0, va = 0.0, vb = 0.0;
            for (int k = 0; k < NP; ++k) {
                const double dx = dirn * (xb[k] - xa[k]);
                da += dx * minv[k] * pa[k];
                db += dx * minv[k] * pb[k];
                dd += dx * dx;
                va += minv[k] * pa[k] * minv[k] * pa[k];
                vb += minv[k] * pb[k] * minv[k] * pb[k];
            }
            if (dd > 0.0 && va > 0.0 && vb > 0.0)
                mg_turn = std::min(mg_turn, std::min(std::fabs(da) / std::sqrt(dd * va), std::fabs(db) / std::sqrt(dd * vb)));
            return da >= 0.0 && db >= 0.0;
        };
        for (int it = 0; it < NIT; ++it) {
            uint32_t w[12];
            for (int blk = 0; blk < 3; ++blk) {
                const uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)it, chain_id, 0u};
                philox(ctr, key, w + 4 * blk);
            }
            double p0[NP];
            for (int k = 0; k < NP / 2; ++k) {
                const double r = std::sqrt(-2.0 * std::log(u01(w[2 * k]))), a = 2.0 * PI * u01(w[2 * k + 1]);
                p0[2 * k] = r * std::cos(a) / std::sqrt(minv[2 * k]);
                p0[2 * k + 1] = r * std::sin(a) / std::sqrt(minv[2 * k + 1]);
            }
            const double H0 = -lp + kinetic(p0);
            const double log_u = std::log(u01(w[10])) - H0;   // slice variable u ~ U(0, exp(-H0))
            mg_slice = mg_turn = INFINITY;
            // the tree's two ends, the proposal
            double xl[NP], pl[NP], gl[NP], xr[NP], pr[NP], grr[NP], xm[NP], gm[NP], lpl = lp, lpr = lp, lpm = lp;
            for (int k = 0; k < NP; ++k) {
                xl[k] = xr[k] = xm[k] = x[k];
                pl[k] = pr[k] = p0[k];
                gl[k] = grr[k] = gm[k] = gr[k];
            }
            long n = 1;
            bool s_tree = true;
            int j = 0, leaf = 0;
            double alpha_sum = 0.0;
            while (s_tree && j < D) {
                uint32_t wj[4];
                const uint32_t cj[4] = {(uint32_t)j, (uint32_t)it, chain_id, 2u};
                philox(cj, key, wj);
                const int dirn = u01(wj[0]) < 0.5 ? -1 : 1;
                // the subtree of 2^j leaves grows from the end in direction dirn
                double xe[NP], pe[NP], ge[NP], lpe;
                for (int k = 0; k < NP; ++k) {
                    xe[k] = dirn < 0 ? xl[k] : xr[k];
                    pe[k] = dirn < 0 ? pl[k] : pr[k];
                    ge[k] = dirn < 0 ? gl[k] : grr[k];
                }
                lpe = dirn < 0 ? lpl : lpr;
                double xs[NP] = {0.0}, gs[NP] = {0.0}, lps = 0.0, ckx[13][NP], ckp[13][NP];
                long n_sub = 0;
                bool s_sub = true;
                const long n_leaf = 1L << j;
                for (long k = 0; k < n_leaf && s_sub; ++k) {
                    // one leapfrog step of size dirn * eps
                    const double e = dirn * eps;
                    for (int t = 0; t < NP; ++t) pe[t] += 0.5 * e * ge[t];
                    for (int t = 0; t < NP; ++t) xe[t] += e * minv[t] * pe[t];
                    eval(xe, &lpe, ge);
                    for (int t = 0; t < NP; ++t) pe[t] += 0.5 * e * ge[t];
                    const double H = -lpe + kinetic(pe);
                    alpha_sum += std::isfinite(H) ? std::min(1.0, std::exp(H0 - H)) : 0.0;
                    if (std::isfinite(H)) mg_slice = std::min(mg_slice, std::fabs(log_u + H));
                    ++leaf;
                    if (log_u <= -H) {   // the leaf lies in the slice: a valid proposal
                        ++n_sub;
                        uint32_t wl[4];
                        const uint32_t cl[4] = {(uint32_t)(leaf - 1), (uint32_t)it, chain_id, 3u};
                        philox(cl, key, wl);
                        if (u01(wl[0]) * n_sub < 1.0) {   // probability 1 / n_sub
                            for (int t = 0; t < NP; ++t) { xs[t] = xe[t]; gs[t] = ge[t]; }
                            lps = lpe;
                        }
                    }
                    if (!(log_u < DELTA_MAX - H)) s_sub = false;   // divergence (or a non-finite H)
                    // the first leaf of every dyadic block that starts here
                    for (int l = 1; l <= j; ++l)
                        if (k % (1L << l) == 0)
                            for (int t = 0; t < NP; ++t) { ckx[l][t] = xe[t]; ckp[l][t] = pe[t]; }
                    // every block that ends here (innermost first): its ends must not have turned
                    for (int l = 1; l <= j && s_sub; ++l)
                        if ((k + 1) % (1L << l) == 0 && !no_uturn(ckx[l], ckp[l], xe, pe, dirn)) s_sub = false;
                }
                for (int k = 0; k < NP; ++k) {
                    if (dirn < 0) { xl[k] = xe[k]; pl[k] = pe[k]; gl[k] = ge[k]; }
                    else { xr[k] = xe[k]; pr[k] = pe[k]; grr[k] = ge[k]; }
                }
                if (dirn < 0) lpl = lpe; else lpr = lpe;
                if (s_sub && n_sub > 0 && u01(wj[1]) * n < n_sub) {   // probability min(1, n_sub / n)
                    for (int k = 0; k < NP; ++k) { xm[k] = xs[k]; gm[k] = gs[k]; }
                    lpm = lps;
                }
                n += n_sub;
                s_tree = s_sub && no_uturn(xl, pl, xr, pr, 1);
                ++j;
            }
            for (int k = 0; k < NP; ++k) { x[k] = xm[k]; gr[k] = gm[k]; }
            lp = lpm;
            const double alpha = alpha_sum / leaf;
            if (trace_depth) trace_depth[((size_t)it * C + ch) * n_gal + g] = j;
            if (trace_steps) trace_steps[((size_t)it * C + ch) * n_gal + g] = leaf;
            if (trace_margin) {
                trace_margin[(((size_t)it * C + ch) * n_gal + g) * 2] = mg_slice;
                trace_margin[(((size_t)it * C + ch) * n_gal + g) * 2 + 1] = mg_turn;
            }
            if (it < NW) {
                const double mm = it - da_start + 1.0, eta = 1.0 / (mm + t0);
                hbar = (1.0 - eta) * hbar + eta * (delta - alpha);
                const double leps = mu - std::sqrt(mm) / gamma * hbar, wk = std::pow(mm, -kappa);
                leps_bar = wk * leps + (1.0 - wk) * leps_bar;
                eps = std::exp(it == NW - 1 ? leps_bar : leps);
                if (win < n_win && it >= w_start[win]) {
                    const double nn = it - w_start[win] + 1.0;
                    for (int k = 0; k < NP; ++k) {
                        const double d = x[k] - wmu[k];
                        wmu[k] += d / nn;
                        wm2[k] += d * (x[k] - wmu[k]);
                    }
                    if (it == w_end[win] - 1) {
                        for (int k = 0; k < NP; ++k) {
                            minv[k] = nn / (nn + 5.0) * (wm2[k] / (nn - 1.0)) + 1e-3 * 5.0 / (nn + 5.0);
                            wmu[k] = wm2[k] = 0.0;
                        }
                        mu = std::log(10.0 * eps);
                        hbar = leps_bar = 0.0;
                        da_start = it + 1;
                        ++win;
                    }
                }
            } else {
                acc_sum += alpha;
                ++n_rec;
                for (int k = 0; k < NP; ++k) {
                    const double th = physical(k, x[k]), d = th - mean[k];
                    mean[k] += d / n_rec;
                    m2[k] += d * (th - mean[k]);
                    if (samples) samples[(((size_t)(it - NW) * C + ch) * n_gal + g) * NP + k] = th;
                }
            }
        }
        if (inv_metric)
            for (int k = 0; k < NP; ++k) inv_metric[(size_t)cg * NP + k] = minv[k];
        cacc[cg] = acc_sum;
        if (step) step[cg] = eps;
    }
    delete X;
    for (int g = 0; g < n_gal; ++g) {
        double acc = 0.0;
        for (int ch = 0; ch < C; ++ch) acc += cacc[(size_t)ch * n_gal + g];
        if (accept) accept[g] = acc / ((double)C * NS);
        for (int k = 0; k < NP; ++k) {
            double gm = 0.0, W = 0.0, B = 0.0, ss = 0.0;
            for (int ch = 0; ch < C; ++ch) {
                const size_t o = ((size_t)ch * n_gal + g) * NP + k;
                gm += cmean[o];
                W += cm2[o] / (NS - 1);
            }
            gm /= C;
            W /= C;
            for (int ch = 0; ch < C; ++ch) {
                const size_t o = ((size_t)ch * n_gal + g) * NP + k;
                B += (cmean[o] - gm) * (cmean[o] - gm);
                ss += cm2[o] + NS * (cmean[o] - gm) * (cmean[o] - gm);
            }
            const double Bn = (C > 1) ? B / (C - 1) : 0.0;
            const double V = (NS - 1.0) / NS * W + Bn;
            if (post_mean) post_mean[(size_t)g * NP + k] = gm;
            if (post_sd) post_sd[(size_t)g * NP + k] = std::sqrt(ss / ((double)C * NS - 1.0));
            if (rhat) rhat[(size_t)g * NP + k] = (C > 1) ? std::sqrt(V / W) : NaN;
        }
    }
    return 0;
}

}  // extern "C"
