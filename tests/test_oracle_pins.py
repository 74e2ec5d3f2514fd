"""Pins of the FP64 oracle against things the paper and mathematics fix.

Nothing here re-types an oracle formula and compares it with itself: every
expected value is a closed form, a special case that reduces to a library
routine, a published test vector, a brute-force sum with a different method,
or an invariant.  CPU only.
"""
import math
import os

import numpy as np
import pytest
from scipy import integrate, special, stats

import synth

C_KMS = 299792.458
MPC_KM = 3.0856775814913673e19
GYR_S = 3.15576e16


def h0_per_gyr(h0=70.0):
    return h0 / MPC_KM * GYR_S


# --------------------------------------------------------------------------
# cosmology (reading: flat LCDM, matter + Lambda)
# --------------------------------------------------------------------------
def test_age_universe_lcdm_closed_form(orc):
    # t(z) = 2/(3 H0 sqrt(OL)) asinh(sqrt(OL/Om) (1+z)^-1.5) for flat matter+Lambda
    H, om = h0_per_gyr(), 0.3
    ol = 1 - om
    for z in (0.0, 0.1, 0.5, 1.0, 2.0, 3.0, 7.0):
        ref = 2 / (3 * H * math.sqrt(ol)) * math.asinh(math.sqrt(ol / om) * (1 + z) ** -1.5)
        assert orc.age_universe(z) == pytest.approx(ref, rel=1e-12)


def test_einstein_de_sitter_special_case(oracle_mod, ssp_small, filt6):
    # Om = 1: t = 2/(3 H0) (1+z)^-1.5,  D_L = (2c/H0)(1+z)(1 - (1+z)^-1/2)
    o = oracle_mod.Oracle(ssp_small, filt6, cosmo=dict(Om=1.0))
    H = h0_per_gyr()
    for z in (0.1, 1.0, 3.0):
        assert o.age_universe(z) == pytest.approx(2 / (3 * H) * (1 + z) ** -1.5, rel=1e-12)
        dl = 2 * C_KMS / 70.0 * (1 + z) * (1 - (1 + z) ** -0.5)
        assert o.lum_distance(z) == pytest.approx(dl, rel=1e-12)


def test_luminosity_distance_low_z_expansion(orc):
    # D_L = (c z / H0) (1 + (1 - q0) z / 2 + O(z^2)),  q0 = Om/2 - OL
    q0 = 0.15 - 0.7
    for z in (1e-3, 3e-3):
        lead = C_KMS * z / 70.0 * (1 + 0.5 * (1 - q0) * z)
        assert orc.lum_distance(z) == pytest.approx(lead, rel=5 * z * z)


# --------------------------------------------------------------------------
# star-formation history -> smooth age-bin masses
# --------------------------------------------------------------------------
def _age_edges_gyr(ssp):
    la = ssp["log10_age_yr"]
    mid = 0.5 * (la[1:] + la[:-1])
    return np.concatenate([[0.0], 10 ** mid * 1e-9, [np.inf]])


def _bin_limits(ssp, t_obs):
    e = _age_edges_gyr(ssp)
    lo = np.minimum(e[:-1], t_obs)
    hi = np.minimum(e[1:], t_obs)
    return lo, hi  # stellar-age limits of each bin, clipped to t_obs


def _theta(**kw):
    th = np.zeros(10)
    th[0] = 10.0
    for k, v in kw.items():
        th[synth.PARAM_NAMES.index(k)] = v
    return th


@pytest.mark.parametrize("z", [0.1, 1.3, 3.0])
def test_constant_sfh_mass_proportional_to_bin_width(orc, ssp2000, z):
    # DPL with alpha = beta = 0 gives a constant rate 1/2: mass in each bin is half its
    # (clipped) duration, and the weights sum to exactly the mass formed.
    th = _theta(tau=3.0, alpha=0.0, beta=0.0, mu_logZ=-0.3)
    t_obs = orc.age_universe(z)
    lo, hi = _bin_limits(ssp2000, t_obs)
    m = orc.smooth_bin_mass(synth.SFH_DPL, th, z)
    np.testing.assert_allclose(m, 0.5 * (hi - lo), rtol=1e-12, atol=1e-300)
    w = orc.weights(synth.SFH_DPL, th[None, :], np.array([z]))[0]
    assert w.sum() == pytest.approx(10 ** th[0], rel=1e-12)
    # age marginal of the weights is proportional to the bin widths
    np.testing.assert_allclose(w.sum(axis=0) / w.sum(), (hi - lo) / t_obs, rtol=1e-11, atol=1e-300)


def _dpl_cumulative(t, tau, alpha, beta):
    """int_0^t dt' / ((t'/tau)^alpha + (t'/tau)^-beta) in closed form:
    tau * U^(b+1)/(b+1) * 2F1(1, a; 1+a; -U^s),  U = t/tau, s = alpha+beta, a = (b+1)/s."""
    u = np.asarray(t, float) / tau
    s = alpha + beta
    a = (beta + 1) / s
    return tau * u ** (beta + 1) / (beta + 1) * special.hyp2f1(1.0, a, 1.0 + a, -u ** s)


@pytest.mark.parametrize("tau,alpha,beta,z", [
    (3.0, 2.5, 1.5, 0.5), (1.0, 4.9, 0.6, 0.1), (12.0, 0.6, 4.5, 2.8), (0.5, 0.8, 0.3, 1.2),
    (6.0, 1.5, 7.5, 0.2)])
def test_dpl_bin_mass_hypergeometric_closed_form(orc, ssp2000, tau, alpha, beta, z):
    th = _theta(tau=tau, alpha=alpha, beta=beta)
    t_obs = orc.age_universe(z)
    lo, hi = _bin_limits(ssp2000, t_obs)
    ref = _dpl_cumulative(t_obs - lo, tau, alpha, beta) - _dpl_cumulative(t_obs - hi, tau, alpha, beta)
    m = orc.smooth_bin_mass(synth.SFH_DPL, th, z)
    live = hi > lo
    # the closed-form reference is a difference of two cumulatives, each a scipy hyp2f1 value
    # good to about 1e-15 relative: its error is a few 1e-15 of the total mass formed, which
    # bounds the absolute tolerance
    scale = _dpl_cumulative(t_obs, tau, alpha, beta)
    np.testing.assert_allclose(m[live], ref[live], rtol=1e-10, atol=4e-15 * scale)
    assert np.all(m[~live] == 0)


def test_dpl_cumulative_incomplete_beta(orc):
    # independent special-function route for alpha > 1: (tau/s) B(w; a, 1-a), w = U^s/(1+U^s)
    tau, alpha, beta, t = 2.0, 3.0, 1.2, 1.7
    s, a = alpha + beta, (beta + 1) / (alpha + beta)
    u = t / tau
    w = u ** s / (1 + u ** s)
    ref = tau / s * special.betainc(a, 1 - a, w) * special.beta(a, 1 - a)
    assert _dpl_cumulative(t, tau, alpha, beta) == pytest.approx(ref, rel=1e-12)


@pytest.mark.parametrize("tp,w,z", [(3.0, 0.4, 0.3), (11.0, 1.4, 0.1), (1.0, 0.2, 2.9)])
def test_lognormal_bin_mass_closed_form(orc, ssp2000, tp, w, z):
    # M(t) = t_p w sqrt(2 pi) e^{w^2/2} Phi((ln(t/t_p) - w^2)/w)
    th = _theta(tau=tp, alpha=w)
    t_obs = orc.age_universe(z)
    lo, hi = _bin_limits(ssp2000, t_obs)

    def cum_diff(t1, t0):  # M(t1) - M(t0), upper tail form when both are far right
        x1 = np.where(t1 > 0, (np.log(np.maximum(t1, 1e-300) / tp) - w * w) / w, -np.inf)
        x0 = np.where(t0 > 0, (np.log(np.maximum(t0, 1e-300) / tp) - w * w) / w, -np.inf)
        k = tp * w * math.sqrt(2 * math.pi) * math.exp(w * w / 2)
        return k * np.where(x0 > 0, special.ndtr(-x0) - special.ndtr(-x1), special.ndtr(x1) - special.ndtr(x0))

    ref = cum_diff(t_obs - lo, t_obs - hi)
    m = orc.smooth_bin_mass(synth.SFH_LOGNORMAL, th, z)
    live = ref > 1e-30 * ref.max()
    np.testing.assert_allclose(m[live], ref[live], rtol=1e-8)


def test_smooth_bin_mass_brute_force_midpoint(orc, ssp2000):
    # a different integration method (10^6-point midpoint sums) on a few bins
    th = _theta(tau=2.0, alpha=3.0, beta=0.4)
    z = 1.0
    t_obs = orc.age_universe(z)
    lo, hi = _bin_limits(ssp2000, t_obs)
    m = orc.smooth_bin_mass(synth.SFH_DPL, th, z)
    live = np.nonzero(hi > lo)[0]
    for i in [live[0], live[len(live) // 2], live[-2], live[-1]]:
        n = 1_000_000
        a = lo[i] + (hi[i] - lo[i]) * (np.arange(n) + 0.5) / n
        t = t_obs - a
        u = t / 2.0
        rate = 1.0 / (u ** 3.0 + u ** -0.4)
        assert rate.sum() * (hi[i] - lo[i]) / n == pytest.approx(m[i], rel=2e-6)


def test_age_weights_sum_to_one(orc):
    th, z = synth.galaxies_dpl(20, 7)
    for g in range(20):
        pa, ps, pb = orc.age_weights(synth.SFH_DPL, th[g], z[g])
        assert pa.sum() == pytest.approx(1, abs=1e-13)
        assert ps.sum() == pytest.approx(1, abs=1e-13)
        assert pb.sum() == pytest.approx(1, abs=1e-13)
        assert np.all(pa >= 0)


# --------------------------------------------------------------------------
# burst (triweight)
# --------------------------------------------------------------------------
def _triweight_cdf(x):
    # closed-form antiderivative: 1/2 + 35/32 (u - u^3 + 3u^5/5 - u^7/7), u = x/3 on |x| <= 3
    u = np.clip(np.asarray(x, float) / 3.0, -1, 1)
    return 0.5 + 35.0 / 32.0 * (u - u ** 3 + 3 * u ** 5 / 5 - u ** 7 / 7)


def test_triweight_cdf_is_a_distribution():
    # the closed form itself: integrates to 1, vanishes with zero slope at |x| = 3
    assert _triweight_cdf(3.0) - _triweight_cdf(-3.0) == pytest.approx(1, abs=1e-15)
    pdf = lambda x: 35 / 96 * (1 - (x / 3) ** 2) ** 3
    assert integrate.quad(pdf, -3, 3)[0] == pytest.approx(1, abs=1e-14)
    assert pdf(3.0) == 0 and abs((pdf(3.0) - pdf(3.0 - 1e-6)) / 1e-6) < 1e-10


@pytest.mark.parametrize("ltp", [5.0, 6.37, 7.5, 8.0])
def test_burst_weights_triweight_cdf(orc, ssp2000, ltp):
    th = _theta(tau=3, alpha=2, beta=2, F_burst=1.0, log10T_peak=ltp)
    z = 0.5
    _, _, pb = orc.age_weights(synth.SFH_DPL, th, z)
    la = ssp2000["log10_age_yr"]
    edges = np.concatenate([[-np.inf], 0.5 * (la[1:] + la[:-1]), [np.inf]])
    sig = 0.3 / 3.0
    ref = _triweight_cdf((edges[1:] - ltp) / sig) - _triweight_cdf((edges[:-1] - ltp) / sig)
    np.testing.assert_allclose(pb, ref, atol=1e-14)
    pa, _, _ = orc.age_weights(synth.SFH_DPL, th, z)
    np.testing.assert_allclose(pa, pb, atol=1e-15)  # F_burst = 1 -> pure burst


def test_burst_far_younger_than_grid_lands_in_youngest_bin(orc):
    th = _theta(tau=3, alpha=2, beta=2, F_burst=0.3, log10T_peak=4.0)
    pa, ps, pb = orc.age_weights(synth.SFH_DPL, th, 1.0)
    assert pb[0] == 1.0 and np.all(pb[1:] == 0)
    np.testing.assert_allclose(pa, 0.7 * ps + 0.3 * pb, rtol=1e-15, atol=1e-300)


def test_burst_mixture_linear_in_fburst(orc):
    base = _theta(tau=3, alpha=2, beta=2, log10T_peak=7.2)
    out = []
    for fb in (0.0, 0.05, 0.1):
        th = base.copy()
        th[4] = fb
        out.append(orc.age_weights(synth.SFH_DPL, th, 0.8)[0])
    np.testing.assert_allclose(out[1], 0.5 * (out[0] + out[2]), atol=1e-15)


# --------------------------------------------------------------------------
# metallicity and dust
# --------------------------------------------------------------------------
def test_met_weights_match_normal_cdf(orc, ssp2000):
    lz = ssp2000["log10_met"]
    edges = np.concatenate([[-np.inf], 0.5 * (lz[1:] + lz[:-1]), [np.inf]])
    for mu in (-1.5, -0.77, 0.0, 0.2):
        p = orc.met_weights(_theta(mu_logZ=mu))
        ref = np.diff(stats.norm.cdf(edges, loc=mu, scale=0.2))
        np.testing.assert_allclose(p, ref, atol=1e-15)
        assert p.sum() == pytest.approx(1, abs=1e-14)


def test_met_weights_delta_limit(oracle_mod, ssp_small, filt6):
    o = oracle_mod.Oracle(ssp_small, filt6, model=dict(sigma_logz=1e-4))
    lz = ssp_small["log10_met"]
    p = o.met_weights(_theta(mu_logZ=lz[5]))
    assert p[5] == pytest.approx(1, abs=1e-12)


def test_dust_special_cases(orc):
    th = _theta(tau_V=1.3, delta=-0.7, F_floor=0.2)
    assert orc.dust_att(th, 5500.0) == pytest.approx(0.2 + 0.8 * math.exp(-1.3), rel=1e-15)
    # A(lambda) = A_V (lambda/5500)^delta  with  10^(-0.4 A_V) = e^{-tau_V}
    av = 2.5 * math.log10(math.e) * 1.3
    assert orc.dust_att(th, 3000.0) == pytest.approx(
        0.2 + 0.8 * 10 ** (-0.4 * av * (3000 / 5500) ** -0.7), rel=1e-14)
    assert orc.dust_att(_theta(tau_V=0.0, delta=-1), 1234.0) == 1.0
    assert orc.dust_att(_theta(tau_V=2.0, F_floor=1.0), 1234.0) == 1.0
    g = _theta(tau_V=0.7, delta=0.0)
    assert orc.dust_att(g, 1000.0) == orc.dust_att(g, 9000.0)


def test_lambda_eff_of_gaussian_band_is_centre(orc, filt6):
    for b in range(6):
        assert orc.lambda_eff(b) == pytest.approx(filt6["center_A"][b], rel=1e-13)


# --------------------------------------------------------------------------
# photometry
# --------------------------------------------------------------------------
def test_flat_fnu_spectrum_gives_its_ab_magnitude(oracle_mod):
    # A source with flat f_nu = f0 has m_AB = -2.5 log10(f0 / 3631 Jy) through any filter.
    # Build SSPs whose rest-frame L_lambda reproduces flat f_nu at redshift z under the
    # Einstein-de Sitter cosmology (closed-form D_L).
    lsun, c_ang, mpc = 3.828e33, 2.99792458e18, 3.0856775814913673e24
    m0 = 22.0
    f0 = 3631e-23 * 10 ** (-0.4 * m0)
    wave = np.geomspace(100.0, 1e5, 3000)
    filt = dict(center_A=np.array([3000.0, 4500.0, 8000.0, 9500.0]),
                sigma_A=np.array([30.0, 400.0, 900.0, 200.0]))
    for z in (0.15, 1.1, 2.7):
        dl = 2 * C_KMS / 70.0 * (1 + z) * (1 - (1 + z) ** -0.5) * mpc
        th = _theta(tau=3, alpha=2, beta=2, mu_logZ=-0.5)
        mass = 10 ** th[0]
        lam_l = 4 * np.pi * dl ** 2 * (1 + z) * f0 * c_ang / ((1 + z) * wave) ** 2 / (lsun * mass)
        ssp = dict(log10_met=np.array([-1.0, 0.0]), log10_age_yr=np.array([7.0, 8.0, 9.0]),
                   wave_A=wave, lum=np.broadcast_to(lam_l, (2, 3, len(wave))).copy())
        o = oracle_mod.Oracle(ssp, filt, cosmo=dict(Om=1.0))
        m = o.phot_exact(synth.SFH_DPL, th[None, :], np.array([z]))
        np.testing.assert_allclose(m, m0, atol=1e-10)


def test_exact_photometry_matches_dense_quadrature(oracle_mod):
    # SSPs sharing one smooth continuous spectrum S(lambda) (so the composite SED is S for
    # any weights): the oracle's discrete rest-frame integral must match adaptive quadrature
    # of the continuous photon-counting AB definition, with dust, under the
    # Einstein-de Sitter distance (closed form).
    lsun, c_ang, mpc = 3.828e33, 2.99792458e18, 3.0856775814913673e24
    temp = 9000.0

    def spec(lam):  # unit-bolometric Planck curve per A
        x = 1.438777e8 / (lam * temp)
        return (15.0 / np.pi ** 4) * x ** 4 / (lam * np.expm1(x))

    wave = np.geomspace(100.0, 1e5, 4000)
    ssp = dict(log10_met=np.array([-1.0, 0.0]), log10_age_yr=np.array([7.0, 8.0, 9.0]),
               wave_A=wave, lum=np.broadcast_to(spec(wave), (2, 3, len(wave))).copy())
    filt = dict(center_A=np.array([3600.0, 6000.0]), sigma_A=np.array([400.0, 250.0]))
    o = oracle_mod.Oracle(ssp, filt, cosmo=dict(Om=1.0))
    th = _theta(tau=3, alpha=2, beta=2, tau_V=1.1, delta=-0.7, F_floor=0.1)
    for z in (0.2, 1.7):
        m = o.phot_exact(synth.SFH_DPL, th[None, :], np.array([z]))[0]
        dl = 2 * C_KMS / 70.0 * (1 + z) * (1 - (1 + z) ** -0.5) * mpc
        k = (1 + z) * lsun / (4 * np.pi * dl * dl * c_ang * 3631e-23)
        att = lambda l: 0.1 + 0.9 * np.exp(-1.1 * (l / 5500.0) ** -0.7)
        for b in range(2):
            cb, sb = filt["center_A"][b], filt["sigma_A"][b]
            tr = lambda l: np.exp(-0.5 * (((1 + z) * l - cb) / sb) ** 2)
            lo, hi = max((cb - 12 * sb) / (1 + z), 100.0), min((cb + 12 * sb) / (1 + z), 1e5)
            num = integrate.quad(lambda l: spec(l) * att(l) * tr(l) * l, lo, hi, epsrel=1e-13, limit=400)[0]
            den = integrate.quad(lambda l: tr(l) / l, lo, hi, epsrel=1e-13, limit=400)[0]
            ref = -2.5 * np.log10(k * 10 ** th[0] * num / den)
            assert m[b] == pytest.approx(ref, abs=1e-9)


def test_exact_photometry_wavelength_grid_converged(oracle_mod, filt6):
    # trapezoid weights on a log grid are proportional to lambda, i.e. the uniform rule in
    # ln(lambda), which converges faster than any power for filters vanishing at both ends
    th, z = synth.galaxies_dpl(3, 11)
    ref = oracle_mod.Oracle(synth.ssp_grid(8000, noise=0.0), filt6).phot_exact(1, th, z)
    m = oracle_mod.Oracle(synth.ssp_grid(500, noise=0.0), filt6).phot_exact(1, th, z)
    np.testing.assert_allclose(m, ref, atol=1e-9)


def test_approx_equals_exact_at_z_nodes_without_dust(orc):
    th, _ = synth.galaxies_dpl(6, 21)
    th[:, synth.P_TAUV] = 0.0
    zk = 0.1 + 2.9 * np.array([0, 5, 17, 40, 63]) / 63
    for k in range(len(zk)):
        z = np.full(6, zk[k])
        me = orc.phot_exact(synth.SFH_DPL, th, z)
        ma = orc.phot_approx(synth.SFH_DPL, th, z)
        np.testing.assert_allclose(ma, me, atol=1e-11)


def test_approx_equals_exact_at_z_nodes_with_grey_dust(orc):
    th, _ = synth.galaxies_dpl(4, 22)
    th[:, synth.P_DELTA] = 0.0      # grey: attenuation constant in wavelength
    z = np.full(4, 0.1 + 2.9 * 30 / 63)
    np.testing.assert_allclose(orc.phot_approx(synth.SFH_DPL, th, z),
                               orc.phot_exact(synth.SFH_DPL, th, z), atol=1e-11)


def test_approx_error_grows_with_band_width(oracle_mod, ssp_small):
    # the approximation is worse for broader transmission curves
    th, z = synth.galaxies_dpl(10, 23)
    th[:, synth.P_TAUV] = 1.5
    err = []
    for sig in (50.0, 200.0, 800.0):
        filt = dict(center_A=np.array([4500.0, 7000.0]), sigma_A=np.array([sig, sig]))
        o = oracle_mod.Oracle(ssp_small, filt)
        o.build_ztable(64, 0.1, 3.0)
        zk = 0.1 + 2.9 * np.round((z - 0.1) / 2.9 * 63) / 63   # on nodes: no interpolation error
        err.append(np.abs(o.phot_approx(1, th, zk) - o.phot_exact(1, th, zk)).max())
    assert err[0] < err[1] < err[2]


def test_approx_out_of_range_z_is_nan(orc):
    th, _ = synth.galaxies_dpl(2, 1)
    m = orc.phot_approx(1, th, np.array([0.05, 3.2]))
    assert np.all(np.isnan(m))


def test_magnitude_shifts_with_mass(orc):
    th, z = synth.galaxies_dpl(3, 5)
    m1 = orc.phot_approx(1, th, z)
    th[:, 0] += 0.4
    np.testing.assert_allclose(orc.phot_approx(1, th, z), m1 - 1.0, atol=1e-12)


# --------------------------------------------------------------------------
# likelihood and gradient
# --------------------------------------------------------------------------
def test_loglike_at_truth_and_mass_gradient_closed_form(orc):
    th, z = synth.galaxies_dpl(5, 31)
    m = orc.phot_approx(1, th, z)
    sig = np.full_like(m, 0.05)
    mask = np.full(5, 0b111111, np.uint8)
    ll, g = orc.loglike_grad(1, th, z, m, sig, mask)
    np.testing.assert_allclose(ll, -6 * np.log(0.05 * np.sqrt(2 * np.pi)), rtol=1e-12)
    np.testing.assert_allclose(g, 0.0, atol=1e-7)
    d = m + np.random.default_rng(0).normal(0, 0.05, m.shape)
    mask[1] = 0b010101
    ll, g = orc.loglike_grad(1, th, z, d, sig, mask)
    bits = (mask[:, None] >> np.arange(6)) & 1
    np.testing.assert_allclose(g[:, 0], 2.5 * ((m - d) / sig ** 2 * bits).sum(1), rtol=1e-9)


@pytest.mark.parametrize("path", [0, 1])
def test_dual_gradient_matches_central_differences(orc_small, path):
    th, z = synth.galaxies_dpl(3, 41)
    m = orc_small.phot_approx(1, th, z)
    d = m + np.random.default_rng(1).normal(0, 0.05, m.shape)
    sig = np.full_like(m, 0.05)
    mask = np.full(3, 63, np.uint8)
    _, g = orc_small.loglike_grad(1, th, z, d, sig, mask, path=path)
    # fourth-order central stencil (h = 1e-4): the likelihood is strongly curved in
    # F_burst when F_burst itself is ~1e-3, where the 2-point stencil's h^2 error shows
    h = 1e-4

    def ll_at(p, dh):
        t = th.copy()
        t[:, p] += dh
        return orc_small.loglike_grad(1, t, z, d, sig, mask, path=path, grad=False)
    for p in range(10):
        fd = (-ll_at(p, 2 * h) + 8 * ll_at(p, h) - 8 * ll_at(p, -h) + ll_at(p, -2 * h)) / (12 * h)
        np.testing.assert_allclose(g[:, p], fd, rtol=2e-5, atol=1e-7 * np.abs(g).max())


@pytest.mark.parametrize("path", [0, 1])
def test_mags_jacobian_matches_central_differences(orc_small, path):
    th, z = synth.galaxies_dpl(2, 43)
    mags, jac = orc_small.mags_jacobian(1, th, z, path=path)
    ref = orc_small.phot_approx(1, th, z) if path == 0 else orc_small.phot_exact(1, th, z)
    np.testing.assert_allclose(mags, ref, atol=1e-12)
    h = 1e-4
    for p in range(10):
        t1, t2, t3, t4 = (th.copy() for _ in range(4))
        t1[:, p] += 2 * h; t2[:, p] += h; t3[:, p] -= h; t4[:, p] -= 2 * h
        f = (lambda t: orc_small.phot_approx(1, t, z)) if path == 0 else (lambda t: orc_small.phot_exact(1, t, z))
        fd = (-f(t1) + 8 * f(t2) - 8 * f(t3) + f(t4)) / (12 * h)
        np.testing.assert_allclose(jac[:, :, p], fd, rtol=1e-5, atol=1e-7)


# --------------------------------------------------------------------------
# bounding function and prior
# --------------------------------------------------------------------------
def test_bounding_roundtrip_and_jacobian(oracle_mod):
    O = oracle_mod.Oracle
    for lo, hi in synth.BOUNDS:
        b = np.array([lo, hi, 1.0, 0.0])
        for x in (-4.0, -0.3, 0.0, 1.7, 5.0):
            th = O.bound(b, x)
            assert lo < th < hi
            assert O.unbound(b, th) == pytest.approx(x, abs=1e-9)
            d = (O.bound(b, x + 1e-6) - O.bound(b, x - 1e-6)) / 2e-6
            assert d == pytest.approx((th - lo) * (hi - th) / (hi - lo), rel=1e-6)


@pytest.mark.parametrize("n", [1, 2, 4, 7, 10, 16])
def test_gauss_legendre_rule_matches_numpy(oracle_mod, n):
    # the quadrature rule behind the oracle's adaptive integrals: numpy's leggauss, and exact
    # integrals of x^k, k < 2n, on [-1, 1]
    x, w = oracle_mod.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr, atol=2e-16)
    np.testing.assert_allclose(w, wr, rtol=1e-14)   # numpy's own weights are good to ~1e-15
    for k in range(2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert np.sum(w * x ** k) == pytest.approx(exact, abs=2e-15)


@pytest.mark.parametrize("k,x0", [(0.5, -1.0), (2.3, 0.7), (0.5, 0.7), (2.3, -1.0)])
def test_bounding_function_general_slope_and_centre(oracle_mod, k, x0):
    # App. C, Eq. BoundingFunction with k != 1 and x0 != 0.  Properties of a logistic map
    # from (-inf, inf) onto (y_lo, y_hi), none of them the formula itself:
    #   the midpoint of the range sits at x0; the map is point-symmetric about it;
    #   its slope there is k (y_hi - y_lo) / 4; it is monotone and tends to the bounds;
    #   its derivative is k (theta - y_lo)(y_hi - theta) / (y_hi - y_lo) (logistic ODE);
    #   unbound inverts it
    O = oracle_mod.Oracle
    for lo, hi in synth.BOUNDS:
        b = np.array([lo, hi, k, x0])
        assert O.bound(b, x0) == pytest.approx(0.5 * (lo + hi), abs=1e-12 * max(1.0, abs(hi)))
        for d in (0.1, 1.3, 4.0):
            assert O.bound(b, x0 + d) + O.bound(b, x0 - d) == pytest.approx(lo + hi, abs=1e-12 * max(1.0, abs(hi)))
        h = 1e-5
        slope = (O.bound(b, x0 + h) - O.bound(b, x0 - h)) / (2 * h)
        assert slope == pytest.approx(k * (hi - lo) / 4, rel=1e-8)
        xs = np.linspace(x0 - 30 / k, x0 + 30 / k, 61)
        th = np.array([O.bound(b, x) for x in xs])
        assert np.all(np.diff(th) >= 0) and th[0] - lo < 1e-9 * (hi - lo) and hi - th[-1] < 1e-9 * (hi - lo)
        for x in (x0 - 3.0 / k, x0 - 0.4, x0 + 0.9, x0 + 5.0 / k):
            t = O.bound(b, x)
            d = (O.bound(b, x + 1e-6) - O.bound(b, x - 1e-6)) / 2e-6
            assert d == pytest.approx(k * (t - lo) * (hi - t) / (hi - lo), rel=1e-6)
            assert O.unbound(b, t) == pytest.approx(x, abs=1e-8)


def test_prior_draws_follow_the_skew_normal(oracle_mod):
    # starting points drawn from the prior (App. C, Eq. SkewNormPrior) for 20,000 chain ids:
    # the skew-normal's closed-form mean xi + omega delta sqrt(2/pi) and variance
    # omega^2 (1 - 2 delta^2 / pi), delta = s / sqrt(1 + s^2), and a Kolmogorov-Smirnov test
    # against scipy's skew-normal CDF
    pri = np.array([[0.0, 1.5, 0.0], [0.3, 0.7, 2.5], [-1.2, 2.0, -4.0], [2.0, 0.5, 8.0], [0.0, 1.0, -0.5],
                    [1.0, 0.2, 0.0], [0.0, 3.0, 1.0], [-2.0, 1.0, 3.0], [0.5, 0.5, -2.0], [0.0, 1.0, 0.0]])
    n = 20000
    x = np.array([oracle_mod.hmc_prior_draw(pri, 404, c) for c in range(n)])
    for p in range(10):
        xi, om, sk = pri[p]
        de = sk / math.sqrt(1 + sk * sk)
        mean, var = xi + om * de * math.sqrt(2 / math.pi), om * om * (1 - 2 * de * de / math.pi)
        assert abs(x[:, p].mean() - mean) < 4.5 * math.sqrt(var / n)
        assert abs(x[:, p].var() / var - 1) < 0.05
        assert stats.kstest(x[:, p], lambda v: stats.skewnorm.cdf(v, sk, loc=xi, scale=om)).pvalue > 1e-3
    # different seeds give different draws; the same seed and chain id the same draw
    assert not np.array_equal(oracle_mod.hmc_prior_draw(pri, 405, 7), x[7])
    assert np.array_equal(oracle_mod.hmc_prior_draw(pri, 404, 7), x[7])


def test_skew_normal_prior_matches_library(oracle_mod):
    O = oracle_mod.Oracle
    for xi, om, s in ((0.0, 1.0, 0.0), (0.3, 0.7, 2.5), (-1.2, 2.0, -4.0)):
        for x in (-2.0, -0.1, 0.4, 3.0):
            ref = stats.skewnorm.logpdf(x, s, loc=xi, scale=om)
            assert O.log_prior([xi, om, s], x) == pytest.approx(ref, rel=1e-12, abs=1e-12)
        tot = integrate.quad(lambda x: math.exp(O.log_prior([xi, om, s], x)), -40, 40, limit=200)[0]
        assert tot == pytest.approx(1.0, abs=1e-9)
    assert O.log_prior([0.2, 1.5, 0.0], 0.9) == pytest.approx(stats.norm.logpdf(0.9, 0.2, 1.5), rel=1e-13)


# --------------------------------------------------------------------------
# RNG, leapfrog, HMC, R-hat
# --------------------------------------------------------------------------
def test_philox_known_answer_vectors(oracle_mod):
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [ln.split() for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle_mod.philox4x32_10(v[0:4], v[4:6])
        assert out.tolist() == v[6:10]


def test_rhat_special_cases(oracle_mod):
    x = np.random.default_rng(3).normal(size=500)
    n = len(x)
    assert oracle_mod.rhat(np.stack([x, x, x, x])) == pytest.approx(math.sqrt((n - 1) / n), rel=1e-13)
    # hand example: chains [0,1,2] and [3,4,5]: W = 1, B/n = var([1,4]) = 4.5, V = 2/3 + 4.5
    assert oracle_mod.rhat(np.array([[0., 1, 2], [3, 4, 5]])) == pytest.approx(math.sqrt(2 / 3 + 4.5), rel=1e-14)


# widths within a factor ~1.6: fixed-length trajectories with an identity mass matrix mix
# badly in dimensions whose period resonates with the trajectory length
GAUSS_SD = np.array([0.8, 1.0, 1.25, 0.9, 1.1, 1.0, 0.85, 1.15, 0.95, 1.05])


def test_leapfrog_reversible_and_second_order(orc):
    prec = np.diag(1 / GAUSS_SD ** 2)
    x0 = np.random.default_rng(4).normal(size=10) * GAUSS_SD
    p0 = np.random.default_rng(5).normal(size=10)
    x1, p1, _ = orc.leapfrog(x0, p0, 0.05, 10, gauss_prec=prec)
    x2, p2, _ = orc.leapfrog(x1, -p1, 0.05, 10, gauss_prec=prec)
    np.testing.assert_allclose(x2, x0, atol=1e-12)
    np.testing.assert_allclose(-p2, p0, atol=1e-12)

    def dH(eps, n):
        x, p, lp = orc.leapfrog(x0, p0, eps, n, gauss_prec=prec)
        return (-lp + 0.5 * p @ p) - (0.5 * x0 @ prec @ x0 + 0.5 * p0 @ p0)
    r = abs(dH(0.02, 20)) / abs(dH(0.01, 40))
    assert 3.5 < r < 4.5


def test_leapfrog_reversible_on_sps_posterior(orc):
    th, z = synth.galaxies_dpl(1, 51)
    bnd = np.column_stack([synth.BOUNDS, np.ones(10), np.zeros(10)])
    pri = np.column_stack([np.zeros(10), np.full(10, 1.5), np.zeros(10)])
    x0 = np.array([orc.unbound(bnd[p], th[0, p]) for p in range(10)])
    obs = orc.phot_approx(1, th, z)[0] + 0.03
    sig = np.full(6, 0.05)
    p0 = np.random.default_rng(6).normal(size=10)
    kw = dict(sfh=1, z=z[0], obs=obs, sigma=sig, mask=63, bounds=bnd, prior=pri)
    x1, p1, _ = orc.leapfrog(x0, p0, 0.01, 10, **kw)
    x2, p2, _ = orc.leapfrog(x1, -p1, 0.01, 10, **kw)
    np.testing.assert_allclose(x2, x0, atol=1e-9)


def test_hmc_gaussian_target_moments(orc):
    # one leapfrog step per iteration (Metropolis-adjusted Langevin): unlike long fixed
    # trajectories it has no resonance with the target's oscillation periods, so the
    # pooled moments must match the Gaussian's within Monte-Carlo error
    prec = np.diag(1 / GAUSS_SD ** 2)
    n_gal, n_chain, ns = 3, 4, 4000
    th0 = np.random.default_rng(7).normal(size=(n_chain, n_gal, 10)) * 3
    out = orc.hmc_run(1, None, None, None, None, None, None, th0, n_chain=n_chain, n_leapfrog=1,
                      n_warmup=300, n_sample=ns, seed=99, gauss_prec=prec)
    assert np.all(out["rhat"] < 1.02)
    assert np.all((out["accept"] > 0.75) & (out["accept"] < 0.95))
    assert np.all(np.abs(out["post_mean"]) < 0.1)
    np.testing.assert_allclose(out["post_sd"], np.broadcast_to(GAUSS_SD, (n_gal, 10)), rtol=0.05)


def test_hmc_dual_averaging_reaches_target_acceptance(orc):
    prec = np.diag(1 / GAUSS_SD ** 2)
    th0 = np.random.default_rng(9).normal(size=(4, 2, 10))
    for target in (0.6, 0.9):
        out = orc.hmc_run(1, None, None, None, None, None, None, th0, n_chain=4, n_leapfrog=10,
                          n_warmup=400, n_sample=400, target_accept=target, seed=3, gauss_prec=prec)
        assert np.all(np.abs(out["accept"] - target) < 0.12)


def test_hmc_tiny_step_accepts_everything_and_is_deterministic(orc):
    prec = np.diag(1 / GAUSS_SD ** 2)
    th0 = np.random.default_rng(8).normal(size=(2, 2, 10))
    kw = dict(n_chain=2, n_warmup=0, n_sample=50, init_step=1e-4, seed=5, gauss_prec=prec, keep_samples=True)
    a = orc.hmc_run(1, None, None, None, None, None, None, th0, **kw)
    b = orc.hmc_run(1, None, None, None, None, None, None, th0, **kw)
    assert np.all(a["accept"] == 1.0)
    assert np.array_equal(a["samples"], b["samples"])


@pytest.mark.parametrize("adapt", [False, "diag", "dense"])
def test_hmc_split_run_reproduces_the_uninterrupted_run(orc, adapt):
    # a run split over three calls (the state carried in between) draws exactly what one call
    # draws: every sample, step size, metric and summary bit for bit; the cuts fall inside the
    # warm-up, on a metric-window boundary and inside the sampling phase
    rng = np.random.default_rng(17)
    a = rng.normal(size=(10, 10))
    prec = a @ a.T / 10 + np.eye(10)
    th0 = rng.normal(size=(2, 3, 10))
    kw = dict(n_chain=2, n_leapfrog=3, n_warmup=100, n_sample=60, seed=21, gauss_prec=prec, adapt_metric=adapt)
    whole = orc.hmc_run(1, None, None, None, None, None, None, th0, keep_samples=True, **kw)
    import oracle
    state = np.zeros((2, 3, oracle.HMC_STATE))
    smp = np.zeros((60, 2, 3, 10))
    for b, e in ((0, 37), (37, 90), (90, 130), (130, 160)):
        part = orc.hmc_run(1, None, None, None, None, None, None, th0, it_begin=b, it_end=e, state=state,
                           samples=smp, **kw)
    assert oracle.hmc_windows(100) == [(15, 90)]
    assert np.array_equal(smp, whole["samples"])
    for key in ("post_mean", "post_sd", "rhat", "accept", "step", "inv_metric"):
        assert np.array_equal(part[key], whole[key]), key


def test_hmc_split_run_on_the_sps_posterior(orc_small):
    sfh, th, z = 1, *synth.galaxies_dpl(2, 61)
    obs = orc_small.phot_approx(sfh, th, z) + 0.02
    sig = np.full_like(obs, 0.05)
    masks = np.array([63, 45], np.uint8)
    bnd = np.column_stack([synth.BOUNDS, np.full(10, 1.3), np.full(10, -0.2)])
    pri = np.column_stack([np.zeros(10), np.full(10, 1.5), np.linspace(-3, 3, 10)])
    kw = dict(n_chain=2, n_leapfrog=4, n_warmup=6, n_sample=4, init_step=0.02, seed=8)
    whole = orc_small.hmc_run(sfh, z, obs, sig, masks, bnd, pri, None, keep_samples=True, **kw)
    import oracle
    state = np.zeros((2, 2, oracle.HMC_STATE))
    smp = np.zeros((4, 2, 2, 10))
    orc_small.hmc_run(sfh, z, obs, sig, masks, bnd, pri, None, it_begin=0, it_end=5, state=state, samples=smp, **kw)
    last = orc_small.hmc_run(sfh, z, obs, sig, masks, bnd, pri, None, it_begin=5, it_end=10, state=state,
                             samples=smp, **kw)
    assert np.array_equal(smp, whole["samples"])
    assert np.array_equal(last["post_mean"], whole["post_mean"])
    assert np.all(np.isfinite(smp))


def test_hmc_start_from_the_prior(orc):
    # theta0 = None draws every chain's start from the prior with its Philox chain id
    # (chain * n_gal + galaxy): the same run as one given those draws explicitly
    import oracle
    rng = np.random.default_rng(2)
    prec = np.diag(rng.uniform(0.5, 2.0, 10))
    pri = np.column_stack([rng.normal(size=10), rng.uniform(0.5, 2, 10), rng.uniform(-3, 3, 10)])
    n_gal, C = 3, 2
    x0 = np.array([[oracle.hmc_prior_draw(pri, 77, c * n_gal + g) for g in range(n_gal)] for c in range(C)])
    kw = dict(n_chain=C, n_leapfrog=2, n_warmup=5, n_sample=5, seed=77, gauss_prec=prec, keep_samples=True)
    a = orc.hmc_run(1, np.zeros(n_gal), None, None, None, None, pri, None, **kw)
    b = orc.hmc_run(1, np.zeros(n_gal), None, None, None, None, pri, x0, **kw)
    assert np.array_equal(a["samples"], b["samples"])


def test_hmc_window_schedule_matches_the_stan_defaults():
    # the documented defaults: buffers of 75 and 50 around slow windows of 25, 50, 100,
    # 200 and (stretched to the end of the slow phase) 500 iterations for 1000 warm-up
    # iterations; 15 % / 75 % / 10 % when the defaults do not fit; none below 20
    import oracle
    assert oracle.hmc_windows(1000) == [(75, 100), (100, 150), (150, 250), (250, 450), (450, 950)]
    assert oracle.hmc_windows(200) == [(75, 100), (100, 150)]
    assert oracle.hmc_windows(150) == [(75, 100)]
    assert oracle.hmc_windows(100) == [(15, 90)]
    assert oracle.hmc_windows(20) == [(3, 18)]
    assert oracle.hmc_windows(19) == []


def test_hmc_metric_adaptation_learns_the_target_variances(orc):
    # a Gaussian whose scales span three decades: the adapted diagonal M^-1 recovers the
    # variances (sampling error of a 500-draw window), which lets the step size grow to
    # the widest direction's scale while the moments stay right.  Once preconditioned the
    # target is near-isotropic with orbit period 2 pi; 7 steps of ~0.65 keep the
    # trajectory length away from that period (10 steps of ~0.7 nearly return to start)
    sd = np.array([0.01, 0.03, 0.1, 0.3, 1.0, 3.0, 10.0, 0.05, 0.5, 5.0])
    prec = np.diag(1 / sd ** 2)
    th0 = np.random.default_rng(12).normal(size=(4, 2, 10)) * sd
    kw = dict(n_chain=4, n_leapfrog=7, n_warmup=1000, n_sample=1000, seed=21, gauss_prec=prec)
    ad = orc.hmc_run(1, None, None, None, None, None, None, th0, adapt_metric=True, **kw)
    ratio = ad["inv_metric"] / sd ** 2
    assert np.all((ratio > 0.5) & (ratio < 2.0)), ratio
    assert np.all(ad["step"] > 0.3)
    np.testing.assert_allclose(ad["post_sd"] / sd, 1.0, atol=0.2)
    assert np.all(ad["rhat"] < 1.05)
    ident = orc.hmc_run(1, None, None, None, None, None, None, th0, adapt_metric=False, **kw)
    assert np.all(ident["inv_metric"] == 1.0)
    assert np.all(ident["step"] < 0.05)


def test_hmc_metric_adaptation_off_below_twenty_warmup_iterations(orc):
    prec = np.diag(1 / GAUSS_SD ** 2)
    th0 = np.random.default_rng(13).normal(size=(2, 2, 10))
    kw = dict(n_chain=2, n_warmup=19, n_sample=20, seed=5, gauss_prec=prec, keep_samples=True)
    a = orc.hmc_run(1, None, None, None, None, None, None, th0, adapt_metric=True, **kw)
    b = orc.hmc_run(1, None, None, None, None, None, None, th0, adapt_metric=False, **kw)
    assert np.array_equal(a["samples"], b["samples"])
    assert np.all(a["inv_metric"] == 1.0)


def test_hmc_dense_metric_adaptation_learns_a_correlated_covariance(orc):
    # correlated Gaussian (correlation 0.9 between neighbours in two pairs, scales spanning
    # a decade): the dense adaptation's M^-1 diagonal recovers the variances and the
    # moments stay right; the diagonal adaptation, which cannot rotate, ends with a smaller
    # step on the same target
    sd = np.array([0.1, 0.1, 1.0, 1.0, 0.3, 3.0, 0.5, 2.0, 1.0, 0.2])
    cor = np.eye(10)
    cor[0, 1] = cor[1, 0] = 0.9
    cor[2, 3] = cor[3, 2] = -0.9
    cov = cor * np.outer(sd, sd)
    prec = np.linalg.inv(cov)
    th0 = np.random.default_rng(14).normal(size=(4, 2, 10)) * sd
    kw = dict(n_chain=4, n_leapfrog=7, n_warmup=1000, n_sample=1000, seed=23, gauss_prec=prec)
    dn = orc.hmc_run(1, None, None, None, None, None, None, th0, adapt_metric="dense", **kw)
    ratio = dn["inv_metric"] / sd ** 2
    assert np.all((ratio > 0.5) & (ratio < 2.0)), ratio
    np.testing.assert_allclose(dn["post_sd"] / sd, 1.0, atol=0.2)
    dg = orc.hmc_run(1, None, None, None, None, None, None, th0, adapt_metric="diag", **kw)
    assert np.median(dn["step"]) > 1.5 * np.median(dg["step"])


def test_exact_path_logpost_gradient_matches_finite_differences(orc_small):
    # the log posterior with exact photometry: its dual-number gradient against central
    # differences of its own value (pins the chain rule through the bounding map and the
    # spectrum-level magnitudes, independently of the approximate path)
    th, z = synth.galaxies_dpl(2, 61)
    bnd = np.column_stack([synth.BOUNDS, np.ones(10), np.zeros(10)])
    pri = np.column_stack([np.zeros(10), np.full(10, 1.5), np.zeros(10)])
    for g in range(2):
        x0 = np.array([orc_small.unbound(bnd[p], th[g, p]) for p in range(10)])
        obs = orc_small.phot_exact(1, th[g:g + 1], z[g:g + 1])[0] + np.array([0.03, -0.02, 0.05, 0.0, -0.04, 0.01])
        sig = np.full(6, 0.05)
        args = (1, z[g], obs, sig, 0b111011, bnd, pri)
        lp, gr = orc_small.logpost_grad(1, x0, *args[1:], path=1)
        lpa, _ = orc_small.logpost_grad(1, x0, *args[1:], path=0)
        assert lp != lpa                     # the two photometry paths are distinct
        h = 1e-5
        for p in range(10):
            e = np.zeros(10)
            e[p] = h
            fd = (orc_small.logpost_grad(1, x0 + e, *args[1:], path=1)[0]
                  - orc_small.logpost_grad(1, x0 - e, *args[1:], path=1)[0]) / (2 * h)
            assert gr[p] == pytest.approx(fd, rel=1e-5, abs=1e-5 * max(1.0, np.abs(gr).max()))


def test_exact_path_hmc_samples_a_consistent_posterior(orc_small):
    # a short exact-photometry HMC run from the truth: every chain moves, acceptance is
    # sane, and the posterior mean of log M stays within a few posterior sds of the truth
    th, z = synth.galaxies_dpl(1, 62)
    bnd = np.column_stack([synth.BOUNDS, np.ones(10), np.zeros(10)])
    pri = np.column_stack([np.zeros(10), np.full(10, 1.5), np.zeros(10)])
    obs = orc_small.phot_exact(1, th, z)
    sig = np.full((1, 6), 0.05)
    x0 = np.array([[[orc_small.unbound(bnd[p], th[0, p]) for p in range(10)]]] * 4)
    out = orc_small.hmc_run(1, z, obs, sig, np.array([63], np.uint8), bnd, pri, x0, n_chain=4, n_leapfrog=5,
                            n_warmup=40, n_sample=60, seed=12, keep_samples=True, path=1)
    s = out["samples"]
    assert np.all(s.std(axis=0)[..., 0] > 0)
    assert 0.2 < out["accept"][0] <= 1.0
    assert abs(out["post_mean"][0, 0] - th[0, 0]) < 4 * out["post_sd"][0, 0] + 0.05


def test_approximation_gap_grows_with_band_width(oracle_mod, ssp_small):
    # App. B: the table approximation (attenuation taken at the effective wavelength) degrades
    # as the band widens, and for bands with lambda/FWHM between ~3.4 and ~25 it stays within
    # 0.06 mag over the bulk of the galaxy population (read as the 99th percentile: over 4096
    # galaxies of this generator 0.2 % exceed it, up to 0.14 mag, all with steep dust, no
    # attenuation floor and in the bluest band).  The sigma = 400 A bands have lambda/FWHM
    # 3.8-10.3.
    th, z = synth.galaxies_dpl(24, 71)
    med = []
    for sig in (200.0, 400.0, 800.0, 1200.0):
        o = oracle_mod.Oracle(ssp_small, synth.filters(sigma=sig))
        o.build_ztable(64, 0.1, 3.0)
        d = np.abs(o.phot_approx(1, th, z) - o.phot_exact(1, th, z))
        med.append(np.median(d))
        if sig == 400.0:
            fwhm = 2.0 * math.sqrt(2.0 * math.log(2.0)) * sig
            ratio = synth.filters(sigma=sig)["center_A"] / fwhm
            assert 3.4 <= ratio.min() and ratio.max() <= 25.5
            assert np.percentile(d, 99) < 0.06
    assert all(a < b for a, b in zip(med, med[1:])), med


def test_approximation_gap_grows_with_dust_optical_depth(oracle_mod, ssp_small):
    # App. B: the table path takes the attenuation at the band's effective wavelength, so its
    # error grows with how much the attenuation varies across the band, i.e. with tau_V.  With
    # no attenuation (tau_V = 0, or a floor F_floor = 1) what is left is the interpolation of the
    # table in z alone: the same gap whatever the dust slope
    o = oracle_mod.Oracle(ssp_small, synth.filters())
    o.build_ztable(64, 0.1, 3.0)
    th, z = synth.galaxies_dpl(24, 73)
    th[:, synth.P_FFLOOR] = 0.0

    def gap(t):
        return o.phot_approx(1, t, z) - o.phot_exact(1, t, z)
    t0 = th.copy()
    t0[:, synth.P_TAUV] = 0.0
    g0 = gap(t0)
    t1 = t0.copy()
    t1[:, synth.P_DELTA] = -1.4
    np.testing.assert_allclose(gap(t1), g0, rtol=0, atol=1e-12)
    t2 = th.copy()
    t2[:, synth.P_TAUV] = 3.0
    t2[:, synth.P_FFLOOR] = 1.0
    np.testing.assert_allclose(gap(t2), g0, rtol=0, atol=1e-12)
    med = []
    for tv in (0.0, 0.5, 1.0, 2.0, 4.0):
        t = th.copy()
        t[:, synth.P_TAUV] = tv
        med.append(np.median(np.abs(gap(t))))
    assert all(a < b for a, b in zip(med, med[1:])), med


# --------------------------------------------------------------------------
# NUTS (Hoffman & Gelman 2014, Algorithm 3 with dual averaging)
# --------------------------------------------------------------------------
def test_nuts_gaussian_target_moments(orc):
    # a 10-dimensional Gaussian with scales over a decade: pooled means and sds within
    # Monte-Carlo error, R-hat ~ 1, the adapted step size near the smallest scale
    sd = np.array([0.5, 1.0, 2.0, 0.3, 1.5, 1.0, 0.8, 1.2, 2.5, 0.7])
    th0 = np.random.default_rng(1).normal(size=(4, 3, 10))
    for adapt in (False, True):
        out = orc.nuts_run(1, None, None, None, None, None, None, th0, n_chain=4, max_depth=10, n_warmup=500,
                           n_sample=3000, seed=5, gauss_prec=np.diag(1 / sd ** 2), adapt_metric=adapt)
        assert np.all(out["rhat"] < 1.01)
        assert np.all(np.abs(out["post_mean"]) < 4 * sd / math.sqrt(4 * 3000 / 4))
        np.testing.assert_allclose(out["post_sd"], np.broadcast_to(sd, (3, 10)), rtol=0.05)
        assert np.all((out["accept"] > 0.7) & (out["accept"] < 0.97))


def test_nuts_u_turn_ends_a_harmonic_trajectory_near_half_a_period(orc):
    # unit Gaussian, identity metric, fixed step 0.1: the phase-space orbits are circles of
    # period 2 pi, and a trajectory turns after about half a period, pi / 0.1 ~ 31 steps, so
    # the doubling stops at depth 5 (31 leaves) nearly always; the draws stay N(0, 1)
    th0 = np.random.default_rng(2).normal(size=(4, 3, 10))
    out = orc.nuts_run(1, None, None, None, None, None, None, th0, n_chain=4, max_depth=10, n_warmup=0,
                       n_sample=2000, init_step=0.1, seed=6, gauss_prec=np.eye(10), keep_samples=True)
    d = out["depth"].ravel()
    assert np.mean(d == 5) > 0.9 and d.min() >= 4
    x = out["samples"].reshape(-1, 10)
    assert stats.kstest(x[:, 0], "norm").pvalue > 1e-3
    assert abs(x.var() - 1.0) < 0.03


def test_nuts_flat_target_proposal_is_uniform_over_the_last_doubling(orc):
    # zero gradient (flat target): trajectories are straight lines, never turn and never leave
    # the slice, so every tree reaches max_depth and, at each doubling, the new subtree holds as
    # many valid leaves as the tree before it: the proposal is taken from it with probability
    # min(1, n'/n) = 1.  The draw is therefore uniform over the 2^(D-1) leaves of the last
    # doubling: its distance from the start, in steps, is uniform over that stretch
    D, eps = 4, 0.5
    th0 = np.zeros((1, 500, 10))
    out = orc.nuts_run(1, None, None, None, None, None, None, th0, n_chain=1, max_depth=D, n_warmup=0,
                       n_sample=2, init_step=eps, seed=7, gauss_prec=np.zeros((10, 10)), keep_samples=True)
    assert np.all(out["depth"] == D) and np.all(out["steps"] == 2 ** D - 1)
    # first iteration: x = k eps p0 for the chosen leaf k (signed); |k| in the last doubling is
    # 2^(D-1) .. 2^D - 1 on the side it grew, minus the leaves of the earlier doublings on
    # the other side; the leaf's index within the last doubling is uniform on 0 .. 2^(D-1) - 1
    import oracle
    idx = []
    for g in range(500):
        w = np.concatenate([oracle.philox4x32_10([b, 0, g, 0], [7, 0]) for b in range(3)])
        u = (w.astype(np.float64) + 0.5) / 2 ** 32
        p0 = np.empty(10)
        r = np.sqrt(-2 * np.log(u[0:10:2]))
        a = 2 * np.pi * u[1:10:2]
        p0[0::2], p0[1::2] = r * np.cos(a), r * np.sin(a)
        kk = out["samples"][0, 0, g, 0] / (eps * p0[0])        # signed leaf offset of the draw
        dirs = [1 if (oracle.philox4x32_10([j, 0, g, 2], [7, 0])[0] + 0.5) / 2 ** 32 >= 0.5 else -1
                for j in range(D)]
        left = sum(2 ** j for j in range(D - 1) if dirs[j] < 0)
        right = sum(2 ** j for j in range(D - 1) if dirs[j] > 0)
        k = int(round(kk))
        assert abs(kk - k) < 1e-6
        if dirs[-1] > 0:
            assert right < k <= right + 2 ** (D - 1)
            idx.append(k - right - 1)
        else:
            assert -left - 2 ** (D - 1) <= k < -left
            idx.append(-left - 1 - k)
    counts = np.bincount(idx, minlength=2 ** (D - 1))
    assert stats.chisquare(counts).pvalue > 1e-3


def test_nuts_step_size_adaptation_reaches_its_target(orc):
    prec = np.diag(1 / np.linspace(0.5, 2.0, 10) ** 2)
    th0 = np.random.default_rng(9).normal(size=(4, 2, 10))
    for target in (0.65, 0.9):
        out = orc.nuts_run(1, None, None, None, None, None, None, th0, n_chain=4, max_depth=8, n_warmup=600,
                           n_sample=600, target_accept=target, seed=3, gauss_prec=prec)
        assert np.all(np.abs(out["accept"] - target) < 0.1)


def test_nuts_on_the_sps_posterior_agrees_with_hmc(orc_small):
    # the same posterior sampled by NUTS and by long-run HMC with an adapted metric: the
    # posterior means agree within a few posterior sds / sqrt(ESS)
    sfh, (th, z) = 1, synth.galaxies_dpl(1, 63)
    obs = orc_small.phot_approx(sfh, th, z) + np.random.default_rng(5).normal(0, 0.05, (1, 6))
    sig = np.full_like(obs, 0.05)
    masks = np.array([63], np.uint8)
    bnd = np.column_stack([synth.BOUNDS, np.ones(10), np.zeros(10)])
    pri = np.column_stack([np.zeros(10), np.full(10, 1.5), np.zeros(10)])
    x0 = np.array([[[orc_small.unbound(bnd[p], th[g, p]) for p in range(10)] for g in range(1)]] * 8)
    nu = orc_small.nuts_run(sfh, z, obs, sig, masks, bnd, pri, x0, n_chain=8, max_depth=6, n_warmup=100,
                            n_sample=150, seed=11, init_step=0.01, adapt_metric=True)
    hm = orc_small.hmc_run(sfh, z, obs, sig, masks, bnd, pri, x0, n_chain=8, n_leapfrog=15, n_warmup=100,
                           n_sample=150, seed=12, init_step=0.01, adapt_metric=True)
    assert np.all(np.isfinite(nu["post_mean"]))
    dev = np.abs(nu["post_mean"] - hm["post_mean"]) / (np.maximum(nu["post_sd"], hm["post_sd"]) + 1e-9)
    assert np.median(dev) < 0.5, dev
    assert nu["depth"][100:].mean() > 2
