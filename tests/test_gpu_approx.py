"""GPU parity of the approximate path, weights, z table, likelihood and its
adjoint against the FP64 oracle (same seeded float32 inputs)."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import (bound_jacobian, bounds_prior, dev, f32, gal_inputs, general_bounds_prior, grad_close, grad_ok,
                        grad_tol, grad_vec_ok, soa)

pytestmark = pytest.mark.gpu

MAG_TOL = 1e-4           # FP32 path vs FP64 oracle, magnitudes


@pytest.fixture(scope="module")
def ctx(ssp2000, filt6):
    import paper_2506_19919_amd as sps
    c = sps.Context(ssp2000, filt6, precisions=(sps.SPS_F64, sps.SPS_F32), max_gal=1 << 20)
    c.build_ztable(64, 0.1, 3.0)
    yield c
    c.close()


def test_ztable_matches_oracle(ctx, orc):
    q = ctx.get_ztable().astype(np.float64)
    ref = orc.q
    big = np.abs(ref) > 1e-30 * np.abs(ref).max()
    np.testing.assert_allclose(q[big], ref[big], rtol=2e-6)


@pytest.mark.parametrize("kind,n", [("dpl", 1), ("dpl", 63), ("lognormal_burst", 130), ("dpl", 257)])
def test_weights_match_oracle(ctx, orc, kind, n):
    sfh, th, z = gal_inputs(kind, n, 11 + n)
    w = ctx.weights(sfh, soa(th), dev(z)).cpu().numpy().astype(np.float64)
    ref = orc.weights(sfh, th, z)
    for g in range(n):
        np.testing.assert_allclose(w[g].sum(), 10 ** th[g, 0], rtol=2e-5)
        # every weight within 1e-4 relative, or 1e-7 of the mass formed for the tiny tail bins
        np.testing.assert_allclose(w[g], ref[g], rtol=1e-4, atol=1e-7 * 10 ** th[g, 0])


@pytest.mark.parametrize("kind,n", [("lognormal_burst", 1000), ("dpl", 1000), ("lognormal", 65)])
def test_approx_mags_match_oracle(ctx, orc, kind, n):
    sfh, th, z = gal_inputs(kind, n, 100 + n)
    m = ctx.phot_approx(sfh, soa(th), dev(z)).cpu().numpy().astype(np.float64)
    ref = orc.phot_approx(sfh, th, z)
    assert np.abs(m - ref).max() <= MAG_TOL, np.abs(m - ref).max()


def test_approx_edge_cases(ctx, orc):
    sfh, th, z = gal_inputs("dpl", 5, 7)
    z[1], z[3] = 0.05, 3.5          # outside the table -> NaN for those galaxies only
    z[2] = 3.0                      # last node exactly
    z[4] = 0.1                      # first node exactly
    m = ctx.phot_approx(sfh, soa(th), dev(z)).cpu().numpy()
    assert np.all(np.isnan(m[[1, 3]])) and np.all(np.isfinite(m[[0, 2, 4]]))
    ref = orc.phot_approx(sfh, th, z)
    np.testing.assert_allclose(m[[0, 2, 4]], ref[[0, 2, 4]], atol=MAG_TOL)
    # the out-of-table redshifts are reported by the next status check, which clears the flag
    import paper_2506_19919_amd as sps
    with pytest.raises(sps.SpsError) as e:
        ctx.status()
    assert e.value.code == sps.SPS_E_RANGE
    ctx.status()
    ctx.phot_approx(sfh, soa(th[[0, 2, 4]]), dev(z[[0, 2, 4]]))
    ctx.status()
    # empty batch is a no-op
    empty = torch.empty((10, 0), device="cuda")
    out = ctx.phot_approx(sfh, empty, torch.empty(0, device="cuda"))
    assert out.shape == (0, 6)


def _obs(orc, sfh, th, z, seed, masks=None):
    m = orc.phot_approx(sfh, th, z)
    noise, sig = synth.photometric_noise(len(z), 6, seed)
    if masks is None:
        masks = np.full(len(z), 63, np.uint8)
    return f32(m + noise), f32(sig), masks


@pytest.mark.parametrize("n", [1, 200, 1000])
def test_loglike_grad_matches_oracle(ctx, orc, n):
    sfh, th, z = gal_inputs("dpl", n, 300 + n)
    obs, sig, masks = _obs(orc, sfh, th, z, 9, synth.band_masks(n, 6, 5))
    ll, g = ctx.loglike_grad(sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8))
    ll, g = ll.cpu().numpy().astype(np.float64), g.cpu().numpy().T.astype(np.float64)
    rl, rg = orc.loglike_grad(sfh, th, z, obs, sig, masks)
    m_gpu = ctx.phot_approx(sfh, soa(th), dev(z)).cpu().numpy()
    prop, m_ref = grad_tol(orc, sfh, th, z, sig, masks, m_gpu)
    dm = np.abs(m_gpu - m_ref).max()
    assert dm <= 1e-4
    # logL = -chi2/2 + const: |dlogL| <= sum_b |r_b| |dm_b| / s_b + rounding
    r = np.abs(m_ref - obs) / sig
    assert np.all(np.abs(ll - rl) <= np.sum(r * (np.abs(m_gpu - m_ref) + 2e-6) / sig, axis=1) + 1e-5 * np.abs(rl) + 1e-5)
    ok = grad_ok(g, rg, prop)
    assert ok.all(), (dm, np.argwhere(~ok)[:10], g[~ok][:10], rg[~ok][:10], prop[~ok][:10])
    # the propagated term is a small part of the budget for most components
    assert np.median(prop / np.maximum(np.abs(rg), 1e-12)) < 1e-3


def test_loglike_value_only_matches_grad_call(ctx, orc):
    sfh, th, z = gal_inputs("dpl", 300, 17)
    obs, sig, masks = _obs(orc, sfh, th, z, 3)
    args = (sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8))
    l1 = ctx.loglike_grad(*args, grad=False).cpu().numpy()
    l2, _ = ctx.loglike_grad(*args)
    np.testing.assert_array_equal(l1, l2.cpu().numpy())


def test_loglike_lognormal_grad(ctx, orc):
    sfh, th, z = gal_inputs("lognormal_burst", 200, 23)
    obs, sig, masks = _obs(orc, sfh, th, z, 4)
    ll, g = ctx.loglike_grad(sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8))
    rl, rg = orc.loglike_grad(sfh, th, z, obs, sig, masks)
    g = g.cpu().numpy().T.astype(np.float64)
    assert np.all(g[:, 3] == 0)                    # slot 3 is unused by the log-normal SFH
    m_gpu = ctx.phot_approx(sfh, soa(th), dev(z)).cpu().numpy()
    prop, _ = grad_tol(orc, sfh, th, z, sig, masks, m_gpu)
    ok = grad_ok(g, rg, prop)
    assert ok.all(), (np.argwhere(~ok)[:10], g[~ok][:10], rg[~ok][:10])


def test_logpost_grad_matches_oracle(ctx, orc):
    sfh, th, z = gal_inputs("dpl", 40, 31)
    obs, sig, masks = _obs(orc, sfh, th, z, 6)
    bnd, pri = bounds_prior()
    x = f32(np.array([[orc.unbound(bnd[p], th[g, p]) for p in range(10)] for g in range(40)]))
    lp, gr = ctx.logpost_grad(sfh, soa(x), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8), dev(bnd), dev(pri))
    lp, gr = lp.cpu().numpy(), gr.cpu().numpy().T.astype(np.float64)
    # physical parameters the GPU sees, for the propagated-error bound (chain rule d theta / d x)
    thx = np.array([[orc.bound(bnd[p], x[g, p]) for p in range(10)] for g in range(40)])
    m_gpu = ctx.phot_approx(sfh, soa(f32(thx)), dev(z)).cpu().numpy()
    prop, _ = grad_tol(orc, sfh, thx, z, sig, masks, m_gpu)
    dth = (thx - bnd[:, 0]) * (bnd[:, 1] - thx) / (bnd[:, 1] - bnd[:, 0])
    for g in range(40):
        rl, rg = orc.logpost_grad(sfh, x[g], z[g], obs[g], sig[g], masks[g], bnd, pri)
        assert abs(lp[g] - rl) < 1e-3 * max(1.0, abs(rl))
        ok = grad_ok(gr[g:g + 1], rg[None, :], prop[g:g + 1] * dth[g] * 1.01)
        assert ok.all(), (g, gr[g], rg, prop[g] * dth[g])


@pytest.mark.parametrize("n", [40, 130])
def test_logpost_grad_skewed_prior_general_bounds(ctx, orc, n):
    # App. C with k != 1, x0 != 0 and s != 0: both branches of the skew-normal log prior
    # (Phi directly, and the scaled complementary error function where s y < -5)
    sfh, th, z = gal_inputs("dpl", n, 37 + n)
    obs, sig, masks = _obs(orc, sfh, th, z, 8, synth.band_masks(n, 6, 3))
    bnd1, _ = bounds_prior()
    x_mid = np.median([[orc.unbound(bnd1[p], th[g, p]) for p in range(10)] for g in range(n)], axis=0)
    bnd, pri = general_bounds_prior(x_mid)
    x = f32(np.array([[orc.unbound(bnd[p], th[g, p]) for p in range(10)] for g in range(n)]))
    assert np.all(np.isfinite(x))
    y9 = (x[:, 9] - pri[9, 0]) / pri[9, 1]
    assert np.sum(pri[9, 2] * y9 < -5) >= n // 4 and np.sum(pri[9, 2] * y9 > -5) >= 1
    lp, gr = ctx.logpost_grad(sfh, soa(x), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8), dev(bnd), dev(pri))
    lp, gr = lp.cpu().numpy(), gr.cpu().numpy().T.astype(np.float64)
    thx = np.array([[orc.bound(bnd[p], x[g, p]) for p in range(10)] for g in range(n)])
    m_gpu = ctx.phot_approx(sfh, soa(f32(thx)), dev(z)).cpu().numpy()
    prop, _ = grad_tol(orc, sfh, thx, z, sig, masks, m_gpu)
    for g in range(n):
        rl, rg = orc.logpost_grad(sfh, x[g], z[g], obs[g], sig[g], masks[g], bnd, pri)
        assert abs(lp[g] - rl) < 1e-3 * max(1.0, abs(rl)), (g, lp[g], rl)
        ok = grad_ok(gr[g:g + 1], rg[None, :], prop[g:g + 1] * bound_jacobian(bnd, thx[g]) * 1.01)
        assert ok.all(), (g, gr[g], rg)


def test_deterministic_across_runs(ctx, orc):
    sfh, th, z = gal_inputs("dpl", 777, 41)
    obs, sig, masks = _obs(orc, sfh, th, z, 8)
    args = (sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8))
    a = [t.cpu().numpy() for t in ctx.loglike_grad(*args)]
    b = [t.cpu().numpy() for t in ctx.loglike_grad(*args)]
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_kernel_timing_records_the_model_kernel(ctx, orc):
    import paper_2506_19919_amd as sps
    sfh, th, z = gal_inputs("dpl", 300, 43)
    obs, sig, masks = _obs(orc, sfh, th, z, 8)
    args = (sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8))
    ref = [t.cpu().numpy() for t in ctx.loglike_grad(*args)]
    ctx.set_kernel_timing(3)
    try:
        for _ in range(5):
            out = [t.cpu().numpy() for t in ctx.loglike_grad(*args)]
        ms = ctx.kernel_times()
    finally:
        ctx.set_kernel_timing(0)
    # the last three launches, each a positive duration; results unchanged by the events
    assert ms.shape == (3,) and np.all(ms > 0.0) and np.all(ms < 1e3)
    np.testing.assert_array_equal(out[0], ref[0])
    np.testing.assert_array_equal(out[1], ref[1])
    with pytest.raises(sps.SpsError):
        ctx.kernel_times()


def test_autograd_function_uses_the_adjoint(ctx, orc):
    import paper_2506_19919_amd as sps
    sfh, th, z = gal_inputs("dpl", 50, 51)
    obs, sig, masks = _obs(orc, sfh, th, z, 10)
    p = soa(th).requires_grad_(True)
    ll = sps.loglike(ctx, p, dev(z), dev(obs), dev(sig), dev(masks, torch.uint8))
    (2.0 * ll.sum()).backward()
    _, direct = ctx.loglike_grad(sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8))
    np.testing.assert_array_equal(p.grad.cpu().numpy(), 2.0 * direct.cpu().numpy())


def test_full_size_loglike_sampled(ctx, orc):
    # 10^6 galaxies (the likelihood workload's size), in the launch the benchmark times;
    # a sample of 64 galaxies is checked one by one against the oracle
    n = 1_000_000
    th, z = synth.galaxies_dpl(n, 103)
    th, z = f32(th), f32(z)
    rng = np.random.default_rng(5)
    pick = rng.choice(n, 64, replace=False)
    obs = f32(np.full((n, 6), 22.0))
    sig = f32(np.full((n, 6), 0.05))
    obs[pick] = f32(orc.phot_approx(1, th[pick], z[pick]) + rng.normal(0, 0.05, (64, 6)))
    masks = np.full(n, 63, np.uint8)
    ll, g = ctx.loglike_grad(1, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8))
    m_all = ctx.phot_approx(1, soa(th), dev(z)).cpu().numpy()
    ll, g = ll.cpu().numpy()[pick], g.cpu().numpy().T[pick].astype(np.float64)
    rl, rg = orc.loglike_grad(1, th[pick], z[pick], obs[pick], sig[pick], masks[pick])
    prop, m_ref = grad_tol(orc, 1, th[pick], z[pick], sig[pick], masks[pick], m_all[pick])
    assert np.abs(m_all[pick] - m_ref).max() <= 1e-4
    assert np.all(np.abs(ll - rl) < 0.05 + 1e-4 * np.abs(rl))
    assert grad_ok(g, rg, prop).all()


def test_parameter_box_corners_match_oracle(ctx, orc):
    # every parameter at its bounds (or at the edge of the workload ranges) one at a time on
    # top of a mid-range galaxy: flat and steep double power laws, tau at both ends, bursts
    # older and younger than the whole age grid, no / maximal dust, grey dust, full floor,
    # and a galaxy with no band in its mask (log L = 0, zero gradient)
    base = np.array([10.0, 3.0, 2.0, 2.0, 0.05, 7.0, -0.5, 1.0, -0.7, 0.1])
    cases = [(1, 0.1), (1, 14.0), (2, 0.1), (2, 8.0), (3, 0.1), (3, 8.0), (4, 0.0), (4, 0.2),
             (5, 4.5), (5, 8.5), (6, -2.0), (6, 0.4), (7, 0.0), (7, 4.0), (8, 0.0), (8, -1.5),
             (9, 0.0), (9, 0.5)]
    th = np.tile(base, (len(cases) + 1, 1))
    for r, (p, v) in enumerate(cases):
        th[r, p] = v
    th, n = f32(th), len(th)
    z = f32(np.linspace(0.12, 2.9, n))
    sfh = synth.SFH_DPL
    m = ctx.phot_approx(sfh, soa(th), dev(z)).cpu().numpy()
    m_ref = orc.phot_approx(sfh, th, z)
    assert np.abs(m - m_ref).max() <= MAG_TOL, np.abs(m - m_ref).max(axis=1)
    obs, sig, masks = _obs(orc, sfh, th, z, 21)
    masks[-1] = 0
    ll, g = ctx.loglike_grad(sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8))
    ll, g = ll.cpu().numpy().astype(np.float64), g.cpu().numpy().T.astype(np.float64)
    rl, rg = orc.loglike_grad(sfh, th, z, obs, sig, masks)
    prop, _ = grad_tol(orc, sfh, th, z, sig, masks, m)
    assert ll[-1] == 0.0 and np.all(g[-1] == 0.0)
    assert np.all(np.abs(ll - rl) <= 1e-3 * np.abs(rl) + 1e-4)
    ok = grad_ok(g, rg, prop)
    assert ok.all(), (np.argwhere(~ok)[:10], g[~ok][:10], rg[~ok][:10])


def test_weights_at_parameter_box_corners(ctx, orc):
    base = np.array([10.0, 3.0, 2.0, 2.0, 0.05, 7.0, -0.5, 1.0, -0.7, 0.1])
    rows = []
    for p, v in [(1, 0.1), (1, 14.0), (2, 8.0), (3, 8.0), (4, 0.2), (5, 4.5), (5, 8.5), (6, -2.0), (6, 0.4)]:
        t = base.copy()
        t[p] = v
        rows.append(t)
    th = f32(np.array(rows))
    z = f32(np.linspace(0.1, 3.0, len(th)))
    w = ctx.weights(synth.SFH_DPL, soa(th), dev(z)).cpu().numpy().astype(np.float64)
    ref = orc.weights(synth.SFH_DPL, th, z)
    for g in range(len(th)):
        np.testing.assert_allclose(w[g].sum(), 10 ** th[g, 0], rtol=2e-5)
        np.testing.assert_allclose(w[g], ref[g], rtol=1e-4, atol=1e-7 * 10 ** th[g, 0])


@pytest.mark.parametrize("n_band", [3, 8])
def test_other_band_counts_match_oracle(oracle_mod, ssp2000, n_band):
    """The per-wave LDS block is sized by the band count (the FP32 table row sums outgrow the
    24-bit columns from 7 bands on): magnitudes, log L and gradient at 3 and 8 bands."""
    import paper_2506_19919_amd as sps
    filt = synth.filters(n_band)
    o = oracle_mod.Oracle(ssp2000, filt)
    o.build_ztable(64, 0.1, 3.0)
    c = sps.Context(ssp2000, filt, precisions=(sps.SPS_F64, sps.SPS_F32), max_gal=4096)
    try:
        c.build_ztable(64, 0.1, 3.0)
        n = 300
        sfh, th, z = gal_inputs("dpl", n, 900 + n_band)
        m = c.phot_approx(sfh, soa(th), dev(z)).cpu().numpy().astype(np.float64)
        m_ref = o.phot_approx(sfh, th, z)
        assert m.shape == (n, n_band)
        assert np.abs(m - m_ref).max() <= MAG_TOL, np.abs(m - m_ref).max()
        noise, sig = synth.photometric_noise(n, n_band, 31)
        obs, sig = f32(m_ref + noise), f32(sig)
        masks = synth.band_masks(n, n_band, 7, lo=min(3, n_band), hi=n_band)
        ll, g = c.loglike_grad(sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8))
        ll, g = ll.cpu().numpy().astype(np.float64), g.cpu().numpy().T.astype(np.float64)
        rl, rg = o.loglike_grad(sfh, th, z, obs, sig, masks)
        prop, _ = grad_tol(o, sfh, th, z, sig, masks, m)
        assert np.all(np.abs(ll - rl) <= 1e-3 * np.abs(rl) + 1e-4)
        ok = grad_ok(g, rg, prop)
        assert ok.all(), (np.argwhere(~ok)[:10], g[~ok][:10], rg[~ok][:10])
    finally:
        c.close()


def test_many_table_nodes(ssp2000, filt6, orc):
    # a 1000-node z table: 1000 sort buckets (four per thread of the sort's scans) over a ragged
    # batch of several sort blocks; magnitudes and the likelihood gradient against the oracle
    # built on the same nodes
    import oracle
    import paper_2506_19919_amd as sps
    n, n_z = 3001, 1000
    c = sps.Context(ssp2000, filt6, precisions=(sps.SPS_F32,), max_gal=4096)
    try:
        c.build_ztable(n_z, 0.1, 3.0)
        o = oracle.Oracle(ssp2000, filt6)
        o.build_ztable(n_z, 0.1, 3.0)
        sfh, th, z = gal_inputs("dpl", n, 4242)
        m = c.phot_approx(sfh, soa(th), dev(z)).cpu().numpy().astype(np.float64)
        ref = o.phot_approx(sfh, th, z)
        assert np.abs(m - ref).max() <= MAG_TOL, np.abs(m - ref).max()
        obs, sig, masks = _obs(o, sfh, th, z, 17, synth.band_masks(n, 6, 18))
        ll, g = c.loglike_grad(sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8))
        g = g.cpu().numpy().T.astype(np.float64)
        rl, rg = o.loglike_grad(sfh, th, z, obs, sig, masks)
        prop, m_ref = grad_tol(o, sfh, th, z, sig, masks, m)
        assert grad_ok(g, rg, prop).all()
        r = np.abs(m_ref - obs) / sig
        bar = np.sum(r * (np.abs(m - m_ref) + 2e-6) / sig, axis=1) + 1e-5 * np.abs(rl) + 1e-5
        assert np.all(np.abs(ll.cpu().numpy() - rl) <= bar)
        c.status()
    finally:
        c.close()
