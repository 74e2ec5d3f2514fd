"""GPU parity of the exact (MFMA) photometry and its likelihood gradient against
the FP64 oracle: FP64 path <= 1e-9 mag, FP32 <= 1e-4 mag, BF16 hi+lo split
<= 2e-3 mag, gradients <= 1e-3 relative (with a floor)."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import dev, f32, gal_inputs, grad_ok, grad_tol, soa

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx2000(ssp2000, filt6):
    import paper_2506_19919_amd as sps
    c = sps.Context(ssp2000, filt6, precisions=(sps.SPS_F64, sps.SPS_F32, sps.SPS_BF16X), max_gal=1 << 16,
                    max_exact=1 << 14)
    yield c
    c.close()


@pytest.fixture(scope="module")
def ssp5000():
    return synth.ssp_grid(5000)


@pytest.fixture(scope="module")
def ctx5000(ssp5000, filt6):
    import paper_2506_19919_amd as sps
    c = sps.Context(ssp5000, filt6, precisions=(sps.SPS_F64, sps.SPS_F32, sps.SPS_BF16X), max_gal=1 << 16,
                    max_exact=4096)
    yield c
    c.close()


@pytest.fixture(scope="module")
def orc5000(oracle_mod, ssp5000, filt6):
    return oracle_mod.Oracle(ssp5000, filt6)


def test_exact_f64_lognormal_64_galaxies(ctx2000, orc):
    import paper_2506_19919_amd as sps
    sfh, th, z = gal_inputs("lognormal", 64, 101)
    m = ctx2000.phot_exact(sfh, soa(th, torch.float64), dev(z, torch.float64), prec=sps.SPS_F64)
    ref = orc.phot_exact(sfh, th, z)
    err = np.abs(m.cpu().numpy() - ref).max()
    assert err <= 1e-9, err


@pytest.mark.parametrize("n", [1, 70])
def test_exact_f64_dpl_ragged(ctx2000, orc, n):
    import paper_2506_19919_amd as sps
    sfh, th, z = gal_inputs("dpl", n, 7 + n)
    m = ctx2000.phot_exact(sfh, soa(th, torch.float64), dev(z, torch.float64), prec=sps.SPS_F64)
    err = np.abs(m.cpu().numpy() - orc.phot_exact(sfh, th, z)).max()
    assert err <= 1e-8, err


@pytest.mark.parametrize("prec_name,tol", [("SPS_F32", 1e-4), ("SPS_BF16X", 2e-3)])
def test_exact_forward_5000_wavelengths(ctx5000, orc5000, prec_name, tol):
    import paper_2506_19919_amd as sps
    sfh, th, z = gal_inputs("dpl", 130, 105)
    m = ctx5000.phot_exact(sfh, soa(th), dev(z), prec=getattr(sps, prec_name)).cpu().numpy()
    err = np.abs(m - orc5000.phot_exact(sfh, th, z)).max()
    assert err <= tol, err


@pytest.mark.parametrize("prec_name,tol", [("SPS_F32", 1e-4), ("SPS_BF16X", 2e-3)])
def test_exact_loglike_grad(ctx5000, orc5000, prec_name, tol):
    import paper_2506_19919_amd as sps
    n = 24
    sfh, th, z = gal_inputs("dpl", n, 205)
    m = orc5000.phot_exact(sfh, th, z)
    noise, sig = synth.photometric_noise(n, 6, 205)
    obs, sig = f32(m + noise), f32(sig)
    masks = synth.band_masks(n, 6, 3)
    prec = getattr(sps, prec_name)
    ll, g = ctx5000.loglike_grad(sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8),
                                 path=sps.SPS_PATH_EXACT, prec=prec)
    rl, rg = orc5000.loglike_grad(sfh, th, z, obs, sig, masks, path=1)
    ll, g = ll.cpu().numpy(), g.cpu().numpy().T.astype(np.float64)
    # |dlogL| <= sum_b |r_b| / sigma * (mag error)
    r = np.abs((m - obs) / sig) * ((masks[:, None] >> np.arange(6)) & 1)
    assert np.all(np.abs(ll - rl) <= (r.sum(1) / 0.05) * tol + 1e-3)
    m_gpu = ctx5000.phot_exact(sfh, soa(th), dev(z), prec=prec).cpu().numpy()
    prop, _ = grad_tol(orc5000, sfh, th, z, sig, masks, m_gpu, path=1)
    ok = grad_ok(g, rg, prop)
    assert ok.all(), (np.argwhere(~ok)[:8], g[~ok][:8], rg[~ok][:8], prop[~ok][:8])


@pytest.mark.parametrize("prec_name,tol", [("SPS_F32", 1e-4), ("SPS_BF16X", 2e-3)])
def test_exact_loglike_grad_large_batch(ctx2000, orc, prec_name, tol):
    # 16,384 galaxies: the gradient GEMM has enough output tiles to run without the K split
    # (the batch size of the exact-photometry HMC); sampled galaxies against the oracle
    import paper_2506_19919_amd as sps
    n = 16_384
    sfh, th, z = gal_inputs("dpl", n, 305)
    rng = np.random.default_rng(1)
    pick = np.sort(rng.choice(n, 8, replace=False))
    noise, sig = synth.photometric_noise(n, 6, 306)
    obs = f32(np.full((n, 6), 22.0))
    obs[pick] = f32(orc.phot_exact(sfh, th[pick], z[pick]) + noise[pick])
    sig = f32(sig)
    masks = synth.band_masks(n, 6, 307)
    prec = getattr(sps, prec_name)
    ll, g = ctx2000.loglike_grad(sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8),
                                 path=sps.SPS_PATH_EXACT, prec=prec)
    ll, g = ll.cpu().numpy(), g.cpu().numpy().T.astype(np.float64)
    assert np.isfinite(ll).all() and np.isfinite(g).all()
    rl, rg = orc.loglike_grad(sfh, th[pick], z[pick], obs[pick], sig[pick], masks[pick], path=1)
    m = orc.phot_exact(sfh, th[pick], z[pick])
    r = np.abs((m - obs[pick]) / sig[pick]) * ((masks[pick][:, None] >> np.arange(6)) & 1)
    assert np.all(np.abs(ll[pick] - rl) <= (r.sum(1) / 0.05) * tol + 1e-3)
    # the whole batch's magnitudes (ranked by z inside the library, returned in input order)
    m_all = ctx2000.phot_exact(sfh, soa(th), dev(z), prec=prec).cpu().numpy()
    assert np.isfinite(m_all).all()
    assert np.abs(m_all[pick] - m).max() <= tol
    prop, _ = grad_tol(orc, sfh, th[pick], z[pick], sig[pick], masks[pick], m_all[pick], path=1)
    ok = grad_ok(g[pick], rg, prop)
    assert ok.all(), (np.argwhere(~ok)[:8], g[pick][~ok][:8], rg[~ok][:8], prop[~ok][:8])


@pytest.mark.parametrize("prec_name,tol", [("SPS_F32", 1e-4), ("SPS_BF16X", 2e-3)])
def test_exact_loglike_grad_grouped_rbar_every_output(ssp2000, filt6, orc, prec_name, tol):
    # 40,003 galaxies (the size class of the exact-photometry HMC, where the gradient kernel
    # takes four galaxies per block; 40,003 = 4 x 10,000 + 3 leaves a ragged last block):
    # 32 distinct galaxies, each repeated, so that every output, wherever the internal z
    # ranking puts its row, is checked against its prototype's oracle value.  Their redshifts
    # lie in three of the ranking's 0.125-wide z buckets, so the copies of different galaxies
    # mix inside a bucket and a block's four rows are mostly different galaxies
    import paper_2506_19919_amd as sps
    n, k = 40_003, 32
    sfh, th0, _ = gal_inputs("dpl", k, 311)
    z0 = f32(np.random.default_rng(315).uniform(1.0, 1.35, k))
    noise, sig0 = synth.photometric_noise(k, 6, 312)
    obs0 = f32(orc.phot_exact(sfh, th0, z0) + noise)
    sig0 = f32(sig0)
    masks0 = synth.band_masks(k, 6, 313)
    rep = np.random.default_rng(314).integers(0, k, n)
    rep[:k] = np.arange(k)
    th, z, obs, sig, masks = th0[rep], z0[rep], obs0[rep], sig0[rep], masks0[rep]
    prec = getattr(sps, prec_name)
    c = sps.Context(ssp2000, filt6, precisions=(sps.SPS_F32, sps.SPS_BF16X), max_gal=n, max_exact=n)
    try:
        ll, g = c.loglike_grad(sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8),
                               path=sps.SPS_PATH_EXACT, prec=prec)
        m_all = c.phot_exact(sfh, soa(th), dev(z), prec=prec).cpu().numpy()
    finally:
        c.close()
    ll, g = ll.cpu().numpy(), g.cpu().numpy().T.astype(np.float64)
    rl, rg = orc.loglike_grad(sfh, th0, z0, obs0, sig0, masks0, path=1)
    m0 = orc.phot_exact(sfh, th0, z0)
    assert np.abs(m_all - m0[rep]).max() <= tol
    r = np.abs((m0 - obs0) / sig0) * ((masks0[:, None] >> np.arange(6)) & 1)
    assert np.all(np.abs(ll - rl[rep]) <= (r.sum(1)[rep] / 0.05) * tol + 1e-3)
    # per prototype, the propagation allowance of its largest magnitude difference over its copies
    dm_max = np.zeros((k, 6))
    np.maximum.at(dm_max, rep, np.abs(m_all - m0[rep]))
    prop, _ = grad_tol(orc, sfh, th0, z0, sig0, masks0, m0 + dm_max, path=1)
    ok = grad_ok(g, rg[rep], prop[rep])
    assert ok.all(), (np.argwhere(~ok)[:8], g[~ok][:8], rg[rep][~ok][:8])


@pytest.mark.parametrize("prec_name,tol", [("SPS_F32", 1e-4), ("SPS_BF16X", 2e-3)])
def test_exact_full_size_sampled(ctx5000, orc5000, prec_name, tol):
    # the benchmarked configuration: 4096 galaxies x 1128 SSPs x 5000 wavelengths (32 row
    # tiles, K split of the gradient GEMM, filter-support windows over random z); magnitudes,
    # log L and gradients of sampled galaxies against the oracle
    import paper_2506_19919_amd as sps
    n = 4096
    sfh, th, z = gal_inputs("dpl", n, 105)
    rng = np.random.default_rng(2)
    pick = np.sort(rng.choice(n, 6, replace=False))
    noise, sig = synth.photometric_noise(n, 6, 205)
    m_ref = orc5000.phot_exact(sfh, th[pick], z[pick])
    obs = f32(np.full((n, 6), 22.0))
    obs[pick] = f32(m_ref + noise[pick])
    sig = f32(sig)
    masks = synth.band_masks(n, 6, 5)
    prec = getattr(sps, prec_name)
    m_all = ctx5000.phot_exact(sfh, soa(th), dev(z), prec=prec).cpu().numpy()
    assert np.isfinite(m_all).all()
    assert np.abs(m_all[pick] - m_ref).max() <= tol
    ll, g = ctx5000.loglike_grad(sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8),
                                 path=sps.SPS_PATH_EXACT, prec=prec)
    ll, g = ll.cpu().numpy(), g.cpu().numpy().T.astype(np.float64)
    assert np.isfinite(ll).all() and np.isfinite(g).all()
    rl, rg = orc5000.loglike_grad(sfh, th[pick], z[pick], obs[pick], sig[pick], masks[pick], path=1)
    r = np.abs((m_ref - obs[pick]) / sig[pick]) * ((masks[pick][:, None] >> np.arange(6)) & 1)
    assert np.all(np.abs(ll[pick] - rl) <= (r.sum(1) / 0.05) * tol + 1e-3)
    prop, _ = grad_tol(orc5000, sfh, th[pick], z[pick], sig[pick], masks[pick], m_all[pick], path=1)
    ok = grad_ok(g[pick], rg, prop)
    assert ok.all(), (np.argwhere(~ok)[:8], g[pick][~ok][:8], rg[~ok][:8], prop[~ok][:8])


@pytest.mark.parametrize("prec_name,tol", [("SPS_F32", 1e-4), ("SPS_BF16X", 2e-3)])
def test_exact_lognormal_burst_forward_and_grad(ctx2000, orc, prec_name, tol):
    # the log-normal star-formation history with a burst through the FP32 / BF16X exact path
    import paper_2506_19919_amd as sps
    n = 150
    sfh, th, z = gal_inputs("lognormal_burst", n, 131)
    prec = getattr(sps, prec_name)
    m_ref = orc.phot_exact(sfh, th, z)
    m = ctx2000.phot_exact(sfh, soa(th), dev(z), prec=prec).cpu().numpy()
    assert np.abs(m - m_ref).max() <= tol
    k = 24
    noise, sig = synth.photometric_noise(k, 6, 132)
    obs, sig = f32(m_ref[:k] + noise), f32(sig)
    masks = synth.band_masks(k, 6, 133)
    ll, g = ctx2000.loglike_grad(sfh, soa(th[:k]), dev(z[:k]), dev(obs), dev(sig), dev(masks, torch.uint8),
                                 path=sps.SPS_PATH_EXACT, prec=prec)
    rl, rg = orc.loglike_grad(sfh, th[:k], z[:k], obs, sig, masks, path=1)
    ll, g = ll.cpu().numpy(), g.cpu().numpy().T.astype(np.float64)
    r = np.abs((m_ref[:k] - obs) / sig) * ((masks[:, None] >> np.arange(6)) & 1)
    assert np.all(np.abs(ll - rl) <= (r.sum(1) / 0.05) * tol + 1e-3)
    prop, _ = grad_tol(orc, sfh, th[:k], z[:k], sig, masks, m[:k], path=1)
    ok = grad_ok(g, rg, prop)
    assert ok.all(), (np.argwhere(~ok)[:8], g[~ok][:8], rg[~ok][:8], prop[~ok][:8])


@pytest.mark.parametrize("n", [1, 129])
@pytest.mark.parametrize("prec_name,tol", [("SPS_F32", 1e-4), ("SPS_BF16X", 2e-3)])
def test_exact_ragged_batches(ctx2000, orc, n, prec_name, tol):
    # one galaxy, and a second 128-galaxy row tile holding one galaxy: padded rows must not
    # leak into the real ones (forward and gradient)
    import paper_2506_19919_amd as sps
    sfh, th, z = gal_inputs("dpl", n, 400 + n)
    prec = getattr(sps, prec_name)
    m_ref = orc.phot_exact(sfh, th, z)
    m = ctx2000.phot_exact(sfh, soa(th), dev(z), prec=prec).cpu().numpy()
    assert np.abs(m - m_ref).max() <= tol
    noise, sig = synth.photometric_noise(n, 6, 500 + n)
    obs, sig = f32(m_ref + noise), f32(sig)
    masks = synth.band_masks(n, 6, 600 + n)
    ll, g = ctx2000.loglike_grad(sfh, soa(th), dev(z), dev(obs), dev(sig), dev(masks, torch.uint8),
                                 path=sps.SPS_PATH_EXACT, prec=prec)
    rl, rg = orc.loglike_grad(sfh, th, z, obs, sig, masks, path=1)
    ll, g = ll.cpu().numpy(), g.cpu().numpy().T.astype(np.float64)
    r = np.abs((m_ref - obs) / sig) * ((masks[:, None] >> np.arange(6)) & 1)
    assert np.all(np.abs(ll - rl) <= (r.sum(1) / 0.05) * tol + 1e-3)
    prop, _ = grad_tol(orc, sfh, th, z, sig, masks, m, path=1)
    ok = grad_ok(g, rg, prop)
    assert ok.all(), (np.argwhere(~ok)[:8], g[~ok][:8], rg[~ok][:8], prop[~ok][:8])


def test_exact_matches_approx_at_z_nodes_without_dust(ctx2000, orc):
    # both GPU paths reduce to the same sum when the attenuation is flat (tau_V = 0)
    import paper_2506_19919_amd as sps
    sfh, th, _ = gal_inputs("dpl", 40, 77)
    th[:, synth.P_TAUV] = 0.0
    z = f32(0.1 + 2.9 * (np.arange(40) % 63) / 63)
    ctx2000.build_ztable(64, 0.1, 3.0)
    me = ctx2000.phot_exact(sfh, soa(th), dev(z), prec=sps.SPS_F32).cpu().numpy()
    ma = ctx2000.phot_approx(sfh, soa(th), dev(z)).cpu().numpy()
    assert np.abs(me - ma).max() <= 2e-4


def test_exact_precision_not_uploaded_is_an_error(ssp2000, filt6):
    import paper_2506_19919_amd as sps
    c = sps.Context(ssp2000, filt6, precisions=(sps.SPS_F64,), max_gal=16, max_exact=16)
    sfh, th, z = gal_inputs("dpl", 4, 1)
    with pytest.raises(sps.SpsError) as e:
        c.phot_exact(sfh, soa(th), dev(z), prec=sps.SPS_BF16X)
    assert e.value.code == sps.SPS_E_STATE
    c.close()


@pytest.mark.parametrize("sigma_A", [200.0, 800.0])
def test_approximation_gap_matches_oracle(ssp2000, oracle_mod, sigma_A):
    # the approximate-minus-exact magnitude gap (App. B) measured on the GPU equals the
    # oracle's per galaxy and band: each FP32 path is within 1e-4 mag of the oracle
    import paper_2506_19919_amd as sps
    filt = synth.filters(sigma=sigma_A)
    c = sps.Context(ssp2000, filt, precisions=(sps.SPS_F32,), max_gal=4096, max_exact=4096)
    try:
        c.build_ztable(64, 0.1, 3.0)
        o = oracle_mod.Oracle(ssp2000, filt)
        o.build_ztable(64, 0.1, 3.0)
        sfh, th, z = gal_inputs("dpl", 96, 72)
        ma = c.phot_approx(sfh, soa(th), dev(z)).cpu().numpy().astype(np.float64)
        me = c.phot_exact(sfh, soa(th), dev(z), prec=sps.SPS_F32).cpu().numpy().astype(np.float64)
        ref = o.phot_approx(sfh, th, z) - o.phot_exact(sfh, th, z)
        assert np.abs((ma - me) - ref).max() <= 2e-4
    finally:
        c.close()


@pytest.mark.gpu
@pytest.mark.parametrize("tau_v", [0.0, 4.0])
def test_approximation_gap_against_dust_matches_oracle(ssp2000, filt6, oracle_mod, tau_v):
    # the tau_V axis of the approximation study (App. B): the GPU's approximate-minus-exact gap
    # equals the oracle's per galaxy and band with every galaxy at one optical depth
    import paper_2506_19919_amd as sps
    c = sps.Context(ssp2000, filt6, precisions=(sps.SPS_F32,), max_gal=4096, max_exact=4096)
    try:
        c.build_ztable(64, 0.1, 3.0)
        o = oracle_mod.Oracle(ssp2000, filt6)
        o.build_ztable(64, 0.1, 3.0)
        sfh, th, z = gal_inputs("dpl", 96, 74)
        th[:, synth.P_TAUV] = tau_v
        ma = c.phot_approx(sfh, soa(th), dev(z)).cpu().numpy().astype(np.float64)
        me = c.phot_exact(sfh, soa(th), dev(z), prec=sps.SPS_F32).cpu().numpy().astype(np.float64)
        ref = o.phot_approx(sfh, th, z) - o.phot_exact(sfh, th, z)
        assert np.abs((ma - me) - ref).max() <= 2e-4
    finally:
        c.close()


def test_exact_call_beyond_the_reservation_is_refused(ssp2000, filt6):
    # compute calls never allocate: a batch larger than sps_reserve_exact sized the workspace
    # for is an error, and reserving more makes the same call work
    import paper_2506_19919_amd as sps
    c = sps.Context(ssp2000, filt6, precisions=(sps.SPS_F32,), max_gal=256, max_exact=64)
    try:
        sfh, th, z = gal_inputs("dpl", 65, 3)
        with pytest.raises(sps.SpsError) as e:
            c.phot_exact(sfh, soa(th), dev(z), prec=sps.SPS_F32)
        assert e.value.code == sps.SPS_E_STATE
        c.reserve_exact(65)
        m = c.phot_exact(sfh, soa(th), dev(z), prec=sps.SPS_F32)
        assert torch.isfinite(m).all()
    finally:
        c.close()
