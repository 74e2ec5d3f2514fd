"""Launch choices that must not change any result (tile order, XCD placement, iterations per
launch, graph replay of the exact-path HMC iteration), graph replays interleaved with eager
work, and the autotuner's choice and cache."""
import json
import os

import numpy as np
import pytest
import torch

import synth
from gpu_common import bounds_prior, dev, f32, gal_inputs, soa

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(ssp2000, filt6):
    import paper_2506_19919_amd as sps
    c = sps.Context(ssp2000, filt6, precisions=(sps.SPS_F32, sps.SPS_BF16X), max_gal=1 << 13, max_exact=1 << 12)
    c.build_ztable(64, 0.1, 3.0)
    c.reserve_nuts(1 << 12, 6)
    default = c.get_launch()
    yield c
    c.set_launch(**default)
    c.close()


def _lik_inputs(orc, n, seed):
    sfh, th, z = gal_inputs("dpl", n, seed)
    noise, sig = synth.photometric_noise(n, 6, seed + 1)
    obs = f32(orc.phot_approx(sfh, th, z) + noise)
    return sfh, soa(th), dev(z), dev(obs), dev(f32(sig)), dev(synth.band_masks(n, 6, seed + 2), torch.uint8)


def _chain_inputs(orc, n, seed, C):
    sfh, th, z = gal_inputs("dpl", n, seed)
    noise, sig = synth.photometric_noise(n, 6, seed + 1)
    obs = f32(orc.phot_approx(sfh, th, z) + noise)
    bnd, pri = bounds_prior()
    xt = np.array([[orc.unbound(bnd[p], th[g, p]) for p in range(10)] for g in range(n)])
    x0 = f32(xt[None] + 0.05 * np.random.default_rng(seed + 3).normal(size=(C, n, 10)))
    return (sfh, dev(z), dev(obs), dev(f32(sig)), dev(synth.band_masks(n, 6, seed + 2), torch.uint8), dev(bnd),
            dev(pri), dev(np.ascontiguousarray(np.transpose(x0, (0, 2, 1)))))


@pytest.mark.parametrize("prec_name", ["SPS_F32", "SPS_BF16X"])
def test_exact_tile_orders_give_the_same_bits(ctx, orc, prec_name):
    import paper_2506_19919_amd as sps
    prec = getattr(sps, prec_name)
    sfh, p, z, obs, sig, mask = _lik_inputs(orc, 700, 901)
    ref = None
    for ring in ((0, 1) if prec == sps.SPS_BF16X else (0,)):
        for order in (0, 1, 2, 3):
            for xcd in (1, 0):
                ctx.set_launch(exact_order=order, exact_xcd=xcd, exact_ring=ring)
                ll, g = ctx.loglike_grad(sfh, p, z, obs, sig, mask, path=sps.SPS_PATH_EXACT, prec=prec)
                m = ctx.phot_exact(sfh, p, z, prec=prec)
                got = (ll.clone(), g.clone(), m.clone())
                if ref is None:
                    ref = got
                    assert torch.isfinite(ll).all()
                else:
                    assert all(torch.equal(a, b) for a, b in zip(got, ref)), (ring, order, xcd)
    ctx.set_launch(exact_order=0, exact_xcd=1, exact_ring=0)


def test_hmc_block_iterations_give_the_same_draws(ctx, orc):
    args = _chain_inputs(orc, 40, 911, 3)
    kw = dict(n_chain=3, n_leapfrog=5, n_warmup=12, n_sample=9, init_step=0.02, seed=17, keep_samples=True)
    out = []
    for b in (25, 4, 1):
        ctx.set_launch(hmc_block_iters=b)
        out.append(ctx.hmc_run(*args, **kw))
    ctx.set_launch(hmc_block_iters=25)
    for o in out[1:]:
        for k in ("samples", "post_mean", "step", "accept"):
            assert torch.equal(o[k], out[0][k]), k


def test_nuts_block_iterations_give_the_same_draws(ctx, orc):
    args = _chain_inputs(orc, 24, 921, 2)
    kw = dict(n_chain=2, max_depth=6, n_warmup=6, n_sample=7, init_step=0.03, seed=18, keep_samples=True,
              keep_depth=True)
    out = []
    for b in (10, 3):
        ctx.set_launch(nuts_block_iters=b)
        out.append(ctx.nuts_run(*args, **kw))
    ctx.set_launch(nuts_block_iters=10)
    for k in ("samples", "depth", "n_leaf", "step"):
        assert torch.equal(out[1][k], out[0][k]), k


def test_exact_hmc_graph_replay_matches_eager_launches(ctx, orc):
    # one captured iteration replayed per iteration (graph on) against the kernels launched one
    # by one (graph off): the same draws; then the graph run split over three calls with eager
    # work and synchronisations between them (every call re-captures and replays)
    import paper_2506_19919_amd as sps
    n, C = 48, 3
    args = _chain_inputs(orc, n, 931, C)
    kw = dict(n_chain=C, n_leapfrog=4, n_warmup=6, n_sample=6, init_step=0.02, seed=19,
              path=sps.SPS_PATH_EXACT, prec=sps.SPS_BF16X)
    ctx.set_launch(hmcx_graph=0)
    eager = ctx.hmc_run(*args, keep_samples=True, **kw)
    ctx.set_launch(hmcx_graph=1)
    graph = ctx.hmc_run(*args, keep_samples=True, **kw)
    for k in ("samples", "post_mean", "post_sd", "step", "accept"):
        assert torch.equal(graph[k], eager[k]), k
    state = ctx.hmc_state(n, C)
    samples = torch.zeros_like(eager["samples"])
    lik = _lik_inputs(orc, 300, 932)
    for b, e in ((0, 4), (4, 9), (9, 12)):
        part = ctx.hmc_run(*args, it_begin=b, it_end=e, state=state, samples=samples, **kw)
        ctx.loglike_grad(*lik)                  # eager work between the replays
        torch.cuda.synchronize()
        ref = eager["samples"][: max(e - 6, 0)]
        assert torch.equal(samples[: max(e - 6, 0)], ref), (b, e)
    for k in ("post_mean", "post_sd", "step"):
        assert torch.equal(part[k], eager[k]), k


def test_autotuner_picks_and_caches(ctx, orc, tmp_path):
    import paper_2506_19919_amd as sps
    path = tmp_path / "tune.json"
    old = os.environ.get("SPS_AUTOTUNE_CACHE")
    os.environ["SPS_AUTOTUNE_CACHE"] = str(path)
    try:
        sfh, p, z, obs, sig, mask = _lik_inputs(orc, 512, 941)
        ch, ms = ctx.autotune_exact(sfh, p, z, obs, sig, mask, prec=sps.SPS_BF16X)
        assert ms > 0 and ctx.get_launch()["exact_order"] == ch["exact_order"]
        entries = json.loads(path.read_text())
        (key, val), = entries.items()
        assert key.startswith("exact|") and val["exact_order"] == ch["exact_order"] and val["ms"] > 0
        ctx.set_launch(exact_order=0, exact_xcd=1, exact_ring=0)
        ch2, ms2 = ctx.autotune_exact(sfh, p, z, obs, sig, mask, prec=sps.SPS_BF16X)
        assert ms2 == 0 and ch2 == ch                     # from the cache, not timed again
        args = _chain_inputs(orc, 32, 942, 2)
        chh, msh = ctx.autotune_hmc(*args, n_chain=2, n_leapfrog=3, n_warmup=4, n_sample=4,
                                    path=sps.SPS_PATH_EXACT, prec=sps.SPS_BF16X)
        assert msh > 0 and chh["hmcx_graph"] in (0, 1)
        chh2, _ = ctx.autotune_hmc(*args, n_chain=2, n_leapfrog=3, n_warmup=4, n_sample=60)
        assert chh2["hmc_block_iters"] in (5, 10, 25, 50)
        assert len(json.loads(path.read_text())) == 3
    finally:
        if old is None:
            del os.environ["SPS_AUTOTUNE_CACHE"]
        else:
            os.environ["SPS_AUTOTUNE_CACHE"] = old
        ctx.set_launch(exact_order=0, exact_xcd=1, hmc_block_iters=25, hmcx_graph=1, exact_ring=0)


def test_launch_choices_out_of_range_are_refused(ctx):
    import paper_2506_19919_amd as sps
    for bad in (dict(exact_order=4), dict(exact_xcd=2), dict(exact_ring=2), dict(hmc_block_iters=0),
                dict(nuts_block_iters=1001), dict(hmcx_graph=-1)):
        with pytest.raises(sps.SpsError) as e:
            ctx.set_launch(**bad)
        assert e.value.code == sps.SPS_E_INVAL
