"""The allocation-free likelihood entry point (sps_loglike_grad_static) against the ordinary
one (sps_loglike_grad, approximate path): the same kernels on the same inputs, so the same
bits, on two calls in a row, the second with a smaller batch (the static scratch keeps the
first call's contents); sizes above its limit are refused."""
import numpy as np
import pytest
import torch

import synth
from gpu_common import dev, f32, gal_inputs, soa

pytestmark = pytest.mark.gpu


def _inputs(orc, n, seed):
    sfh, th, z = gal_inputs("dpl", n, seed)
    noise, sig = synth.photometric_noise(n, 6, seed + 1)
    obs = f32(orc.phot_approx(sfh, th, z) + noise)
    mask = synth.band_masks(n, 6, seed + 2)
    return sfh, soa(th), dev(z), dev(obs), dev(f32(sig)), dev(mask, torch.uint8)


def test_static_entry_point_matches_the_allocating_one(ssp2000, filt6, orc):
    import paper_2506_19919_amd as sps
    c = sps.Context(ssp2000, filt6, precisions=(sps.SPS_F64,), max_gal=1 << 15)
    try:
        c.build_ztable(64, 0.1, 3.0)
        for n, seed in ((20_000, 801), (3_001, 802)):
            args = _inputs(orc, n, seed)
            ref_l, ref_g = c.loglike_grad(*args)
            got_l, got_g = c.loglike_grad_static(*args)
            torch.cuda.synchronize()
            assert torch.equal(got_l, ref_l) and torch.equal(got_g, ref_g), n
            assert torch.isfinite(got_l).all()
            val = c.loglike_grad_static(*args, grad=False)
            assert torch.equal(val, ref_l)
        big = sps.STATIC_MAX_GAL + 1
        sfh, th, z = gal_inputs("dpl", big, 803)
        ones = torch.ones((big, 6), dtype=torch.float32, device="cuda")
        with pytest.raises(sps.SpsError) as e:
            c.loglike_grad_static(sfh, soa(th), dev(z), 20.0 * ones, 0.05 * ones,
                                  torch.full((big,), 63, dtype=torch.uint8, device="cuda"))
        assert e.value.code == sps.SPS_E_INVAL
    finally:
        c.close()
