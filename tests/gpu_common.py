"""Shared helpers for the GPU parity tests: the same seeded float32 inputs go to
the HIP library and to the FP64 oracle."""
import numpy as np
import torch

import synth


def f32(a):
    """Round to float32 and back, so both sides see identical input values."""
    return np.asarray(a, np.float32).astype(np.float64)


def gal_inputs(kind, n, seed):
    if kind == "dpl":
        th, z = synth.galaxies_dpl(n, seed)
        sfh = synth.SFH_DPL
    else:
        th, z = synth.galaxies_lognormal(n, seed, burst=(kind == "lognormal_burst"))
        sfh = synth.SFH_LOGNORMAL
    return sfh, f32(th), f32(z)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda()


def soa(th, dtype=torch.float32):
    return dev(np.ascontiguousarray(th.T), dtype)


def bounds_prior():
    bnd = np.column_stack([synth.BOUNDS, np.ones(10), np.zeros(10)])
    pri = np.column_stack([np.zeros(10), np.full(10, 1.5), np.zeros(10)])
    return f32(bnd), f32(pri)


def grad_vec_ok(g, ref, rtol=1e-3):
    """Per galaxy (rows): max_p |g - ref| <= rtol * max_p |ref|  (max-norm relative error)."""
    return np.abs(g - ref).max(axis=1) <= rtol * np.abs(ref).max(axis=1)


def grad_close(g, ref, rtol=1e-3, floor=1e-3):
    """|g - ref| <= rtol * max(|ref|, floor * max_p |ref_p|) per galaxy (rows = galaxies)."""
    scale = np.maximum(np.abs(ref), floor * np.abs(ref).max(axis=1, keepdims=True))
    return np.abs(g - ref) <= rtol * scale
