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


def grad_tol(orc, sfh, th, z, sig, masks, m_gpu, path=0, rtol=1e-3):
    """Per-component gradient tolerance: rtol relative, plus the first-order propagation of
    the measured magnitude difference through the oracle's Jacobian.

    d logL / d theta_p = -sum_b mask_b (m_b - d_b) / s_b^2  dm_b/dtheta_p, so a magnitude error
    dm_b moves the gradient by sum_b mask_b |dm_b| / s_b^2 |J_bp|; near the posterior mode the
    band sum cancels and this term, not rtol, bounds the agreement of an FP32 path.  The 2e-6
    added to |dm_b| is the rounding of an FP32 magnitude near 25 mag."""
    m_ref, jac = orc.mags_jacobian(sfh, th, z, path=path)
    bits = (np.asarray(masks)[:, None] >> np.arange(m_ref.shape[1])) & 1
    dm = (np.abs(np.asarray(m_gpu, np.float64) - m_ref) + 2e-6) * bits / np.asarray(sig) ** 2
    prop = np.einsum("gb,gbp->gp", dm, np.abs(jac))
    return prop, m_ref


def grad_ok(g, ref, prop, rtol=1e-3):
    return np.abs(g - ref) <= rtol * np.abs(ref) + prop + 1e-6 * np.abs(ref).max(axis=1, keepdims=True)


def general_bounds_prior(x_mid):
    """Bounds with k != 1 and x0 != 0 and skew-normal priors with s != 0 (App. C).

    x_mid [10]: typical unbounded values of the galaxies (for k = 1, x0 = 0); the prior of
    parameter 9 is centred two widths below them with s = -4, so that s y < -5 and the
    far-tail branch of log Phi is taken for most galaxies."""
    k = np.array([0.5, 2.3, 1.0, 0.5, 2.3, 0.8, 1.7, 0.5, 2.3, 1.2])
    x0 = np.array([-1.0, 0.7, 0.0, 0.7, -1.0, 0.3, -0.5, 0.7, -1.0, 0.2])
    bnd = np.column_stack([synth.BOUNDS, k, x0])
    s = np.array([2.5, -4.0, 0.0, 1.5, -2.0, 3.0, -1.0, 2.5, -4.0, -4.0])
    om = np.array([1.5, 1.0, 2.0, 1.5, 1.0, 1.2, 1.5, 2.0, 1.0, 0.5])
    xi = np.array([0.3, -0.2, 0.0, 0.5, -0.4, 0.1, 0.0, -0.3, 0.2, 0.0])
    xi[9] = x_mid[9] - 2 * om[9]
    pri = np.column_stack([xi, om, s])
    return f32(bnd), f32(pri)


def bound_jacobian(bnd, th):
    """d theta / d x of the bounding map at theta: k (theta - lo)(hi - theta) / (hi - lo)."""
    return bnd[:, 2] * (th - bnd[:, 0]) * (bnd[:, 1] - th) / (bnd[:, 1] - bnd[:, 0])


# at most this fraction of chains may be cut short by a near tie: with |log u + dH| < 1e-2 and
# mostly accepted moves a chain meets one in about 2 % of its iterations, so 8 iterations cut
# ~15 % of chains; a quarter keeps the comparison from going vacuous
MAX_EXCUSED = 0.25


def draws_follow_oracle(s_gpu, ref, rtol=1e-3, tie=1e-2):
    """Per chain, whether the GPU's draws follow the oracle's on the same Philox stream.

    s_gpu [sample][chain][galaxy][10]; ref: the oracle's hmc_run output with keep_trace.
    A chain is checked draw by draw (|x - x*| <= rtol max(|x*|, 1) on every parameter) up to
    the first iteration whose Metropolis decision was a near tie in the oracle,
    |log u + H1 - H0| < tie: FP32 magnitudes move H1 - H0 by ~1e-3, enough to flip such a
    decision, after which the two chains legitimately part.  Returns (ok, excused), [chain][galaxy]:
    ok is False for a chain that differs before any near tie; excused marks chains cut short
    by a tie."""
    s_ref = ref["samples"]
    n_s = s_ref.shape[0]
    margin = ref["trace_margin"][-n_s:]                     # sampling iterations [s][c][g]
    n_w = ref["trace_margin"].shape[0] - n_s
    warm_tie = (np.abs(ref["trace_margin"][:n_w]) < tie).any(axis=0) if n_w else np.zeros(margin.shape[1:], bool)
    tie_at = np.abs(margin) < tie
    # iterations up to (excluding) the first tie are compared
    before = np.cumsum(tie_at, axis=0) == 0
    close = np.all(np.abs(s_gpu - s_ref) <= rtol * np.maximum(np.abs(s_ref), 1.0), axis=-1)
    ok = np.all(close | ~before, axis=0) | warm_tie
    excused = warm_tie | tie_at.any(axis=0)
    return ok, excused
