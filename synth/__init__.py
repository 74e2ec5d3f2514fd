"""Seeded synthetic inputs for the SPS photometry / likelihood / HMC workloads.

This module only *draws inputs*: it holds none of the forward model's arithmetic
(no SFH integrals, no photometry, no likelihood).  Both the FP64 oracle (tests)
and the HIP library (tests, benchmark) consume exactly these arrays.

Stand-ins (the paper's MIST SSP grid, its filter curves and its simulated
galaxy sample are not available):

* SSP grid: 12 metallicities log10(Z/Zsun) uniform in [-2, 0.4], 94 log10 ages
  uniform in [5.5, 10.15] yr, log-spaced wavelengths 100 A .. 1e5 A.  Each
  spectrum is a luminosity-scaled mix of two unit-bolometric Planck curves whose
  temperatures fall with age and rise with Z, times 5% lognormal noise.
* Filters: Gaussian transmission (peak 1) centred log-uniformly on 3600..9700 A,
  sigma 400 A (the paper's synthetic-band experiments use Gaussian bands too).
* Galaxies: uniform draws of the 10 free parameters (slot order below) and z.

Parameter slot order (physical units), shared by every entry point:
  0 log10 M_formed [Msun]
  1 tau [Gyr]      (double power law)  | t_peak [Gyr]  (log-normal SFH)
  2 alpha          (double power law)  | width w [ln]  (log-normal SFH)
  3 beta           (double power law)  | unused        (log-normal SFH)
  4 F_burst
  5 log10 T_peak [yr] of the burst
  6 mu_logZ  (median log10 Z/Zsun of the metallicity distribution)
  7 tau_V    (V-band optical depth)
  8 delta    (power-law slope of the attenuation curve)
  9 F_floor  (unobscured sight-line fraction)
"""
from __future__ import annotations

import numpy as np

N_PARAM = 10
(P_LOGM, P_TAU, P_ALPHA, P_BETA, P_FBURST, P_LOGTPEAK,
 P_MUZ, P_TAUV, P_DELTA, P_FFLOOR) = range(N_PARAM)
PARAM_NAMES = ("log10M", "tau", "alpha", "beta", "F_burst", "log10T_peak",
               "mu_logZ", "tau_V", "delta", "F_floor")

SFH_LOGNORMAL = 0
SFH_DPL = 1

H0 = 70.0
OM = 0.3

# Bounding-function ranges (y_lo, y_hi) for the double-power-law model; k = 1, x0 = 0.
BOUNDS = np.array([
    [8.0, 12.5],    # log10 M
    [0.1, 14.0],    # tau [Gyr]
    [0.1, 8.0],     # alpha
    [0.1, 8.0],     # beta
    [0.0, 0.2],     # F_burst
    [4.5, 8.5],     # log10 T_peak
    [-2.0, 0.4],    # mu_logZ
    [0.0, 4.0],     # tau_V
    [-1.5, 0.0],    # delta
    [0.0, 0.5],     # F_floor
])


def ssp_grid(n_wave: int = 2000, seed: int = 1, noise: float = 0.05):
    """Synthetic SSP luminosity grid L[met][age][wave] in Lsun / A per Msun formed.

    ``noise`` is the lognormal scatter (0 gives smooth noise-free spectra)."""
    log10_met = -2.0 + 2.4 * np.arange(12) / 11.0
    log10_age = 5.5 + 0.05 * np.arange(94)
    wave = 10.0 ** (2.0 + 3.0 * np.arange(n_wave) / (n_wave - 1))
    zeta = log10_met[:, None, None]
    a = log10_age[None, :, None]
    lam = wave[None, None, :]
    t_hot = 10.0 ** (4.6 - 0.22 * (a - 5.5)) * (1.0 + 0.05 * zeta)
    t_cold = 10.0 ** (3.75 - 0.05 * (a - 5.5)) * (1.0 + 0.05 * zeta)
    f_hot = 1.0 / (1.0 + 10.0 ** (a - 8.0))
    l_bol = 10.0 ** (3.0 - 0.8 * (a - 5.5))

    def planck_unit(t):  # unit-bolometric Planck curve per A
        x = 1.438777e8 / (lam * t)
        with np.errstate(over="ignore"):
            return (15.0 / np.pi ** 4) * x ** 4 / (lam * np.expm1(x))

    lum = l_bol * (f_hot * planck_unit(t_hot) + (1.0 - f_hot) * planck_unit(t_cold))
    noise_draw = np.random.default_rng(seed).standard_normal((12, 94, n_wave))
    lum = lum * np.exp(noise * noise_draw)
    return dict(log10_met=log10_met, log10_age_yr=log10_age, wave_A=wave,
                lum=np.ascontiguousarray(lum))


def filters(n_band: int = 6, lo: float = 3600.0, hi: float = 9700.0, sigma: float = 400.0):
    """Gaussian filter descriptors (observed-frame centre and width, in A)."""
    b = np.arange(n_band)
    centre = lo * (hi / lo) ** (b / (n_band - 1)) if n_band > 1 else np.array([lo])
    return dict(center_A=np.asarray(centre, float), sigma_A=np.full(n_band, float(sigma)))


def _u(rng, lo, hi, n):
    return rng.uniform(lo, hi, n)


def galaxies_lognormal(n: int, seed: int, burst: bool):
    """Log-normal SFH galaxies (exact / approximate forward workloads).

    Returns (theta [n][10] float64, z [n] float64)."""
    rng = np.random.default_rng(seed)
    th = np.zeros((n, N_PARAM))
    z = _u(rng, 0.1, 3.0, n)
    th[:, P_TAU] = _u(rng, 1.0, 12.0, n)         # peak time [Gyr]
    th[:, P_ALPHA] = _u(rng, 0.2, 1.5, n)        # width [natural log]
    th[:, P_LOGM] = _u(rng, 9.0, 11.5, n)
    th[:, P_MUZ] = _u(rng, -1.5, 0.2, n)
    th[:, P_TAUV] = _u(rng, 0.0, 2.0, n)
    th[:, P_DELTA] = -0.7
    if burst:
        th[:, P_FBURST] = _u(rng, 0.0, 0.1, n)
        th[:, P_LOGTPEAK] = _u(rng, 5.0, 8.0, n)
    else:
        th[:, P_LOGTPEAK] = 7.0
    return th, z


def galaxies_dpl(n: int, seed: int):
    """Double-power-law SFH galaxies (likelihood, HMC and exact value+grad workloads)."""
    rng = np.random.default_rng(seed)
    th = np.zeros((n, N_PARAM))
    z = _u(rng, 0.1, 3.0, n)
    th[:, P_LOGM] = _u(rng, 9.0, 11.5, n)
    th[:, P_TAU] = _u(rng, 1.0, 12.0, n)
    th[:, P_ALPHA] = _u(rng, 0.5, 5.0, n)
    th[:, P_BETA] = _u(rng, 0.5, 5.0, n)
    th[:, P_FBURST] = _u(rng, 0.0, 0.1, n)
    th[:, P_LOGTPEAK] = _u(rng, 5.0, 8.0, n)
    th[:, P_MUZ] = _u(rng, -1.5, 0.2, n)
    th[:, P_TAUV] = _u(rng, 0.0, 2.0, n)
    th[:, P_DELTA] = _u(rng, -1.0, -0.4, n)
    th[:, P_FFLOOR] = _u(rng, 0.0, 0.3, n)
    return th, z


def photometric_noise(n: int, n_band: int, seed: int, sigma: float = 0.05):
    """Gaussian magnitude noise draws N(0, sigma^2) and the per-band sigma array."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, sigma, (n, n_band)), np.full((n, n_band), sigma)


def band_masks(n: int, n_band: int, seed: int, lo: int = 3, hi: int = 6):
    """Per-galaxy bitmask of observed bands: a random subset of lo..hi bands."""
    rng = np.random.default_rng(seed)
    masks = np.zeros(n, np.uint8)
    counts = rng.integers(lo, hi + 1, n)
    for g in range(n):
        sel = rng.permutation(n_band)[:counts[g]]
        masks[g] = np.bitwise_or.reduce(1 << sel)
    return masks


# Skew-normal prior (xi, omega, s) on each unbounded parameter: the s = 0 case (a
# Gaussian of width 1.5 in the unbounded coordinate) for every parameter.
PRIOR = np.array([[0.0, 1.5, 0.0]] * N_PARAM)


def bounds_k_x0() -> np.ndarray:
    """Bounding-function hyper-parameters [10][4] = (y_lo, y_hi, k = 1, x0 = 0)."""
    return np.column_stack([BOUNDS, np.ones(N_PARAM), np.zeros(N_PARAM)])


def prior_draws(n_chain: int, n: int, seed: int) -> np.ndarray:
    """Chain starting points drawn from PRIOR: [n_chain][10][n] unbounded values."""
    rng = np.random.default_rng(seed)
    return rng.normal(PRIOR[:, 0][None, :, None], PRIOR[:, 1][None, :, None], (n_chain, N_PARAM, n))


def soa32(theta: np.ndarray) -> np.ndarray:
    """[n][10] float64 -> [10][n] float32 (the device layout)."""
    return np.ascontiguousarray(theta.T.astype(np.float32))


# Named workloads (shapes, seeds, value ranges).
WORKLOADS = {
    "exact_fwd_f64": dict(n_gal=64, n_wave=2000, sfh=SFH_LOGNORMAL, seed=101, burst=False),
    "approx_fwd_f32": dict(n_gal=100_000, n_wave=2000, sfh=SFH_LOGNORMAL, seed=102, burst=True),
    "loglike_grad_f32": dict(n_gal=1_000_000, n_wave=2000, sfh=SFH_DPL, seed=103, noise_seed=203),
    "hmc_f32": dict(n_gal=16_384, n_chain=4, n_wave=2000, sfh=SFH_DPL, seed=104, mask_seed=204,
                    init_seed=304, philox_seed=404, n_leapfrog=10, n_warmup=200, n_sample=1000),
    "exact_grad_bf16x": dict(n_gal=4096, n_wave=5000, sfh=SFH_DPL, seed=105, noise_seed=205),
}
