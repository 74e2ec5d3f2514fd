"""MI355X-native SPS photometry, likelihood and HMC (binding of libsps.so).

Thin marshalling layer over the C ABI declared in include/sps.h: every step of
the computation runs in the library's HIP kernels.  PyTorch supplies device
memory (tensors) and the current HIP stream.  The library must have been built
(``python paper_2506_19919_amd/build.py``); importing this module on a machine
without it raises immediately.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsps.so")

SPS_OK, SPS_E_INVAL, SPS_E_RANGE, SPS_E_NOMEM, SPS_E_HIP, SPS_E_STATE = range(6)
SPS_F64, SPS_F32, SPS_BF16X = 0, 1, 2
SPS_SFH_LOGNORMAL, SPS_SFH_DPL = 0, 1
SPS_PATH_APPROX, SPS_PATH_EXACT = 0, 1
NPARAM = 10
MAX_BAND = 8

STATIC_MAX_GAL = 32768   # SPS_STATIC_MAX_GAL of include/sps.h

ABI_FUNCTIONS = ("sps_create", "sps_reserve", "sps_reserve_exact", "sps_status", "sps_build_ztable",
                 "sps_get_ztable", "sps_destroy", "sps_last_error", "sps_weights", "sps_phot_approx",
                 "sps_phot_exact", "sps_loglike_grad", "sps_logpost_grad", "sps_hmc_run", "sps_hmc_state_bytes",
                 "sps_set_kernel_timing", "sps_kernel_times", "sps_nuts_run", "sps_reserve_nuts",
                 "sps_loglike_grad_static", "sps_get_launch", "sps_set_launch", "sps_autotune_exact",
                 "sps_autotune_hmc", "sps_phot_vjp")


class SpsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sps error {code}: {msg}")
        self.code = code


class _SspDesc(C.Structure):
    _fields_ = [("n_met", C.c_int), ("n_age", C.c_int), ("n_wave", C.c_int),
                ("log10_met", C.POINTER(C.c_double)), ("log10_age_yr", C.POINTER(C.c_double)),
                ("wave_A", C.POINTER(C.c_double)), ("lum", C.POINTER(C.c_double))]


class _FilterDesc(C.Structure):
    _fields_ = [("n_band", C.c_int), ("center_A", C.POINTER(C.c_double)),
                ("sigma_A", C.POINTER(C.c_double))]


class _ModelDesc(C.Structure):
    _fields_ = [("H0", C.c_double), ("Om", C.c_double), ("sigma_logz", C.c_double),
                ("burst_dlogt", C.c_double)]


class _HmcCfg(C.Structure):
    _fields_ = [("n_chain", C.c_int), ("n_leapfrog", C.c_int), ("n_warmup", C.c_int),
                ("n_sample", C.c_int), ("target_accept", C.c_float), ("init_step", C.c_float),
                ("seed", C.c_ulonglong), ("adapt_metric", C.c_int), ("path", C.c_int), ("prec", C.c_int),
                ("it_begin", C.c_int), ("it_end", C.c_int)]


class _NutsCfg(C.Structure):
    _fields_ = [("n_chain", C.c_int), ("max_depth", C.c_int), ("n_warmup", C.c_int),
                ("n_sample", C.c_int), ("target_accept", C.c_float), ("init_step", C.c_float),
                ("seed", C.c_ulonglong), ("adapt_metric", C.c_int), ("sync_iterations", C.c_int)]


class _LaunchCfg(C.Structure):
    _fields_ = [("exact_order", C.c_int), ("exact_xcd", C.c_int), ("hmc_block_iters", C.c_int),
                ("nuts_block_iters", C.c_int), ("hmcx_graph", C.c_int), ("exact_ring", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2506_19919_amd/build.py")
    lib = C.CDLL(LIB_PATH)
    vp, i = C.c_void_p, C.c_int
    lib.sps_last_error.restype = C.c_char_p
    lib.sps_last_error.argtypes = []
    lib.sps_create.argtypes = [C.POINTER(vp), i, C.POINTER(_SspDesc), C.POINTER(_FilterDesc),
                               C.POINTER(_ModelDesc), C.c_uint, i]
    lib.sps_reserve.argtypes = [vp, i]
    lib.sps_reserve_exact.argtypes = [vp, i]
    lib.sps_status.argtypes = [vp]
    lib.sps_hmc_state_bytes.argtypes = [i, i]
    lib.sps_hmc_state_bytes.restype = C.c_size_t
    lib.sps_build_ztable.argtypes = [vp, i, C.c_double, C.c_double]
    lib.sps_get_ztable.argtypes = [vp, vp]
    lib.sps_destroy.argtypes = [vp]
    lib.sps_destroy.restype = None
    lib.sps_weights.argtypes = [vp, vp, i, i, vp, vp, vp]
    lib.sps_phot_approx.argtypes = [vp, vp, i, i, vp, vp, vp]
    lib.sps_phot_exact.argtypes = [vp, vp, i, i, i, vp, vp, vp]
    lib.sps_loglike_grad.argtypes = [vp, vp, i, i, i, i, vp, vp, vp, vp, vp, vp, vp]
    lib.sps_logpost_grad.argtypes = [vp, vp, i, i, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.sps_hmc_run.argtypes = [vp, vp, C.POINTER(_HmcCfg), i, i, vp, vp, vp, vp, vp, vp, vp, vp,
                                vp, vp, vp, vp, vp, vp, vp]
    lib.sps_nuts_run.argtypes = [vp, vp, C.POINTER(_NutsCfg), i, i, vp, vp, vp, vp, vp, vp, vp, vp,
                                 vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.sps_reserve_nuts.argtypes = [vp, i, i]
    lib.sps_loglike_grad_static.argtypes = [vp, vp, i, i, vp, vp, vp, vp, vp, vp, vp]
    lib.sps_get_launch.argtypes = [vp, C.POINTER(_LaunchCfg)]
    lib.sps_set_launch.argtypes = [vp, C.POINTER(_LaunchCfg)]
    lib.sps_autotune_exact.argtypes = [vp, vp, i, i, i, vp, vp, vp, vp, vp, C.POINTER(_LaunchCfg),
                                       C.POINTER(C.c_float)]
    lib.sps_autotune_hmc.argtypes = [vp, vp, C.POINTER(_HmcCfg), i, i, vp, vp, vp, vp, vp, vp, vp,
                                     C.POINTER(_LaunchCfg), C.POINTER(C.c_float)]
    lib.sps_set_kernel_timing.argtypes = [vp, i]
    lib.sps_kernel_times.argtypes = [vp, vp, i, C.POINTER(i)]
    for name in ABI_FUNCTIONS:
        if name not in ("sps_destroy", "sps_last_error", "sps_hmc_state_bytes"):
            getattr(lib, name).restype = C.c_int
    return lib


_lib = _load()


def lib():
    return _lib


def _check(rc):
    if rc != SPS_OK:
        raise SpsError(rc, _lib.sps_last_error().decode())


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev(t, dtype, shape, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Context:
    """One library context: SSP grid, filters and model constants on one GPU."""

    def __init__(self, ssp: dict, filters: dict, model: dict | None = None, device: int = 0,
                 precisions=(SPS_F64, SPS_F32), max_gal: int = 1 << 20, max_exact: int = 0):
        m = dict(H0=70.0, Om=0.3, sigma_logz=0.2, burst_dlogt=0.3)
        m.update(model or {})
        self._keep = [np.ascontiguousarray(ssp[k], dtype=np.float64)
                      for k in ("log10_met", "log10_age_yr", "wave_A", "lum")]
        self._keep += [np.ascontiguousarray(filters[k], dtype=np.float64) for k in ("center_A", "sigma_A")]
        met, age, wave, lum, cen, sig = self._keep
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        sd = _SspDesc(len(met), len(age), len(wave), dp(met), dp(age), dp(wave), dp(lum))
        fd = _FilterDesc(len(cen), dp(cen), dp(sig))
        md = _ModelDesc(m["H0"], m["Om"], m["sigma_logz"], m["burst_dlogt"])
        mask = 0
        for p in precisions:
            mask |= 1 << p
        h = C.c_void_p()
        _check(_lib.sps_create(C.byref(h), device, C.byref(sd), C.byref(fd), C.byref(md), mask, max_gal))
        self.h = h
        self.device = torch.device("cuda", device)
        self.n_met, self.n_age, self.n_wave, self.n_band = len(met), len(age), len(wave), len(cen)
        self.max_gal = max_gal
        self.max_exact = 0
        self.ztable_spec = None
        if max_exact:
            self.reserve_exact(max_exact)

    def close(self):
        if getattr(self, "h", None):
            _lib.sps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- setup
    def reserve(self, max_gal: int):
        _check(_lib.sps_reserve(self.h, max_gal))
        self.max_gal = max(self.max_gal, max_gal)

    def reserve_exact(self, max_rows: int):
        """Size the exact path's workspace for calls of up to max_rows galaxies (or HMC chains)."""
        _check(_lib.sps_reserve_exact(self.h, max_rows))
        self.max_exact = max(self.max_exact, max_rows)
        self.max_gal = max(self.max_gal, max_rows)

    # ---- launch choices (none changes a result) and their autotuner
    def get_launch(self) -> dict:
        l = _LaunchCfg()
        _check(_lib.sps_get_launch(self.h, C.byref(l)))
        return l.as_dict()

    def set_launch(self, **kw):
        """Change some launch choices: exact_order, exact_xcd, hmc_block_iters, nuts_block_iters,
        hmcx_graph, exact_ring (see sps.h)."""
        l = _LaunchCfg(**{**self.get_launch(), **kw})
        _check(_lib.sps_set_launch(self.h, C.byref(l)))

    def autotune_exact(self, sfh, params, z, obs=None, sigma=None, mask=None, prec=SPS_BF16X, stream=None):
        """Time the exact path's tile orders on these inputs, keep the fastest; returns
        (choices, ms of the chosen one, 0 if it came from SPS_AUTOTUNE_CACHE)."""
        n = self._gal(params, z)
        l, ms = _LaunchCfg(), C.c_float(0)
        _check(_lib.sps_autotune_exact(self.h, _stream(stream), n, sfh, prec, _ptr(params), _ptr(z), _ptr(obs),
                                       _ptr(sigma), _ptr(mask), C.byref(l), C.byref(ms)))
        return l.as_dict(), ms.value

    def autotune_hmc(self, sfh, z, obs, sigma, mask, bounds, prior, theta0, n_chain=4, n_leapfrog=10,
                     n_warmup=200, n_sample=1000, target_accept=0.8, init_step=0.1, seed=404,
                     adapt_metric=False, path=SPS_PATH_APPROX, prec=SPS_F32, stream=None):
        """Time hmc_run's launch choice (iterations per launch, or graph replay on the exact
        path) on a short run of these inputs; returns (choices, ms or 0 if cached)."""
        n = z.shape[0]
        cfg = _HmcCfg(n_chain, n_leapfrog, n_warmup, n_sample, target_accept, init_step, seed,
                      int(bool(adapt_metric)), int(path), int(prec), 0, 0)
        l, ms = _LaunchCfg(), C.c_float(0)
        _check(_lib.sps_autotune_hmc(self.h, _stream(stream), C.byref(cfg), n, sfh, _ptr(z), _ptr(obs), _ptr(sigma),
                                     _ptr(mask), _ptr(bounds), _ptr(prior), _ptr(theta0), C.byref(l), C.byref(ms)))
        return l.as_dict(), ms.value

    def reserve_nuts(self, max_chains: int, max_depth: int = 10):
        """Size the NUTS workspace for up to max_chains chains (n_gal * n_chain) at max_depth."""
        _check(_lib.sps_reserve_nuts(self.h, max_chains, max_depth))
        self.max_gal = max(self.max_gal, max_chains)

    def status(self):
        """Synchronise and raise SpsError for device-side errors flagged since the last check
        (SPS_E_RANGE: a redshift outside the z table; SPS_E_STATE: a mismatched resume blob)."""
        _check(_lib.sps_status(self.h))

    def build_ztable(self, n_z: int = 64, z_lo: float = 0.1, z_hi: float = 3.0):
        _check(_lib.sps_build_ztable(self.h, n_z, C.c_double(z_lo), C.c_double(z_hi)))
        self.ztable_spec = (n_z, z_lo, z_hi)

    def get_ztable(self) -> np.ndarray:
        n_z = self.ztable_spec[0]
        q = np.zeros((n_z, self.n_band, self.n_met, self.n_age), np.float32)
        _check(_lib.sps_get_ztable(self.h, q.ctypes.data_as(C.c_void_p)))
        return q

    # ---- instrumentation
    def set_kernel_timing(self, n_pairs: int):
        """Record HIP events around the approximate path's model kernel in the next calls
        (cycling through n_pairs pairs; 0 turns it off)."""
        _check(_lib.sps_set_kernel_timing(self.h, n_pairs))
        self.timing_pairs = n_pairs

    def kernel_times(self) -> np.ndarray:
        """Milliseconds of the last recorded model-kernel launches, oldest first."""
        n = max(getattr(self, "timing_pairs", 0), 1)
        ms = np.zeros(n, np.float32)
        cnt = C.c_int(0)
        _check(_lib.sps_kernel_times(self.h, ms.ctypes.data_as(C.c_void_p), n, C.byref(cnt)))
        return ms[:cnt.value].copy()

    # ---- helpers
    def _gal(self, params, z, dtype=torch.float32):
        n = z.shape[0]
        _dev(params, dtype, (NPARAM, n), "params", self.device)
        _dev(z, dtype, (n,), "z", self.device)
        return n

    # ---- entry points (same names as the C ABI)
    def weights(self, sfh, params, z, out=None, stream=None):
        n = self._gal(params, z)
        if out is None:
            out = torch.empty((n, self.n_met, self.n_age), dtype=torch.float32, device=self.device)
        _dev(out, torch.float32, (n, self.n_met, self.n_age), "w_out", self.device)
        _check(_lib.sps_weights(self.h, _stream(stream), n, sfh, _ptr(params), _ptr(z), _ptr(out)))
        return out

    def phot_approx(self, sfh, params, z, out=None, stream=None):
        n = self._gal(params, z)
        if out is None:
            out = torch.empty((n, self.n_band), dtype=torch.float32, device=self.device)
        _dev(out, torch.float32, (n, self.n_band), "mag_out", self.device)
        _check(_lib.sps_phot_approx(self.h, _stream(stream), n, sfh, _ptr(params), _ptr(z), _ptr(out)))
        return out

    def phot_exact(self, sfh, params, z, prec=SPS_F32, out=None, stream=None):
        dt = torch.float64 if prec == SPS_F64 else torch.float32
        n = self._gal(params, z, dt)
        if out is None:
            out = torch.empty((n, self.n_band), dtype=dt, device=self.device)
        _dev(out, dt, (n, self.n_band), "mag_out", self.device)
        _check(_lib.sps_phot_exact(self.h, _stream(stream), n, sfh, prec, _ptr(params), _ptr(z), _ptr(out)))
        return out

    def loglike_grad(self, sfh, params, z, obs, sigma, mask, path=SPS_PATH_APPROX, prec=SPS_F32,
                     grad=True, logl_out=None, grad_out=None, stream=None):
        n = self._gal(params, z)
        _dev(obs, torch.float32, (n, self.n_band), "obs", self.device)
        _dev(sigma, torch.float32, (n, self.n_band), "sigma", self.device)
        _dev(mask, torch.uint8, (n,), "band_mask", self.device)
        if logl_out is None:
            logl_out = torch.empty(n, dtype=torch.float32, device=self.device)
        if grad and grad_out is None:
            grad_out = torch.empty((NPARAM, n), dtype=torch.float32, device=self.device)
        _check(_lib.sps_loglike_grad(self.h, _stream(stream), n, sfh, path, prec, _ptr(params), _ptr(z),
                                     _ptr(obs), _ptr(sigma), _ptr(mask), _ptr(logl_out),
                                     _ptr(grad_out) if grad else None))
        return (logl_out, grad_out) if grad else logl_out

    def phot_vjp(self, sfh, params, z, gbar, path=SPS_PATH_APPROX, prec=SPS_F32, grad_out=None, stream=None):
        """sum_b gbar[g][b] dm_b/dtheta_p for the 10 physical parameters, [10][n_gal]: the
        backward of the magnitudes (approximate path, or exact in SPS_F32 / SPS_BF16X)."""
        n = self._gal(params, z)
        _dev(gbar, torch.float32, (n, self.n_band), "gbar", self.device)
        if grad_out is None:
            grad_out = torch.empty((NPARAM, n), dtype=torch.float32, device=self.device)
        _check(_lib.sps_phot_vjp(self.h, _stream(stream), n, sfh, path, prec, _ptr(params), _ptr(z), _ptr(gbar),
                                 _ptr(grad_out)))
        return grad_out

    def loglike_grad_static(self, sfh, params, z, obs, sigma, mask, grad=True, logl_out=None, grad_out=None,
                            stream=None):
        """loglike_grad on the approximate path through the entry point that allocates nothing
        (its buffers are the library's static device array; n_gal <= STATIC_MAX_GAL)."""
        n = self._gal(params, z)
        _dev(obs, torch.float32, (n, self.n_band), "obs", self.device)
        _dev(sigma, torch.float32, (n, self.n_band), "sigma", self.device)
        _dev(mask, torch.uint8, (n,), "band_mask", self.device)
        if logl_out is None:
            logl_out = torch.empty(n, dtype=torch.float32, device=self.device)
        if grad and grad_out is None:
            grad_out = torch.empty((NPARAM, n), dtype=torch.float32, device=self.device)
        _check(_lib.sps_loglike_grad_static(self.h, _stream(stream), n, sfh, _ptr(params), _ptr(z), _ptr(obs),
                                            _ptr(sigma), _ptr(mask), _ptr(logl_out),
                                            _ptr(grad_out) if grad else None))
        return (logl_out, grad_out) if grad else logl_out

    def logpost_grad(self, sfh, x, z, obs, sigma, mask, bounds, prior, stream=None):
        n = self._gal(x, z)
        _dev(obs, torch.float32, (n, self.n_band), "obs", self.device)
        _dev(sigma, torch.float32, (n, self.n_band), "sigma", self.device)
        _dev(mask, torch.uint8, (n,), "band_mask", self.device)
        _dev(bounds, torch.float32, (NPARAM, 4), "bounds", self.device)
        _dev(prior, torch.float32, (NPARAM, 3), "prior", self.device)
        lp = torch.empty(n, dtype=torch.float32, device=self.device)
        g = torch.empty((NPARAM, n), dtype=torch.float32, device=self.device)
        _check(_lib.sps_logpost_grad(self.h, _stream(stream), n, sfh, _ptr(x), _ptr(z), _ptr(obs),
                                     _ptr(sigma), _ptr(mask), _ptr(bounds), _ptr(prior), _ptr(lp), _ptr(g)))
        return lp, g

    def hmc_state(self, n_gal, n_chain):
        """A device buffer for hmc_run's resume state (zero-filled)."""
        nbytes = _lib.sps_hmc_state_bytes(n_gal, n_chain)
        return torch.zeros(nbytes, dtype=torch.uint8, device=self.device)

    def hmc_run(self, sfh, z, obs, sigma, mask, bounds, prior, theta0, n_chain=4, n_leapfrog=10,
                n_warmup=200, n_sample=1000, target_accept=0.8, init_step=0.1, seed=404,
                keep_samples=False, adapt_metric=False, path=SPS_PATH_APPROX, prec=SPS_F32, stream=None,
                it_begin=0, it_end=0, state=None, samples=None):
        """theta0 [chain][10][galaxy] or None (prior draws).  A run split over calls passes
        it_begin / it_end, the same `state` (hmc_state) and, to collect every draw, the same
        `samples` tensor to each call; the summaries come from the call that ends the run."""
        n = z.shape[0]
        _dev(z, torch.float32, (n,), "z", self.device)
        _dev(obs, torch.float32, (n, self.n_band), "obs", self.device)
        _dev(sigma, torch.float32, (n, self.n_band), "sigma", self.device)
        _dev(mask, torch.uint8, (n,), "band_mask", self.device)
        _dev(bounds, torch.float32, (NPARAM, 4), "bounds", self.device)
        _dev(prior, torch.float32, (NPARAM, 3), "prior", self.device)
        if theta0 is not None:
            _dev(theta0, torch.float32, (n_chain, NPARAM, n), "theta0", self.device)
        if state is not None:
            _dev(state, torch.uint8, (_lib.sps_hmc_state_bytes(n, n_chain),), "state", self.device)
        f32 = dict(dtype=torch.float32, device=self.device)
        out = dict(post_mean=torch.empty((NPARAM, n), **f32), post_sd=torch.empty((NPARAM, n), **f32),
                   rhat=torch.empty((NPARAM, n), **f32), accept=torch.empty(n, **f32),
                   step=torch.empty((n_chain, n), **f32),
                   inv_metric=torch.empty((n_chain, NPARAM, n), **f32))
        if samples is not None:
            _dev(samples, torch.float32, (n_sample, n_chain, NPARAM, n), "samples", self.device)
        elif keep_samples:
            samples = torch.empty((n_sample, n_chain, NPARAM, n), **f32)
        cfg = _HmcCfg(n_chain, n_leapfrog, n_warmup, n_sample, target_accept, init_step, seed,
                      int(bool(adapt_metric)), int(path), int(prec), int(it_begin), int(it_end))
        _check(_lib.sps_hmc_run(self.h, _stream(stream), C.byref(cfg), n, sfh, _ptr(z), _ptr(obs),
                                _ptr(sigma), _ptr(mask), _ptr(bounds), _ptr(prior), _ptr(theta0),
                                _ptr(samples), _ptr(out["post_mean"]), _ptr(out["post_sd"]),
                                _ptr(out["rhat"]), _ptr(out["accept"]), _ptr(out["step"]),
                                _ptr(out["inv_metric"]), _ptr(state)))
        if samples is not None:
            out["samples"] = samples
        return out


    def nuts_run(self, sfh, z, obs, sigma, mask, bounds, prior, theta0, n_chain=4, max_depth=10,
                 n_warmup=200, n_sample=1000, target_accept=0.8, init_step=0.1, seed=404,
                 keep_samples=False, adapt_metric=False, sync_iterations=False, keep_depth=False, stream=None):
        """NUTS on the approximate path; theta0 [chain][10][galaxy] or None (prior draws).
        Returns the summaries, n_leaf [chain][galaxy] (leapfrog steps of each chain), lockstep
        (chain steps, wave steps x chains per wave) and optionally samples and depth."""
        n = z.shape[0]
        _dev(z, torch.float32, (n,), "z", self.device)
        _dev(obs, torch.float32, (n, self.n_band), "obs", self.device)
        _dev(sigma, torch.float32, (n, self.n_band), "sigma", self.device)
        _dev(mask, torch.uint8, (n,), "band_mask", self.device)
        _dev(bounds, torch.float32, (NPARAM, 4), "bounds", self.device)
        _dev(prior, torch.float32, (NPARAM, 3), "prior", self.device)
        if theta0 is not None:
            _dev(theta0, torch.float32, (n_chain, NPARAM, n), "theta0", self.device)
        f32 = dict(dtype=torch.float32, device=self.device)
        out = dict(post_mean=torch.empty((NPARAM, n), **f32), post_sd=torch.empty((NPARAM, n), **f32),
                   rhat=torch.empty((NPARAM, n), **f32), accept=torch.empty(n, **f32),
                   step=torch.empty((n_chain, n), **f32),
                   inv_metric=torch.empty((n_chain, NPARAM, n), **f32),
                   n_leaf=torch.empty((n_chain, n), dtype=torch.int32, device=self.device),
                   lockstep=torch.zeros(2, dtype=torch.int64, device=self.device))
        if keep_samples:
            out["samples"] = torch.empty((n_sample, n_chain, NPARAM, n), **f32)
        if keep_depth:
            out["depth"] = torch.empty((n_warmup + n_sample, n_chain, n), dtype=torch.int32, device=self.device)
        cfg = _NutsCfg(n_chain, max_depth, n_warmup, n_sample, target_accept, init_step, seed,
                       int(bool(adapt_metric)), int(bool(sync_iterations)))
        _check(_lib.sps_nuts_run(self.h, _stream(stream), C.byref(cfg), n, sfh, _ptr(z), _ptr(obs), _ptr(sigma),
                                 _ptr(mask), _ptr(bounds), _ptr(prior), _ptr(theta0), _ptr(out.get("samples")),
                                 _ptr(out["post_mean"]), _ptr(out["post_sd"]), _ptr(out["rhat"]),
                                 _ptr(out["accept"]), _ptr(out["step"]), _ptr(out["inv_metric"]),
                                 _ptr(out.get("depth")), _ptr(out["n_leaf"]), _ptr(out["lockstep"])))
        return out


class LogLike(torch.autograd.Function):
    """log L(params) per galaxy with the library's hand-written adjoint as backward."""

    @staticmethod
    def forward(ctx, params, z, obs, sigma, mask, sps_ctx, sfh, path, prec):
        logl, grad = sps_ctx.loglike_grad(sfh, params.detach().contiguous(), z, obs, sigma, mask,
                                          path=path, prec=prec, grad=True)
        ctx.save_for_backward(grad)
        return logl

    @staticmethod
    def backward(ctx, gout):
        (grad,) = ctx.saved_tensors
        return grad * gout.unsqueeze(0), None, None, None, None, None, None, None, None


def loglike(sps_ctx, params, z, obs, sigma, mask, sfh=SPS_SFH_DPL, path=SPS_PATH_APPROX, prec=SPS_F32):
    return LogLike.apply(params, z, obs, sigma, mask, sps_ctx, sfh, path, prec)


class PhotApprox(torch.autograd.Function):
    """Approximate magnitudes [n_gal][n_band] of params [10][n_gal]; backward: the library's
    vector-Jacobian product of the band adjoints."""

    @staticmethod
    def forward(ctx, params, z, sps_ctx, sfh):
        p = params.detach().contiguous()
        ctx.save_for_backward(p, z)
        ctx.sps, ctx.sfh = sps_ctx, sfh
        return sps_ctx.phot_approx(sfh, p, z)

    @staticmethod
    def backward(ctx, gbar):
        p, z = ctx.saved_tensors
        g = ctx.sps.phot_vjp(ctx.sfh, p, z, gbar.contiguous().float(), path=SPS_PATH_APPROX)
        return g, None, None, None


class PhotExact(torch.autograd.Function):
    """Exact magnitudes [n_gal][n_band] in SPS_F32 or SPS_BF16X; backward: the exact path's
    vector-Jacobian product (the adjoint GEMM) of the band adjoints."""

    @staticmethod
    def forward(ctx, params, z, sps_ctx, sfh, prec):
        p = params.detach().contiguous()
        ctx.save_for_backward(p, z)
        ctx.sps, ctx.sfh, ctx.prec = sps_ctx, sfh, prec
        return sps_ctx.phot_exact(sfh, p, z, prec=prec)

    @staticmethod
    def backward(ctx, gbar):
        p, z = ctx.saved_tensors
        g = ctx.sps.phot_vjp(ctx.sfh, p, z, gbar.contiguous().float(), path=SPS_PATH_EXACT, prec=ctx.prec)
        return g, None, None, None, None


def phot_approx(sps_ctx, params, z, sfh=SPS_SFH_DPL):
    return PhotApprox.apply(params, z, sps_ctx, sfh)


def phot_exact(sps_ctx, params, z, sfh=SPS_SFH_DPL, prec=SPS_F32):
    return PhotExact.apply(params, z, sps_ctx, sfh, prec)
