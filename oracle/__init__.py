"""FP64 CPU oracle of the SPS hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its binding) never does.  The C++ source (``sps_oracle.cpp``) follows the
paper's equations step by step in FP64; see its header for the passage each
function follows.  Gradients are forward-mode dual numbers.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sps_oracle.cpp")
LIB = os.path.join(HERE, "libsps_oracle.so")

N_PARAM = 10
DEFAULT_MODEL = dict(sigma_logz=0.2, burst_dlogt=0.3)
COSMO = dict(H0=70.0, Om=0.3)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (-O3, OpenMP).  Portable flags: the library
    also runs on hosts other than the one it was built on."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
               "-Wall", "-Wextra", "-o", tmp, SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB)
    return LIB


class _Ssp(C.Structure):
    _fields_ = [("n_met", C.c_int), ("n_age", C.c_int), ("n_wave", C.c_int),
                ("log10_met", C.POINTER(C.c_double)), ("log10_age_yr", C.POINTER(C.c_double)),
                ("wave_A", C.POINTER(C.c_double)), ("lum", C.POINTER(C.c_double))]


class _Filters(C.Structure):
    _fields_ = [("n_band", C.c_int), ("center_A", C.POINTER(C.c_double)),
                ("sigma_A", C.POINTER(C.c_double))]


class _Cosmo(C.Structure):
    _fields_ = [("H0", C.c_double), ("Om", C.c_double)]


class _Model(C.Structure):
    _fields_ = [("sigma_logz", C.c_double), ("burst_dlogt", C.c_double)]


class _HmcCfg(C.Structure):
    _fields_ = [("n_chain", C.c_int), ("n_leapfrog", C.c_int), ("n_warmup", C.c_int),
                ("n_sample", C.c_int), ("target_accept", C.c_double), ("init_step", C.c_double),
                ("seed", C.c_uint64), ("adapt_metric", C.c_int), ("path", C.c_int),
                ("it_begin", C.c_int), ("it_end", C.c_int)]


HMC_STATE = 400   # doubles of per-chain state carried between the calls of a split run


class _NutsCfg(C.Structure):
    _fields_ = [("n_chain", C.c_int), ("max_depth", C.c_int), ("n_warmup", C.c_int),
                ("n_sample", C.c_int), ("target_accept", C.c_double), ("init_step", C.c_double),
                ("seed", C.c_uint64), ("adapt_metric", C.c_int), ("path", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        _lib = C.CDLL(LIB)
        d = C.c_double
        _lib.orc_age_universe_gyr.restype = d
        _lib.orc_age_universe_gyr.argtypes = [C.c_void_p, d]
        _lib.orc_lum_distance_mpc.restype = d
        _lib.orc_lum_distance_mpc.argtypes = [C.c_void_p, d]
        _lib.orc_dust_att.restype = d
        _lib.orc_dust_att.argtypes = [C.c_void_p, d]
        _lib.orc_lambda_eff.restype = d
        _lib.orc_lambda_eff.argtypes = [C.c_void_p, C.c_int]
        _lib.orc_bound.restype = d
        _lib.orc_bound.argtypes = [C.c_void_p, d]
        _lib.orc_unbound.restype = d
        _lib.orc_unbound.argtypes = [C.c_void_p, d]
        _lib.orc_log_prior.restype = d
        _lib.orc_log_prior.argtypes = [C.c_void_p, d]
        _lib.orc_rhat.restype = d
        _lib.orc_rhat.argtypes = [C.c_int, C.c_int, C.c_void_p]
        _lib.orc_hmc_prior_draw.restype = None
        _lib.orc_philox4x32_10.restype = None
        _lib.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class Oracle:
    """Holds the SSP grid, filters, cosmology and fixed model constants."""

    def __init__(self, ssp: dict, filt: dict, cosmo: dict | None = None, model: dict | None = None):
        self._keep = dict(
            met=_f64(ssp["log10_met"]), age=_f64(ssp["log10_age_yr"]), wave=_f64(ssp["wave_A"]),
            lum=_f64(ssp["lum"]), cen=_f64(filt["center_A"]), sig=_f64(filt["sigma_A"]))
        k = self._keep
        self.n_met, self.n_age, self.n_wave = len(k["met"]), len(k["age"]), len(k["wave"])
        assert k["lum"].shape == (self.n_met, self.n_age, self.n_wave)
        self.n_band = len(k["cen"])
        self.ssp = _Ssp(self.n_met, self.n_age, self.n_wave, _dp(k["met"]), _dp(k["age"]),
                        _dp(k["wave"]), _dp(k["lum"]))
        self.filt = _Filters(self.n_band, _dp(k["cen"]), _dp(k["sig"]))
        c = dict(COSMO, **(cosmo or {}))
        self.cosmo = _Cosmo(c["H0"], c["Om"])
        md = dict(DEFAULT_MODEL, **(model or {}))
        self.model = _Model(md["sigma_logz"], md["burst_dlogt"])
        self.q = None
        self.ztab = None
        self.L = lib()

    # --- cosmology
    def age_universe(self, z):
        return self.L.orc_age_universe_gyr(C.byref(self.cosmo), float(z))

    def lum_distance(self, z):
        return self.L.orc_lum_distance_mpc(C.byref(self.cosmo), float(z))

    # --- weights
    def age_weights(self, sfh, theta, z):
        pa, ps, pb = (np.zeros(self.n_age) for _ in range(3))
        th = _f64(theta)
        rc = self.L.orc_age_weights(C.byref(self.ssp), C.byref(self.cosmo), C.byref(self.model), sfh,
                                    _p(th), C.c_double(z), _p(pa), _p(ps), _p(pb))
        assert rc == 0
        return pa, ps, pb

    def smooth_bin_mass(self, sfh, theta, z):
        m = np.zeros(self.n_age)
        th = _f64(theta)
        rc = self.L.orc_smooth_bin_mass(C.byref(self.ssp), C.byref(self.cosmo), sfh, _p(th),
                                        C.c_double(z), _p(m))
        assert rc == 0
        return m

    def met_weights(self, theta):
        p = np.zeros(self.n_met)
        th = _f64(theta)
        assert self.L.orc_met_weights(C.byref(self.ssp), C.byref(self.model), _p(th), _p(p)) == 0
        return p

    def weights(self, sfh, theta, z):
        th, zz = _f64(theta), _f64(z)
        w = np.zeros((len(zz), self.n_met, self.n_age))
        rc = self.L.orc_weights(C.byref(self.ssp), C.byref(self.cosmo), C.byref(self.model), sfh,
                                len(zz), _p(th), _p(zz), _p(w))
        assert rc == 0
        return w

    def dust_att(self, theta, lam_rest):
        th = _f64(theta)
        return self.L.orc_dust_att(_p(th), float(lam_rest))

    def lambda_eff(self, band):
        return self.L.orc_lambda_eff(C.byref(self.filt), band)

    # --- photometry
    def phot_exact(self, sfh, theta, z):
        th, zz = _f64(theta), _f64(z)
        mags = np.zeros((len(zz), self.n_band))
        rc = self.L.orc_phot_exact(C.byref(self.ssp), C.byref(self.filt), C.byref(self.cosmo),
                                   C.byref(self.model), sfh, len(zz), _p(th), _p(zz), _p(mags))
        assert rc == 0
        return mags

    def build_ztable(self, n_z=64, z_lo=0.1, z_hi=3.0):
        q = np.zeros((n_z, self.n_band, self.n_met, self.n_age))
        rc = self.L.orc_ztable(C.byref(self.ssp), C.byref(self.filt), n_z, C.c_double(z_lo),
                               C.c_double(z_hi), _p(q))
        assert rc == 0
        self.q, self.ztab = q, (n_z, z_lo, z_hi)
        return q

    def _zt(self):
        if self.q is None:
            self.build_ztable()
        n_z, lo, hi = self.ztab
        return n_z, C.c_double(lo), C.c_double(hi), _p(self.q)

    def phot_approx(self, sfh, theta, z):
        th, zz = _f64(theta), _f64(z)
        mags = np.zeros((len(zz), self.n_band))
        n_z, lo, hi, qp = self._zt()
        rc = self.L.orc_phot_approx(C.byref(self.ssp), C.byref(self.filt), C.byref(self.cosmo),
                                    C.byref(self.model), n_z, lo, hi, qp, sfh, len(zz), _p(th),
                                    _p(zz), _p(mags))
        assert rc in (0, 2)
        return mags

    def loglike_grad(self, sfh, theta, z, obs, sigma, mask, path=0, grad=True):
        th, zz = _f64(theta), _f64(z)
        n = len(zz)
        o, s = _f64(obs), _f64(sigma)
        mk = np.ascontiguousarray(mask, dtype=np.uint8)
        ll = np.zeros(n)
        g = np.zeros((n, N_PARAM)) if grad else None
        if path == 0:
            n_z, lo, hi, qp = self._zt()
        else:
            n_z, lo, hi, qp = 0, C.c_double(0), C.c_double(0), None
        rc = self.L.orc_loglike_grad(C.byref(self.ssp), C.byref(self.filt), C.byref(self.cosmo),
                                     C.byref(self.model), path, n_z, lo, hi, qp, sfh, n, _p(th),
                                     _p(zz), _p(o), _p(s), _p(mk), _p(ll), _p(g))
        assert rc in (0, 2)
        return (ll, g) if grad else ll

    def mags_jacobian(self, sfh, theta, z, path=0):
        """Magnitudes [g][b] and their Jacobian [g][b][10] w.r.t. the physical parameters."""
        th, zz = _f64(theta), _f64(z)
        n = len(zz)
        mags = np.zeros((n, self.n_band))
        jac = np.zeros((n, self.n_band, N_PARAM))
        if path == 0:
            n_z, lo, hi, qp = self._zt()
        else:
            n_z, lo, hi, qp = 0, C.c_double(0), C.c_double(0), None
        rc = self.L.orc_mags_jacobian(C.byref(self.ssp), C.byref(self.filt), C.byref(self.cosmo),
                                      C.byref(self.model), path, n_z, lo, hi, qp, sfh, n, _p(th), _p(zz),
                                      _p(mags), _p(jac))
        assert rc in (0, 2)
        return mags, jac

    # --- bounding / prior
    @staticmethod
    def bound(bnd4, x):
        b = _f64(bnd4)
        return lib().orc_bound(_p(b), float(x))

    @staticmethod
    def unbound(bnd4, th):
        b = _f64(bnd4)
        return lib().orc_unbound(_p(b), float(th))

    @staticmethod
    def log_prior(pri3, x):
        p = _f64(pri3)
        return lib().orc_log_prior(_p(p), float(x))

    def logpost_grad(self, sfh, theta_u, z, obs, sigma, mask, bounds, prior, path=0):
        x = _f64(theta_u)
        o, s = _f64(obs), _f64(sigma)
        b, pr = _f64(bounds), _f64(prior)
        lp = np.zeros(1)
        g = np.zeros(N_PARAM)
        n_z, lo, hi, qp = self._zt() if path == 0 else (0, C.c_double(0), C.c_double(0), None)
        rc = self.L.orc_logpost_grad(C.byref(self.ssp), C.byref(self.filt), C.byref(self.cosmo),
                                     C.byref(self.model), int(path), n_z, lo, hi, qp, sfh, _p(x), C.c_double(z),
                                     _p(o), _p(s), C.c_uint8(int(mask)), _p(b), _p(pr), _p(lp), _p(g))
        assert rc == 0
        return lp[0], g

    def leapfrog(self, x, p, eps, n_step, sfh=1, z=None, obs=None, sigma=None, mask=0,
                 bounds=None, prior=None, gauss_prec=None):
        """n_step leapfrog steps from (x, p); returns (x', p', log target at x')."""
        xx, pp = _f64(x).copy(), _f64(p).copy()
        lp = np.zeros(1)
        gp = _f64(gauss_prec) if gauss_prec is not None else None
        if gp is None:
            n_z, lo, hi, qp = self._zt()
            o, s = _f64(obs), _f64(sigma)
            b, pr = _f64(bounds), _f64(prior)
            zz = C.c_double(z)
        else:
            n_z, lo, hi, qp = 0, C.c_double(0), C.c_double(0), None
            o = s = b = pr = None
            zz = C.c_double(0)
        rc = self.L.orc_leapfrog(C.byref(self.ssp), C.byref(self.filt), C.byref(self.cosmo),
                                 C.byref(self.model), n_z, lo, hi, qp, sfh, zz, _p(o), _p(s),
                                 C.c_uint8(int(mask)), _p(b), _p(pr), _p(gp), int(n_step),
                                 C.c_double(eps), _p(xx), _p(pp), _p(lp))
        assert rc == 0
        return xx, pp, lp[0]

    # --- HMC
    def hmc_run(self, sfh, z, obs, sigma, mask, bounds, prior, theta0, n_chain=4, n_leapfrog=10,
                n_warmup=200, n_sample=1000, target_accept=0.8, init_step=0.1, seed=404,
                keep_samples=False, keep_trace=False, gauss_prec=None, gal_id=None, n_gal_total=0,
                adapt_metric=False, path=0, it_begin=0, it_end=0, state=None, samples=None, n_gal=None):
        """theta0 [chain][galaxy][10] unbounded start, or None to draw it from the prior.
        A run split over calls passes it_begin / it_end and the same `state` array
        ([chain][galaxy][HMC_STATE] float64, updated in place) to every call, and `samples`
        (kept across the calls) to collect the draws."""
        if theta0 is not None:
            th0 = _f64(theta0)
            n_gal = th0.shape[1]
            assert th0.shape == (n_chain, n_gal, N_PARAM)
        else:
            th0 = None
            n_gal = len(z) if n_gal is None else n_gal
        if state is not None:
            assert state.dtype == np.float64 and state.flags.c_contiguous
            assert state.shape == (n_chain, n_gal, HMC_STATE)
        cfg = _HmcCfg(n_chain, n_leapfrog, n_warmup, n_sample, target_accept, init_step, seed,
                      {False: 0, True: 1, "diag": 1, "dense": 2}[adapt_metric], int(path), int(it_begin),
                      int(it_end))
        minv = np.zeros((n_chain, n_gal, N_PARAM))
        pm, ps, rh = (np.zeros((n_gal, N_PARAM)) for _ in range(3))
        acc = np.zeros(n_gal)
        step = np.zeros((n_chain, n_gal))
        if samples is not None:
            assert samples.shape == (n_sample, n_chain, n_gal, N_PARAM) and samples.dtype == np.float64
            smp = samples
        else:
            smp = np.zeros((n_sample, n_chain, n_gal, N_PARAM)) if keep_samples else None
        tr = np.zeros((n_warmup + n_sample, n_chain, n_gal)) if keep_trace else None
        tra = np.zeros((n_warmup + n_sample, n_chain, n_gal, 3)) if keep_trace else None
        gp = _f64(gauss_prec) if gauss_prec is not None else None
        if gp is None:
            n_z, lo, hi, qp = self._zt() if path == 0 else (0, C.c_double(0), C.c_double(0), None)
            zz, o, s = _f64(z), _f64(obs), _f64(sigma)
            mk = np.ascontiguousarray(mask, dtype=np.uint8)
            b, pr = _f64(bounds), _f64(prior)
            args = (_p(zz), _p(o), _p(s), _p(mk), _p(b), _p(pr))
        else:
            n_z, lo, hi, qp = 0, C.c_double(0), C.c_double(0), None
            pr = _f64(prior) if prior is not None else None   # prior draws of the start only
            args = (None,) * 5 + (_p(pr),)
        gid = np.ascontiguousarray(gal_id, dtype=np.uint32) if gal_id is not None else None
        rc = self.L.orc_hmc_run(C.byref(self.ssp), C.byref(self.filt), C.byref(self.cosmo),
                                C.byref(self.model), n_z, lo, hi, qp, sfh, C.byref(cfg), n_gal,
                                *args, _p(th0), _p(gp), _p(pm), _p(ps), _p(rh), _p(acc), _p(step),
                                _p(smp), _p(tr), int(n_gal_total), _p(gid), _p(minv), _p(tra), _p(state))
        assert rc == 0, rc
        out = dict(post_mean=pm, post_sd=ps, rhat=rh, accept=acc, step=step, inv_metric=minv)
        if smp is not None:
            out["samples"] = smp
        if keep_trace:
            out["trace_logp"] = tr
            out["trace_alpha"], out["trace_margin"], out["trace_eps"] = tra[..., 0], tra[..., 1], tra[..., 2]
        return out


def _nuts_run(self, sfh, z, obs, sigma, mask, bounds, prior, theta0, n_chain=4, max_depth=10, n_warmup=200,
              n_sample=1000, target_accept=0.8, init_step=0.1, seed=404, keep_samples=False, gauss_prec=None,
              gal_id=None, n_gal_total=0, adapt_metric=False, path=0, n_gal=None):
    """NUTS (Hoffman & Gelman 2014, Algorithm 3 + dual averaging); arguments as hmc_run.
    Returns the summaries, and per iteration the tree depth, the leapfrog steps and how near its
    slice and U-turn decisions came to their thresholds (margin_slice, margin_turn)."""
    if theta0 is not None:
        th0 = _f64(theta0)
        n_gal = th0.shape[1]
        assert th0.shape == (n_chain, n_gal, N_PARAM)
    else:
        th0 = None
        n_gal = len(z) if n_gal is None else n_gal
    cfg = _NutsCfg(n_chain, max_depth, n_warmup, n_sample, target_accept, init_step, seed, int(bool(adapt_metric)),
                   int(path))
    minv = np.zeros((n_chain, n_gal, N_PARAM))
    pm, ps, rh = (np.zeros((n_gal, N_PARAM)) for _ in range(3))
    acc = np.zeros(n_gal)
    step = np.zeros((n_chain, n_gal))
    smp = np.zeros((n_sample, n_chain, n_gal, N_PARAM)) if keep_samples else None
    depth = np.zeros((n_warmup + n_sample, n_chain, n_gal), np.int32)
    steps = np.zeros((n_warmup + n_sample, n_chain, n_gal), np.int32)
    margin = np.zeros((n_warmup + n_sample, n_chain, n_gal, 2))
    gp = _f64(gauss_prec) if gauss_prec is not None else None
    if gp is None:
        n_z, lo, hi, qp = self._zt() if path == 0 else (0, C.c_double(0), C.c_double(0), None)
        zz, o, s = _f64(z), _f64(obs), _f64(sigma)
        mk = np.ascontiguousarray(mask, dtype=np.uint8)
        b, pr = _f64(bounds), _f64(prior)
        args = (_p(zz), _p(o), _p(s), _p(mk), _p(b), _p(pr))
    else:
        n_z, lo, hi, qp = 0, C.c_double(0), C.c_double(0), None
        pr = _f64(prior) if prior is not None else None
        args = (None,) * 5 + (_p(pr),)
    gid = np.ascontiguousarray(gal_id, dtype=np.uint32) if gal_id is not None else None
    rc = self.L.orc_nuts_run(C.byref(self.ssp), C.byref(self.filt), C.byref(self.cosmo), C.byref(self.model), n_z,
                             lo, hi, qp, sfh, C.byref(cfg), n_gal, *args, _p(th0), _p(gp), _p(pm), _p(ps), _p(rh),
                             _p(acc), _p(step), _p(smp), _p(depth), _p(steps), _p(margin), _p(minv), int(n_gal_total),
                             _p(gid))
    assert rc == 0, rc
    out = dict(post_mean=pm, post_sd=ps, rhat=rh, accept=acc, step=step, inv_metric=minv, depth=depth,
               steps=steps, margin_slice=margin[..., 0], margin_turn=margin[..., 1])
    if smp is not None:
        out["samples"] = smp
    return out


Oracle.nuts_run = _nuts_run


def hmc_prior_draw(prior, seed, chain_id):
    """Unbounded starting point drawn from the skew-normal priors [10][3] for one chain id."""
    pr = _f64(prior)
    x = np.zeros(N_PARAM)
    lib().orc_hmc_prior_draw(_p(pr), C.c_uint64(seed), C.c_uint32(chain_id), _p(x))
    return x


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def gauss_legendre(n):
    """Nodes and weights of the oracle's n-point Gauss-Legendre rule on [-1, 1]."""
    x, w = np.zeros(n), np.zeros(n)
    assert lib().orc_gauss_legendre(int(n), _p(x), _p(w)) == 0
    return x, w


def hmc_windows(n_warmup):
    """Slow adaptation windows [(start, end), ...] of a warm-up of n_warmup iterations."""
    s = np.zeros(64, np.int32)
    e = np.zeros(64, np.int32)
    n = lib().orc_hmc_windows(int(n_warmup), 64, _p(s), _p(e))
    return [(int(s[i]), int(e[i])) for i in range(min(n, 64))]


def rhat(x):
    a = _f64(x)
    return lib().orc_rhat(a.shape[0], a.shape[1], _p(a))
