#!/usr/bin/env python
"""Throughput benchmark of the SPS hot path on one MI355X.

Headline step: one value+gradient evaluation of the Gaussian photometric
log-likelihood (approximate photometry) for every galaxy of a batch of
1,000,000 synthetic galaxies (double-power-law SFH with a burst, log-normal
metallicity, power-law dust with a floor, 6 Gaussian bands, 10 parameters),
through the C ABI (sps_loglike_grad).  Inputs are resident in HBM before the
timed region.  Prints ONE JSON line.

Inputs are synthetic (seeded); observed magnitudes are the library's own
forward magnitudes at the true parameters plus N(0, 0.05^2) noise.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published FP32 vector peak (256 CU x 2.4 GHz; the packed-FP32 rate)
PEAK_FP32_VECTOR = 157.3
# counted work of one value+gradient evaluation of one galaxy, in FLOP (lane-ops for the
# weights, transcendentals weighted x4 as quarter-rate instructions):
#   forward contraction over both z-table slices: 2 slices x 6 bands x 1128 SSPs x 2 = 27,072
#   adjoint contraction (d/dP_age over both slices):                              27,072
#   SSP weights (bin quadrature, burst window, metallicity), forward and adjoint: 2 x 10,000
CONTRACTION_FLOP_PER_EVAL = 2 * 27_072
WEIGHTS_OPS_PER_EVAL = 2 * 10_000
WORK_PER_EVAL = CONTRACTION_FLOP_PER_EVAL + WEIGHTS_OPS_PER_EVAL
# forward only (the approximate-magnitude workload): one contraction, one weights pass
WORK_PER_FWD = 27_072 + 10_000
# algorithmic HBM bytes per galaxy of the approximate forward call: 10 parameters + z in,
# 6 magnitudes out (FP32)
APPROX_FWD_BYTES = 4 * (10 + 1 + 6)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_approx_logl_grad_1M_traffic.md")
FWD_COUNTERS_FILE = os.path.join(ROOT, "profiles", "k_approx_mags_100k_counters.md")
EXACT_COUNTERS_FILE = os.path.join(ROOT, "profiles", "exact_4096x5000_kernel_trace.md")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_digest(d=None):
    """sha256 over the code of the HIP sources and headers the kernels are built from (comments
    and whitespace removed, so that an edit of a comment does not void the counters); d: the
    source folder (default: the package's csrc)."""
    import hashlib
    import re
    d = d or os.path.join(ROOT, "paper_2506_19919_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(d, name), encoding="utf-8") as f:
                code = re.sub(r"/\*.*?\*/", " ", f.read(), flags=re.S)
            code = re.sub(r"//[^\n]*", " ", code)
            code = " ".join(code.split())
            h.update(name.encode() + b"\0" + code.encode())
    return h.hexdigest()


def profile_values(path, prefix="traffic_"):
    """The `key: value` lines starting with prefix of a committed rocprofv3 summary, as
    {key: str}, or None when the summary is missing or the kernel sources changed since its
    counters were taken (its `<prefix>source_sha256` line no longer matches)."""
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith(prefix) and ":" in line:
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get(prefix + "source_sha256") != kernel_source_digest():
        return None
    return vals


def measured_traffic(path=TRAFFIC_FILE):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the plain-copy calibration), or None when the
    summary is missing or the kernel sources changed since the counters were taken."""
    vals = profile_values(path)
    if vals is None:
        return None
    try:
        return float(vals["traffic_fetch_bytes_per_launch"]) + float(vals["traffic_write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def measured_busy(path):
    """VALU and matrix-core busy fractions of the kernel a committed counter summary covers
    ({"valu_busy": f, "mfma_busy": f}), or None when missing or stale."""
    vals = profile_values(path, "busy_")
    if vals is None:
        return None
    try:
        return {"valu_busy": float(vals["busy_valu"]), "mfma_busy": float(vals["busy_mfma"])}
    except (KeyError, ValueError):
        return None


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo) and the logical CPUs the process may use."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return {"cpu_model": name, "logical_cpus_available": avail}


def oracle_threads():
    return int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1


def cpu_baseline(ssp, filt, th, z, noise, sig, budget_s=12.0):
    """The FP64 oracle (as it stands) on a bounded sample of the headline workload."""
    import oracle
    orc = oracle.Oracle(ssp, filt)
    orc.build_ztable(64, 0.1, 3.0)

    def run(n):
        t64, z64 = th[:n].astype(np.float64), z[:n].astype(np.float64)
        obs = orc.phot_approx(1, t64, z64) + noise[:n]
        mask = np.full(n, 63, np.uint8)
        t0 = time.perf_counter()
        orc.loglike_grad(1, t64, z64, obs, sig[:n], mask)
        return time.perf_counter() - t0

    probe = 256
    dt = run(probe)
    n = int(min(len(z), max(probe, probe * budget_s / max(dt, 1e-6))))
    dt = run(n)
    return dict(value=n / dt, unit="evals/s", cores=oracle_threads(), kind="oracle",
                sample=f"first {n} galaxies of the 1,000,000-galaxy workload, value+gradient "
                       f"(forward-mode dual numbers), FP64, OpenMP over galaxies", **cpu_model())


def _scaled_sample(run, n_total, probe, budget_s):
    """Times run(probe), then run(n) with n sized so that it takes about budget_s; (n, seconds)."""
    dt = run(probe)
    n = int(min(n_total, max(probe, probe * budget_s / max(dt, 1e-6))))
    return n, (run(n) if n != probe else dt)


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def bench_exact_f64(dev, n=64, steps=20, warmup=3, cpu=True):
    """Exact photometry in FP64 on the matrix cores (the parity workload): n log-normal-SFH
    galaxies x 1128 SSPs x 2000 wavelengths x 6 bands, forward magnitudes."""
    import torch

    import paper_2506_19919_amd as sps
    import synth
    log(f"[bench] exact FP64 forward: {n} galaxies x 2000 wavelengths")
    ssp, filt = synth.ssp_grid(2000), synth.filters()
    ctx = sps.Context(ssp, filt, precisions=(sps.SPS_F64,), max_gal=n, max_exact=n)
    th, z = synth.galaxies_lognormal(n, 101, burst=False)
    params = torch.as_tensor(np.ascontiguousarray(th.T)).to(dev)
    zt = torch.as_tensor(z).to(dev)
    fwd = lambda: ctx.phot_exact(synth.SFH_LOGNORMAL, params, zt, prec=sps.SPS_F64)   # noqa: E731
    t = timed(fwd, steps, warmup)
    mags = fwd().cpu().numpy()
    ctx.close()
    flop = 2.0 * n * 1128 * 2000
    res = {"workload": f"exact photometry forward, FP64, {n} galaxies (log-normal SFH), 1128 SSPs x 2000 "
                       "wavelengths x 6 bands", "unit": "evals/s", "evals_per_s": n / t, "ms_forward": t * 1e3,
           "gemm_tflops": flop / t / 1e12, "fp64_mfma_peak_tflops": 78.6,
           "frac_of_fp64_mfma_peak": flop / t / 1e12 / 78.6}
    log(f"[bench]   FP64 forward {t * 1e3:.3f} ms")
    if cpu:
        import oracle
        orc = oracle.Oracle(ssp, filt)
        t0 = time.perf_counter()
        ref = orc.phot_exact(synth.SFH_LOGNORMAL, th, z)
        dt = time.perf_counter() - t0
        res["max_abs_dmag_vs_oracle"] = float(np.abs(mags - ref).max())
        res["cpu_baseline"] = dict(value=n / dt, unit="evals/s", cores=oracle_threads(), kind="oracle",
                                   sample=f"all {n} galaxies, FP64 forward", **cpu_model())
        log(f"[bench]   max |dm| vs oracle {res['max_abs_dmag_vs_oracle']:.2e}; oracle {dt:.2f} s")
    return res


def bench_approx_fwd(dev, n=100_000, steps=20, warmup=3, cpu=True, budget_s=8.0,
                     sweep=(100_000, 1_000_000, 10_000_000)):
    """Approximate magnitudes (the z-table path), forward only: n log-normal-SFH galaxies with a
    burst, 6 bands; evals/s, algorithmic HBM rate and the model kernel's own duration."""
    import torch

    import paper_2506_19919_amd as sps
    import synth
    log(f"[bench] approximate forward: {n} galaxies")
    ssp, filt = synth.ssp_grid(2000), synth.filters()
    ctx = sps.Context(ssp, filt, precisions=(sps.SPS_F64,), max_gal=n)
    ctx.build_ztable(64, 0.1, 3.0)
    th, z = synth.galaxies_lognormal(n, 102, burst=True)
    params = torch.as_tensor(synth.soa32(th)).to(dev)
    zt = torch.as_tensor(z.astype(np.float32)).to(dev)
    out = torch.empty((n, 6), dtype=torch.float32, device=dev)
    fwd = lambda: ctx.phot_approx(synth.SFH_LOGNORMAL, params, zt, out=out)   # noqa: E731
    for _ in range(warmup):
        fwd()
    torch.cuda.synchronize()
    ctx.set_kernel_timing(steps)
    t = timed(fwd, steps, 0)
    kernel_ms = float(np.mean(ctx.kernel_times()))
    ctx.set_kernel_timing(0)
    ctx.close()
    work = WORK_PER_FWD * n / (kernel_ms * 1e-3) / 1e12
    res = {"workload": f"approximate photometry forward, FP32, {n} galaxies (log-normal SFH with burst), "
                       "6 bands, z table 64 nodes", "unit": "evals/s", "evals_per_s": n / t,
           "ms_per_call": t * 1e3, "kernel": "k_approx<MODE_MAGS>", "kernel_ms": kernel_ms,
           "hbm_gbps_algorithmic_call": APPROX_FWD_BYTES * n / t / 1e9,
           "hbm_gbps_algorithmic_kernel": APPROX_FWD_BYTES * n / (kernel_ms * 1e-3) / 1e9,
           "algorithmic_bytes_per_galaxy": APPROX_FWD_BYTES,
           "work_per_galaxy": WORK_PER_FWD, "work_tflops": work,
           "frac_of_fp32_vector_peak": work / PEAK_FP32_VECTOR}
    busy = measured_busy(FWD_COUNTERS_FILE)
    if busy:
        res.update(busy)
    log(f"[bench]   {t * 1e3:.3f} ms per call (kernel {kernel_ms:.3f} ms), "
        f"{res['hbm_gbps_algorithmic_call']:.1f} GB/s algorithmic")
    if sweep:
        # batch-size sweep (10^5 .. 10^7): at 10^5 galaxies a launch holds ~1,600 waves, below
        # one round of the chip's 2,048 wave slots, so the per-galaxy rate there is latency-bound
        big = max(sweep)
        ths, zs = synth.galaxies_lognormal(big, 112, burst=True)
        cs = sps.Context(ssp, filt, precisions=(sps.SPS_F64,), max_gal=big)
        cs.build_ztable(64, 0.1, 3.0)
        rows = []
        for m in sweep:
            pm = torch.as_tensor(synth.soa32(ths[:m])).to(dev)
            zm = torch.as_tensor(zs[:m].astype(np.float32)).to(dev)
            om = torch.empty((m, 6), dtype=torch.float32, device=dev)
            f = lambda: cs.phot_approx(synth.SFH_LOGNORMAL, pm, zm, out=om)   # noqa: E731,B023
            f()
            torch.cuda.synchronize()
            reps = max(3, min(steps, int(2e6 // m)))
            cs.set_kernel_timing(reps)
            tm = timed(f, reps, 0)
            km = float(np.mean(cs.kernel_times()))
            cs.set_kernel_timing(0)
            rows.append({"n_gal": m, "ms_per_call": tm * 1e3, "kernel_ms": km, "evals_per_s": m / tm,
                         "frac_of_fp32_vector_peak": WORK_PER_FWD * m / (km * 1e-3) / 1e12 / PEAK_FP32_VECTOR})
            log(f"[bench]   sweep {m}: {tm * 1e3:.3f} ms per call, kernel {km:.3f} ms")
            del pm, zm, om
        cs.close()
        res["batch_sweep"] = rows
    if cpu:
        import oracle
        orc = oracle.Oracle(ssp, filt)
        orc.build_ztable(64, 0.1, 3.0)

        def run(m):
            t0 = time.perf_counter()
            orc.phot_approx(synth.SFH_LOGNORMAL, th[:m], z[:m])
            return time.perf_counter() - t0
        m, dt = _scaled_sample(run, n, 512, budget_s)
        res["cpu_baseline"] = dict(value=m / dt, unit="evals/s", cores=oracle_threads(), kind="oracle",
                                   sample=f"first {m} of the {n} galaxies, FP64 forward", **cpu_model())
    return res


def bench_exact(dev, n=4096, steps=5, warmup=2, cpu=False, budget_s=10.0):
    """Exact-photometry value+gradient (MFMA) at 4096 galaxies x 1128 SSPs x 5000 wavelengths."""
    import torch

    import paper_2506_19919_amd as sps
    import synth
    log(f"[bench] exact path: {n} galaxies x 5000 wavelengths")
    ssp, filt = synth.ssp_grid(5000), synth.filters()
    ctx = sps.Context(ssp, filt, precisions=(sps.SPS_F64, sps.SPS_F32, sps.SPS_BF16X), max_gal=n, max_exact=n)
    th, z = synth.galaxies_dpl(n, 105)
    params = torch.as_tensor(np.ascontiguousarray(th.T.astype(np.float32))).to(dev)
    zt = torch.as_tensor(z.astype(np.float32)).to(dev)
    noise, sig = synth.photometric_noise(n, 6, 205)
    mags = ctx.phot_exact(synth.SFH_DPL, params, zt, prec=sps.SPS_F32)
    obs = (mags + torch.as_tensor(noise, dtype=torch.float32, device=dev)).contiguous()
    sigma = torch.as_tensor(sig, dtype=torch.float32, device=dev)
    mask = torch.full((n,), 63, dtype=torch.uint8, device=dev)
    res = {"workload": f"exact photometry value+gradient, {n} galaxies, 1128 SSPs x 5000 wavelengths x 6 bands",
           "unit": "evals/s"}
    # dense-equivalent work of one GEMM: the kernels skip the wavelength tiles outside every
    # band's filter support (about a third of this grid), so rates computed from it are
    # effective rates; the executed matrix-core utilisation is the rocprofv3 busy counter
    gemm_flop = 2.0 * n * 1128 * 5000
    # dense matrix-core peaks of MI355X: FP32 157.3 TFLOP/s; BF16 2.5 PFLOP/s, of which the
    # hi/lo split spends three products per algorithmic one
    peaks = {"f32": (157.3, 1), "bf16x": (2500.0, 3)}
    for name, prec in (("f32", sps.SPS_F32), ("bf16x", sps.SPS_BF16X)):
        # the tile order the autotuner picks for this shape (results do not depend on it)
        chosen, tune_ms = ctx.autotune_exact(synth.SFH_DPL, params, zt, obs, sigma, mask, prec=prec)
        fwd = timed(lambda: ctx.phot_exact(synth.SFH_DPL, params, zt, prec=prec), steps, warmup)
        vg = timed(lambda: ctx.loglike_grad(synth.SFH_DPL, params, zt, obs, sigma, mask,
                                            path=sps.SPS_PATH_EXACT, prec=prec), steps, warmup)
        peak, mult = peaks[name]
        res[name] = {"autotuned": {k: chosen[k] for k in ("exact_order", "exact_xcd", "exact_ring")},
                     "value_grad_evals_per_s": n / vg, "forward_evals_per_s": n / fwd,
                     "ms_value_grad": vg * 1e3, "ms_forward": fwd * 1e3,
                     "dense_equivalent_gemm_tflops_forward": gemm_flop / fwd / 1e12,
                     "dense_equivalent_gemm_tflops_value_grad": 2 * gemm_flop / vg / 1e12,
                     "mfma_peak_tflops": peak,
                     "dense_equivalent_frac_of_peak_forward": mult * gemm_flop / fwd / 1e12 / peak,
                     "dense_equivalent_frac_of_peak_value_grad": mult * 2 * gemm_flop / vg / 1e12 / peak}
        log(f"[bench]   {name}: fwd {fwd * 1e3:.3f} ms, value+grad {vg * 1e3:.3f} ms")
    obs_h = obs.cpu().numpy().astype(np.float64)
    ctx.close()
    # executed matrix-core utilisation of the GEMMs (rocprofv3 SQ_VALU_MFMA_BUSY_CYCLES, from the
    # committed counter summary while the kernel sources match it)
    vals = profile_values(EXACT_COUNTERS_FILE, "busy_")
    if vals:
        for name in ("f32", "bf16x"):
            res[name]["mfma_busy_rocprof"] = {
                part: float(vals[f"busy_mfma_{name}_{part}"]) for part in ("forward", "forward_dust", "gradient")
                if f"busy_mfma_{name}_{part}" in vals}
    if cpu:
        import oracle
        orc = oracle.Oracle(ssp, filt)
        m64 = np.full(n, 63, np.uint8)

        def run(m):
            t0 = time.perf_counter()
            orc.loglike_grad(synth.SFH_DPL, th[:m], z[:m], obs_h[:m], sig[:m], m64[:m], path=1)
            return time.perf_counter() - t0
        m, dt = _scaled_sample(run, n, 16, budget_s)
        res["cpu_baseline"] = dict(value=m / dt, unit="evals/s", cores=oracle_threads(), kind="oracle",
                                   sample=f"first {m} of the {n} galaxies, exact value+gradient, FP64 "
                                          "(forward-mode dual numbers)", **cpu_model())
    return res


def bench_hmc(dev, n, n_warm, n_samp, C=4, L=10, adapt_metric=False, cpu=False, budget_s=12.0):
    """Batched HMC: n galaxies x C chains, L leapfrog steps, warm-up + sampling; converged
    posteriors/min (all ten R-hat < 1.2) and the raw rate over all galaxies.
    adapt_metric: identity mass matrix (False) or the windowed diagonal adaptation (True).
    cpu: also run the oracle's HMC for whole runs of as many chains as it has threads."""
    import torch

    import paper_2506_19919_amd as sps
    import synth
    log(f"[bench] HMC: {n} galaxies x {C} chains, {n_warm} + {n_samp} iterations x {L} leapfrog steps")
    ssp, filt = synth.ssp_grid(2000), synth.filters()
    ctx = sps.Context(ssp, filt, precisions=(sps.SPS_F64,), max_gal=n * C)
    ctx.build_ztable(64, 0.1, 3.0)
    th, z = synth.galaxies_dpl(n, 104)
    params = torch.as_tensor(np.ascontiguousarray(th.T.astype(np.float32))).to(dev)
    zt = torch.as_tensor(z.astype(np.float32)).to(dev)
    noise, sig = synth.photometric_noise(n, 6, 204)
    mags = ctx.phot_approx(synth.SFH_DPL, params, zt)
    obs = (mags + torch.as_tensor(noise, dtype=torch.float32, device=dev)).contiguous()
    sigma = torch.as_tensor(sig, dtype=torch.float32, device=dev)
    mask = torch.as_tensor(synth.band_masks(n, 6, 204)).to(dev)
    bounds = torch.as_tensor(synth.bounds_k_x0(), dtype=torch.float32, device=dev)
    prior = torch.as_tensor(synth.PRIOR, dtype=torch.float32, device=dev)
    theta0 = torch.as_tensor(synth.prior_draws(C, n, 304), dtype=torch.float32, device=dev).contiguous()
    kw = dict(n_chain=C, n_leapfrog=L, n_warmup=n_warm, n_sample=n_samp, seed=404, adapt_metric=adapt_metric)
    # short untimed run: first-call setup (workspace) and code paths warm
    ctx.hmc_run(synth.SFH_DPL, zt, obs, sigma, mask, bounds, prior, theta0, n_chain=C, n_leapfrog=L,
                n_warmup=2, n_sample=2, seed=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = ctx.hmc_run(synth.SFH_DPL, zt, obs, sigma, mask, bounds, prior, theta0, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rhat = out["rhat"].cpu().numpy()
    conv = float(np.mean(np.all(rhat < 1.2, axis=0)))
    evals = float(n) * C * (n_warm + n_samp) * L
    one_shot = None
    if not adapt_metric:
        # the one-shot value+gradient kernel on a batch of the sampler's size (n x C rows: each
        # galaxy repeated per chain, same uneven bands), the rate the fused kernel compares with
        rep = lambda t: torch.cat([t] * C, dim=-1).contiguous()   # noqa: E731
        pb, zb = rep(params), rep(zt)
        ob = torch.cat([obs] * C, dim=0).contiguous()
        sb = torch.cat([sigma] * C, dim=0).contiguous()
        mb = torch.cat([mask] * C, dim=0).contiguous()
        t_one = timed(lambda: ctx.loglike_grad(synth.SFH_DPL, pb, zb, ob, sb, mb), 20, 3)
        one_shot = n * C / t_one
        log(f"[bench]   one-shot value+grad on the same {n * C} rows: {t_one * 1e3:.3f} ms ({one_shot:.3e} evals/s)")
    ctx.close()
    log(f"[bench]   HMC wall {wall:.2f} s, converged fraction {conv:.3f} (adapt_metric={adapt_metric}, L={L})")
    res = {"workload": f"{n} galaxies x {C} chains, {L} leapfrog steps, {n_warm} warm-up + {n_samp} samples, "
                       "approximate photometry, 3-6 bands per galaxy, starts drawn from the prior",
           "mass_matrix": "diagonal, adapted in slow warm-up windows" if adapt_metric else "identity",
           "unit": "converged posteriors/min (all ten R-hat < 1.2)",
           "converged_posteriors_per_min": conv * n / wall * 60.0,
           "converged_fraction_rhat_lt_1.2": conv,
           "posteriors_per_min_all_galaxies": n / wall * 60.0,
           "value_grad_evals_per_s": evals / wall,
           "wall_s": wall,
           "mean_accept": float(out["accept"].mean().item())}
    if one_shot:
        res["one_shot_same_batch_evals_per_s"] = one_shot
        res["fused_over_one_shot_same_batch"] = evals / wall / one_shot
    if cpu:
        import oracle
        m = max(1, oracle_threads() // C)
        orc = oracle.Oracle(ssp, filt)
        orc.build_ztable(64, 0.1, 3.0)
        x0 = np.ascontiguousarray(synth.prior_draws(C, n, 304)[:, :, :m].transpose(0, 2, 1))
        obs_h = obs[:m].cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        ref = orc.hmc_run(synth.SFH_DPL, z[:m], obs_h, sig[:m], mask[:m].cpu().numpy(), synth.bounds_k_x0(),
                          synth.PRIOR, x0, n_chain=C, n_leapfrog=L, n_warmup=n_warm, n_sample=n_samp, seed=404,
                          adapt_metric=adapt_metric)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = dict(value=m / dt * 60.0, unit="posteriors/min (all galaxies)",
                                   cores=oracle_threads(), kind="oracle",
                                   sample=f"first {m} galaxies x {C} chains, the full {n_warm} + {n_samp} "
                                          f"iterations ({m * C} chains, one per thread)",
                                   converged_fraction=float(np.mean(np.all(ref["rhat"] < 1.2, axis=1))),
                                   **cpu_model())
        log(f"[bench]   oracle HMC: {m} galaxies in {dt:.1f} s")
    return res


def bench_nuts(dev, n=16_384, n_warm=100, n_samp=200, C=4, max_depth=8):
    """NUTS on n galaxies of the HMC workload x C chains, both lock-step schedules: the chains
    of a wave starting every iteration together (sync, the vectorised-over-chains form) or each
    chain moving on when its own tree is done.  Reports the wall time, converged posteriors per
    minute, leapfrog steps per second and the lock-step efficiency (the chains' leapfrog steps
    over the steps their waves took times the chains per wave)."""
    import torch

    import paper_2506_19919_amd as sps
    import synth
    log(f"[bench] NUTS: {n} galaxies x {C} chains, {n_warm} + {n_samp} iterations, max depth {max_depth}")
    ssp, filt = synth.ssp_grid(2000), synth.filters()
    ctx = sps.Context(ssp, filt, precisions=(sps.SPS_F64,), max_gal=n * C)
    ctx.build_ztable(64, 0.1, 3.0)
    ctx.reserve_nuts(n * C, max_depth)
    th, z = synth.galaxies_dpl(16_384, 104)
    th, z = th[:n], z[:n]
    params = torch.as_tensor(synth.soa32(th)).to(dev)
    zt = torch.as_tensor(z.astype(np.float32)).to(dev)
    noise, sig = synth.photometric_noise(16_384, 6, 204)
    mags = ctx.phot_approx(synth.SFH_DPL, params, zt)
    obs = (mags + torch.as_tensor(noise[:n], dtype=torch.float32, device=dev)).contiguous()
    sigma = torch.as_tensor(sig[:n], dtype=torch.float32, device=dev).contiguous()
    mask = torch.as_tensor(np.ascontiguousarray(synth.band_masks(16_384, 6, 204)[:n])).to(dev)
    bounds = torch.as_tensor(synth.bounds_k_x0(), dtype=torch.float32, device=dev)
    prior = torch.as_tensor(synth.PRIOR, dtype=torch.float32, device=dev)
    theta0 = torch.as_tensor(np.ascontiguousarray(synth.prior_draws(C, 16_384, 304)[:, :, :n]),
                             dtype=torch.float32, device=dev)
    res = {"workload": f"{n} galaxies of the HMC workload x {C} chains, NUTS max depth {max_depth}, {n_warm} warm-up "
                       f"+ {n_samp} samples, approximate photometry", "unit": "converged posteriors/min"}
    kw = dict(n_chain=C, max_depth=max_depth, n_warmup=n_warm, n_sample=n_samp, seed=404)
    ctx.nuts_run(synth.SFH_DPL, zt, obs, sigma, mask, bounds, prior, theta0, n_chain=C, max_depth=3, n_warmup=1,
                 n_sample=2, seed=1)
    for name, sync in (("sync", True), ("free", False)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ctx.nuts_run(synth.SFH_DPL, zt, obs, sigma, mask, bounds, prior, theta0, sync_iterations=sync,
                           keep_depth=True, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lk = out["lockstep"].cpu().numpy().astype(np.float64)
        conv = float(np.mean(np.all(out["rhat"].cpu().numpy() < 1.2, axis=0)))
        depth = out["depth"].cpu().numpy()
        res[name] = {"wall_s": wall, "converged_fraction_rhat_lt_1.2": conv,
                     "converged_posteriors_per_min": conv * n / wall * 60.0,
                     "posteriors_per_min_all_galaxies": n / wall * 60.0,
                     "leapfrog_steps_per_s": lk[0] / wall, "lockstep_efficiency": lk[0] / max(lk[1], 1.0),
                     "mean_tree_depth": float(depth.mean()), "max_tree_depth": int(depth.max()),
                     "mean_leapfrog_steps_per_iteration": lk[0] / (n * C * (n_warm + n_samp)),
                     "mean_accept": float(out["accept"].mean().item())}
        log(f"[bench]   {name}: wall {wall:.2f} s, lock-step efficiency {res[name]['lockstep_efficiency']:.3f}, "
            f"mean depth {depth.mean():.2f}, converged {conv:.3f}")
    ctx.close()
    return res


def bench_hmc_exact(dev, n, n_iter=6, C=4, L=10, full_iter=1200, approx_wall=None):
    """HMC with exact photometry on the HMC workload's shape: every leapfrog step is one MFMA
    value+gradient over all n x C chains.  A short run (n_iter iterations, timed) gives the
    time per iteration; the full run's length (full_iter iterations) is extrapolated
    linearly, since every iteration does the same work."""
    import torch

    import paper_2506_19919_amd as sps
    import synth
    log(f"[bench] exact-path HMC: {n} galaxies x {C} chains, {n_iter} iterations x {L} leapfrog steps")
    ssp, filt = synth.ssp_grid(2000), synth.filters()
    ctx = sps.Context(ssp, filt, precisions=(sps.SPS_F32, sps.SPS_BF16X), max_gal=n * C, max_exact=n * C)
    ctx.build_ztable(64, 0.1, 3.0)   # with a z table the chains are ranked by z (narrow GEMM tiles)
    th, z = synth.galaxies_dpl(n, 104)
    params = torch.as_tensor(np.ascontiguousarray(th.T.astype(np.float32))).to(dev)
    zt = torch.as_tensor(z.astype(np.float32)).to(dev)
    noise, sig = synth.photometric_noise(n, 6, 204)
    mags = ctx.phot_exact(synth.SFH_DPL, params, zt, prec=sps.SPS_F32)
    obs = (mags + torch.as_tensor(noise, dtype=torch.float32, device=dev)).contiguous()
    sigma = torch.as_tensor(sig, dtype=torch.float32, device=dev)
    mask = torch.as_tensor(synth.band_masks(n, 6, 204)).to(dev)
    bounds = torch.as_tensor(synth.bounds_k_x0(), dtype=torch.float32, device=dev)
    prior = torch.as_tensor(synth.PRIOR, dtype=torch.float32, device=dev)
    theta0 = torch.as_tensor(synth.prior_draws(C, n, 304), dtype=torch.float32, device=dev).contiguous()
    res = {"workload": f"{n} galaxies x {C} chains, {L} leapfrog steps, exact photometry (1128 SSPs x 2000 "
                       f"wavelengths) in every step; {n_iter} iterations timed, {full_iter} extrapolated",
           "unit": "posteriors/min (extrapolated from the timed iterations)"}
    # the GEMMs' launch choice for the chains' batch: the galaxies repeated once per chain (the
    # value+gradient ranks a batch this large by z, as the sampler ranks its chains)
    rep = lambda t: torch.cat([t] * C, dim=-1 if t.dim() == 2 and t.shape[0] == 10 else 0).contiguous()  # noqa: E731
    p_c, z_c, o_c, s_c, m_c = rep(params), rep(zt), rep(obs), rep(sigma), rep(mask)
    n_warm = min(n_iter // 2, 200)   # the full-length check runs the workload's 200 + 1000
    for name, prec in (("f32", sps.SPS_F32), ("bf16x", sps.SPS_BF16X)):
        chosen, _ = ctx.autotune_exact(synth.SFH_DPL, p_c, z_c, o_c, s_c, m_c, prec=prec)
        kw = dict(n_chain=C, n_leapfrog=L, path=sps.SPS_PATH_EXACT, prec=prec, seed=404)
        ctx.hmc_run(synth.SFH_DPL, zt, obs, sigma, mask, bounds, prior, theta0, n_warmup=1, n_sample=2, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = ctx.hmc_run(synth.SFH_DPL, zt, obs, sigma, mask, bounds, prior, theta0, n_warmup=n_warm,
                          n_sample=n_iter - n_warm, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_it = wall / n_iter
        full = per_it * full_iter
        evals = float(n) * C * (n_iter * L + 1)
        r = {"autotuned": {k: chosen[k] for k in ("exact_order", "exact_xcd", "exact_ring")},
             "ms_per_iteration": per_it * 1e3, "value_grad_evals_per_s": evals / wall,
             "projected_wall_s": full, "posteriors_per_min": n / full * 60.0,
             "mean_accept": float(out["accept"].mean().item())}
        if approx_wall:
            r["exact_over_approx_wall"] = full / approx_wall
        res[name] = r
        log(f"[bench]   {name}: {per_it * 1e3:.1f} ms per iteration, {full_iter} iterations ~ {full:.1f} s")
    ctx.close()
    return res


def bench_hmc_exact_graph(dev, n=1024, C=4, L=10, n_iter=20):
    """The exact-path HMC at a small batch (n x C chains), where each leapfrog step's ~10
    kernels are short: one iteration captured as a hipGraph and replayed, against the same
    kernels launched one by one; then the autotuner's own choice for this shape."""
    import torch

    import paper_2506_19919_amd as sps
    import synth
    log(f"[bench] exact-path HMC graph replay: {n} galaxies x {C} chains, {n_iter} iterations")
    ssp, filt = synth.ssp_grid(2000), synth.filters()
    ctx = sps.Context(ssp, filt, precisions=(sps.SPS_BF16X,), max_gal=n * C, max_exact=n * C)
    ctx.build_ztable(64, 0.1, 3.0)
    th, z = synth.galaxies_dpl(16_384, 104)
    th, z = th[:n], z[:n]
    params = torch.as_tensor(synth.soa32(th)).to(dev)
    zt = torch.as_tensor(z.astype(np.float32)).to(dev)
    noise, sig = synth.photometric_noise(16_384, 6, 204)
    mags = ctx.phot_exact(synth.SFH_DPL, params, zt, prec=sps.SPS_BF16X)
    obs = (mags + torch.as_tensor(noise[:n], dtype=torch.float32, device=dev)).contiguous()
    sigma = torch.as_tensor(sig[:n], dtype=torch.float32, device=dev).contiguous()
    mask = torch.as_tensor(np.ascontiguousarray(synth.band_masks(16_384, 6, 204)[:n])).to(dev)
    bounds = torch.as_tensor(synth.bounds_k_x0(), dtype=torch.float32, device=dev)
    prior = torch.as_tensor(synth.PRIOR, dtype=torch.float32, device=dev)
    theta0 = torch.as_tensor(np.ascontiguousarray(synth.prior_draws(C, 16_384, 304)[:, :, :n]),
                             dtype=torch.float32, device=dev)
    args = (synth.SFH_DPL, zt, obs, sigma, mask, bounds, prior, theta0)
    kw = dict(n_chain=C, n_leapfrog=L, n_warmup=n_iter // 2, n_sample=n_iter - n_iter // 2, seed=404,
              path=sps.SPS_PATH_EXACT, prec=sps.SPS_BF16X)
    res = {"workload": f"{n} galaxies x {C} chains ({n * C} chains), {L} leapfrog steps, exact photometry in "
                       f"BF16 hi+lo, {n_iter} iterations", "unit": "ms per iteration"}
    for name, g in (("kernels", 0), ("graph", 1)):
        ctx.set_launch(hmcx_graph=g)
        ctx.hmc_run(*args, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.hmc_run(*args, **kw)
        torch.cuda.synchronize()
        res[f"ms_per_iteration_{name}"] = (time.perf_counter() - t0) / n_iter * 1e3
    res["graph_speedup"] = res["ms_per_iteration_kernels"] / res["ms_per_iteration_graph"]
    chosen, ms = ctx.autotune_hmc(*args, **kw)
    res["autotuned_hmcx_graph"] = chosen["hmcx_graph"]
    log(f"[bench]   {res['ms_per_iteration_kernels']:.2f} ms per iteration launched kernel by kernel, "
        f"{res['ms_per_iteration_graph']:.2f} ms replayed as a graph; autotuner picks graph={chosen['hmcx_graph']}")
    ctx.close()
    return res


def bench_approx_accuracy(dev, n=4096, sigmas=(200.0, 400.0, 800.0), tau_vs=(0.0, 0.5, 1.0, 2.0, 4.0)):
    """Approximate-minus-exact magnitudes (App. B) against the Gaussian band width and against
    the dust optical depth, on the GPU: FP32 exact path vs the z-table path for n galaxies of the
    likelihood workload's generator (for the tau_V axis: 400 A bands, tau_V set to each value
    for every galaxy)."""
    import torch

    import paper_2506_19919_amd as sps
    import synth
    log(f"[bench] approximation accuracy: {n} galaxies, band sigma {sigmas} A")
    ssp = synth.ssp_grid(2000)
    th, z = synth.galaxies_dpl(n, 107)
    params = torch.as_tensor(np.ascontiguousarray(th.T.astype(np.float32))).to(dev)
    zt = torch.as_tensor(z.astype(np.float32)).to(dev)
    res = {"workload": f"{n} galaxies (DPL SFH, burst, dust), 6 Gaussian bands 3600-9700 A, "
                       "|m_approx - m_exact| per galaxy and band, FP32 exact path", "unit": "mag"}
    for sig in sigmas:
        filt = synth.filters(sigma=sig)
        ctx = sps.Context(ssp, filt, precisions=(sps.SPS_F32,), max_gal=n, max_exact=n)
        ctx.build_ztable(64, 0.1, 3.0)
        d = (ctx.phot_approx(synth.SFH_DPL, params, zt)
             - ctx.phot_exact(synth.SFH_DPL, params, zt, prec=sps.SPS_F32)).abs().cpu().numpy()
        ctx.close()
        ratio = filt["center_A"] / (2.0 * np.sqrt(2.0 * np.log(2.0)) * sig)
        res[f"sigma_{int(sig)}A"] = {"lambda_over_fwhm": [float(ratio.min()), float(ratio.max())],
                                     "median": float(np.median(d)), "p95": float(np.percentile(d, 95)),
                                     "max": float(d.max())}
        log(f"[bench]   sigma {sig:.0f} A: median {np.median(d):.2e}, p95 {np.percentile(d, 95):.2e}, "
            f"max {d.max():.2e} mag")
    filt = synth.filters()
    ctx = sps.Context(ssp, filt, precisions=(sps.SPS_F32,), max_gal=n, max_exact=n)
    ctx.build_ztable(64, 0.1, 3.0)
    # the generator's attenuation floors (F_floor up to 0.3) flatten F_att at large tau_V; the
    # second sweep sets every floor to 0
    for floor in (None, 0.0):
        for tv in tau_vs:
            t2 = th.copy()
            t2[:, synth.P_TAUV] = tv
            if floor is not None:
                t2[:, synth.P_FFLOOR] = floor
            p2 = torch.as_tensor(synth.soa32(t2)).to(dev)
            d = (ctx.phot_approx(synth.SFH_DPL, p2, zt)
                 - ctx.phot_exact(synth.SFH_DPL, p2, zt, prec=sps.SPS_F32)).abs().cpu().numpy()
            key = f"tau_v_{tv:g}" + ("" if floor is None else "_no_floor")
            res[key] = {"sigma_A": 400.0, "f_floor": "generator U(0, 0.3)" if floor is None else floor,
                        "median": float(np.median(d)), "p95": float(np.percentile(d, 95)), "max": float(d.max())}
            log(f"[bench]   {key}: median {np.median(d):.2e}, p95 {np.percentile(d, 95):.2e}, max {d.max():.2e} mag")
    ctx.close()
    return res


def bench_posterior_agreement(dev, n=1024, C=4, L=10, n_warm=200, n_samp=1000):
    """App. B's second test: the same sampler, same starts and draws, with approximate and with
    exact (BF16 hi+lo) photometry on n galaxies of the HMC workload; the posterior means are
    compared in units of the posterior sd."""
    import torch

    import paper_2506_19919_amd as sps
    import synth
    log(f"[bench] approximate vs exact posteriors: {n} galaxies x {C} chains, {n_warm} + {n_samp} iterations")
    ssp, filt = synth.ssp_grid(2000), synth.filters()
    ctx = sps.Context(ssp, filt, precisions=(sps.SPS_F32, sps.SPS_BF16X), max_gal=n * C, max_exact=n * C)
    ctx.build_ztable(64, 0.1, 3.0)
    th, z = synth.galaxies_dpl(16_384, 104)
    th, z = th[:n], z[:n]
    params = torch.as_tensor(np.ascontiguousarray(th.T.astype(np.float32))).to(dev)
    zt = torch.as_tensor(z.astype(np.float32)).to(dev)
    noise, sig = synth.photometric_noise(16_384, 6, 204)
    mags = ctx.phot_exact(synth.SFH_DPL, params, zt, prec=sps.SPS_F32)
    obs = (mags + torch.as_tensor(noise[:n], dtype=torch.float32, device=dev)).contiguous()
    sigma = torch.as_tensor(sig[:n], dtype=torch.float32, device=dev).contiguous()
    mask = torch.as_tensor(np.ascontiguousarray(synth.band_masks(16_384, 6, 204)[:n])).to(dev)
    bounds = torch.as_tensor(synth.bounds_k_x0(), dtype=torch.float32, device=dev)
    prior = torch.as_tensor(synth.PRIOR, dtype=torch.float32, device=dev)
    theta0 = torch.as_tensor(np.ascontiguousarray(synth.prior_draws(C, 16_384, 304)[:, :, :n]),
                             dtype=torch.float32, device=dev)
    kw = dict(n_chain=C, n_leapfrog=L, n_warmup=n_warm, n_sample=n_samp, seed=404)
    t0 = time.perf_counter()
    ap = ctx.hmc_run(synth.SFH_DPL, zt, obs, sigma, mask, bounds, prior, theta0, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ex = ctx.hmc_run(synth.SFH_DPL, zt, obs, sigma, mask, bounds, prior, theta0, path=sps.SPS_PATH_EXACT,
                     prec=sps.SPS_BF16X, **kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.close()
    pa, sa = ap["post_mean"].cpu().numpy(), ap["post_sd"].cpu().numpy()
    pe, se = ex["post_mean"].cpu().numpy(), ex["post_sd"].cpu().numpy()
    d = np.abs(pe - pa) / np.maximum(np.maximum(sa, se), 1e-12)
    conv = np.all(ap["rhat"].cpu().numpy() < 1.2, axis=0) & np.all(ex["rhat"].cpu().numpy() < 1.2, axis=0)
    res = {"workload": f"{n} galaxies of the HMC workload x {C} chains, {L} leapfrog steps, {n_warm} + {n_samp} "
                       "iterations, same starts and Philox draws; exact path in BF16 hi+lo",
           "median_abs_mean_diff_over_sd": float(np.median(d)),
           "p90_abs_mean_diff_over_sd": float(np.percentile(d, 90)),
           "median_sd_ratio_exact_over_approx": float(np.median(se / np.maximum(sa, 1e-12))),
           "both_converged_fraction": float(conv.mean()),
           "median_abs_mean_diff_over_sd_converged": float(np.median(d[:, conv])) if conv.any() else None,
           "wall_s_approx": t1 - t0, "wall_s_exact": t2 - t1}
    log(f"[bench]   |mean diff| / sd: median {res['median_abs_mean_diff_over_sd']:.3f}, 90th pct "
        f"{res['p90_abs_mean_diff_over_sd']:.3f}; wall {t1 - t0:.2f} s approx, {t2 - t1:.2f} s exact")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-gal", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-exact", action="store_true")
    ap.add_argument("--no-hmc", action="store_true")
    ap.add_argument("--no-hmc-exact", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true")
    ap.add_argument("--no-approx-fwd", action="store_true")
    ap.add_argument("--no-nuts", action="store_true")
    ap.add_argument("--no-posterior-agreement", action="store_true")
    ap.add_argument("--hmc-exact-iters", type=int, default=6,
                    help="iterations timed in the exact-path HMC leg (the full run length is extrapolated)")
    ap.add_argument("--hmc-gal", type=int, default=16_384)
    ap.add_argument("--hmc-warmup", type=int, default=200)
    ap.add_argument("--hmc-sample", type=int, default=1000)
    ap.add_argument("--legs", default="all",
                    help="comma-separated legs to run after the headline (all, or any of exact_f64, approx_fwd, "
                         "exact, accuracy, hmc, nuts, posterior_agreement, hmc_exact)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="also run 3 plain 1 GiB device copies (reference for the HBM byte counters)")
    args = ap.parse_args()
    if args.hmc_exact_iters < 4:
        ap.error("--hmc-exact-iters must be at least 4 (half warm-up, and at least two samples)")
    legs = set(args.legs.split(","))

    def leg(name, off):
        return not off and ("all" in legs or name in legs)

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the hot path shards by "
                                   "independent galaxies and is measured per GPU (--gpus 1)"}))
        sys.exit(2)

    import torch

    import paper_2506_19919_amd as sps
    import synth

    dev = torch.device("cuda", 0)
    n = args.n_gal
    log(f"[bench] setup: {n} galaxies")
    ssp, filt = synth.ssp_grid(2000), synth.filters()
    ctx = sps.Context(ssp, filt, precisions=(sps.SPS_F64, sps.SPS_F32), max_gal=max(n, 1 << 16))
    ctx.build_ztable(64, 0.1, 3.0)
    th, z = synth.galaxies_dpl(n, 103)
    th32, z32 = th.astype(np.float32), z.astype(np.float32)
    noise, sig = synth.photometric_noise(n, 6, 203)
    params = torch.as_tensor(np.ascontiguousarray(th32.T)).to(dev)
    zt = torch.as_tensor(z32).to(dev)
    mags = ctx.phot_approx(synth.SFH_DPL, params, zt)
    obs = (mags + torch.as_tensor(noise, dtype=torch.float32, device=dev)).contiguous()
    sigma = torch.as_tensor(sig, dtype=torch.float32, device=dev)
    mask = torch.full((n,), 63, dtype=torch.uint8, device=dev)
    logl = torch.empty(n, dtype=torch.float32, device=dev)
    grad = torch.empty((10, n), dtype=torch.float32, device=dev)

    def step():
        ctx.loglike_grad(synth.SFH_DPL, params, zt, obs, sigma, mask, logl_out=logl, grad_out=grad)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"[bench] warmup done ({args.warmup} steps)")
    if args.traffic_probe:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("[bench] traffic probe: 3 copies of 1 GiB done")
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    ctx.set_kernel_timing(args.steps)   # events around k_approx itself, on the stream it runs on
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step()
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    kernel_ms = float(np.mean(ctx.kernel_times()))
    ctx.set_kernel_timing(0)
    ms_per_step = wall / args.steps * 1e3
    value = n * args.steps / wall
    log(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step (step events {per_launch_ms:.3f} ms, "
        f"k_approx events {kernel_ms:.3f} ms)")

    achieved = WORK_PER_EVAL * n / (kernel_ms * 1e-3) / 1e12
    contraction_rate = CONTRACTION_FLOP_PER_EVAL * n / (kernel_ms * 1e-3) / 1e12
    out = {
        "metric": "photometry value+grad evals/s (exact vs approx); HMC posteriors/min, 1 GPU",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (contractions: bf16 hi+lo x3 on MFMA, f32 accumulate)",
        "data": "synthetic",
        "config": {
            "workload": "log-likelihood value+gradient, approximate photometry, 1,000,000 galaxies, "
                        "10 parameters, 6 bands, SSP grid 12 x 94 x 2000, z table 64 nodes",
            "n_gal": n, "n_param": 10, "n_band": 6, "n_ssp": 1128, "n_wave": 2000, "n_z": 64,
            "parallelism": "single GPU; galaxies data-parallel",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP32_VECTOR,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_VECTOR,
            "traffic": measured_traffic(),
            "traffic_unit": "bytes per launch (HBM, rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": "k_approx<MODE_LOGL_GRAD>, per-launch time from HIP events recorded around it on "
                      "its stream",
            "kernel_ms": kernel_ms,
            "step_ms_events": per_launch_ms,
            "work_per_eval": {"contraction_flop": CONTRACTION_FLOP_PER_EVAL,
                              "weights_lane_ops": WEIGHTS_OPS_PER_EVAL, "total": WORK_PER_EVAL},
            "work_per_launch": WORK_PER_EVAL * n,
            "contraction_only_tflops": contraction_rate,
            "contraction_only_frac": contraction_rate / PEAK_FP32_VECTOR,
        },
    }
    busy = measured_busy(TRAFFIC_FILE)
    if busy:
        out["roofline"].update(busy)
    del params, zt, obs, sigma, mask, logl, grad, mags
    ctx.close()
    cpu = not args.no_cpu_baseline
    if leg("exact_f64", args.no_exact):
        out["exact_f64"] = bench_exact_f64(dev, cpu=cpu)
    if leg("approx_fwd", args.no_approx_fwd):
        out["approx_fwd"] = bench_approx_fwd(dev, cpu=cpu)
    if leg("exact", args.no_exact):
        out["exact"] = bench_exact(dev, cpu=cpu)
    if leg("accuracy", args.no_accuracy):
        out["approx_accuracy"] = bench_approx_accuracy(dev)
    if leg("hmc", args.no_hmc):
        out["hmc"] = bench_hmc(dev, args.hmc_gal, args.hmc_warmup, args.hmc_sample, cpu=cpu)
        out["hmc_adapted_metric"] = bench_hmc(dev, args.hmc_gal, args.hmc_warmup, args.hmc_sample,
                                              adapt_metric=True)
    if leg("nuts", args.no_nuts):
        out["nuts"] = bench_nuts(dev)
    if leg("posterior_agreement", args.no_posterior_agreement):
        out["posterior_agreement"] = bench_posterior_agreement(dev)
    if leg("hmc_exact", args.no_hmc_exact):
        aw = out["hmc"]["wall_s"] if "hmc" in out else None
        out["hmc_exact"] = bench_hmc_exact(dev, args.hmc_gal, n_iter=args.hmc_exact_iters,
                                           full_iter=args.hmc_warmup + args.hmc_sample, approx_wall=aw)
    if leg("hmc_exact", args.no_hmc_exact):
        out["hmc_exact_graph"] = bench_hmc_exact_graph(dev)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(ssp, filt, th32, z32, noise, sig)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
