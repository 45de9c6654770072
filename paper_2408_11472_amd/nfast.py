"""Regular mode and the n_fast sweep (Sec. III.A premise, Sec. IV.A Fig. 4,
Sec. IV.B Fig. 5-6).

The fast mode rests on the premise that the Doppler spectrum of each gate
changes slowly compared with the pulse interval (Sec. III.A).  Its cost falls
with n_fast (Fig. 4) while the multi-looked power waveforms stay those of the
regular mode, in which the surface is updated at every pulse (Fig. 6; the
retracked SWH differs by ~2 cm, Sec. IV.B).  This module measures both on one
scene:

* the **regular mode** is the library's path with n_fast = 1: every pulse is
  its own spectrum, the eq. (1) weights are 1 at that pulse and 0 at its
  neighbours, so Y[x, g] is the coherent sum of the scatterers of gate g at
  pulse x (the per-pulse simulation, Sec. III.A);
* the **fast mode** at n_fast in {250, 500, 750, 1000, 1250} (the values of
  Sec. IV), with N = the smallest power of two >= 2 n_fast Doppler bins
  (capped at 2048, beyond which the long-time signal is read periodically);
* the run time of each mode on the GPU (Fig. 4) and the fidelity of its
  multi-look waveform against the regular mode's: per-gate differences in
  units of their speckle standard deviation (the variance of a mean of
  correlated pulse powers, from the integrated autocorrelation time of each
  series), the total-power ratio, and the pulse-to-pulse correlation of the
  IQ signal, which Sec. IV.B reads as reproduced by the fast mode.

Everything that simulates runs in the library's kernels; the statistics
below are host arithmetic on the IQ the kernels produced.
"""
from __future__ import annotations

import time
from dataclasses import replace

import numpy as np

from . import workloads

SWEEP_NFAST = (250, 500, 750, 1000, 1250)
MAX_DOPPLER_BINS = 2048


def doppler_bins(n_fast: int) -> int:
    """Bins of a mode: 2 for the regular mode (only the bin sum reaches Y at
    offset 0), else the smallest power of two covering the 2 n_fast pulses
    of a segment, at most MAX_DOPPLER_BINS."""
    if n_fast <= 1:
        return 2
    n = 1
    while n < 2 * n_fast:
        n <<= 1
    return min(n, MAX_DOPPLER_BINS)


def sweep_scene(nx=1024, spacing=2.5, n_pulses=5000, n_gates=128, cwm=1, seed=41):
    """The sweep's scene: nx^2 facets of spacing^2 (1024^2 of 6.25 m^2: one
    tile of Sec. IV, whose scatterers are 6.24 m^2), a wind sea of U10 =
    9 m/s (fully developed: SWH 0.21 U10^2 / g = 1.73 m, peak wavelength
    67 m) plus a Gaussian swell of SWH 4 m (peak 250 m), CWM on (the Sec. IV.A
    case); the track is placed for n_pulses pulses and shared by every mode.
    Returns a Workload of the regular mode; mode() derives the others."""
    wl = workloads.make(f"nfast_sweep_{nx}sq_{spacing:g}m_g{n_gates}_p{n_pulses}",
                        nx, nx, spacing,
                        workloads.Sea(swh=1.73, peak_wavelength=67.0, seed=seed,
                                      swell=dict(swh=4.0, peak_wavelength=250.0,
                                                 sigma_kx=0.006, sigma_ky=0.006)),
                        n_gates, doppler_bins(1), 1, n_pulses, cwm=cwm)
    return wl


def mode(scene: workloads.Workload, n_fast: int) -> workloads.Workload:
    """The scene run with updates every n_fast pulses over the whole intervals
    that fit the scene's pulses (same track and window for every mode)."""
    n_pulses = scene.n_pulses
    U = n_pulses // n_fast
    radar = replace(scene.radar, n_fast=n_fast, n_doppler=doppler_bins(n_fast))
    return replace(scene, name=f"{scene.name}_nf{n_fast}", radar=radar, n_updates=U)


def run_mode(sim, prep, wl, torch, stream=None):
    """Algorithm 1 and post-processing for one mode on a prepared spectrum:
    (T_fast, Y, seconds of GPU time between events on the launch stream)."""
    st = stream if stream is not None else torch.cuda.current_stream()
    T = sim.empty_spectra(wl.n_spec)
    Y = torch.empty((wl.n_pulses, wl.radar.n_gates), dtype=sim.complex_dtype, device="cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    T.zero_()
    sim.run(None, wl.n_updates, t_fast=T, y=Y, prepared=prep, stream=st)
    e1.record(st)
    e1.synchronize()
    return T, Y, e0.elapsed_time(e1) / 1e3


# ---------------------------------------------------------------- statistics

def integrated_autocorrelation_time(x, c=5.0):
    """Integrated autocorrelation time tau = 1/2 + sum_{k>=1} rho(k) of a
    stationary series x[..., n] (last axis), with Sokal's self-consistent
    window (sum up to the first lag M >= c tau); the variance of the mean of
    n samples is var(x) 2 tau / n.  Returns tau per series (>= 1/2)."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[-1]
    d = x - x.mean(axis=-1, keepdims=True)
    m = 1 << (2 * n - 1).bit_length()
    f = np.fft.rfft(d, n=m, axis=-1)
    acov = np.fft.irfft(f * np.conj(f), n=m, axis=-1)[..., :n] / n
    var = acov[..., :1]
    rho = np.where(var > 0, acov / np.where(var > 0, var, 1.0), 0.0)
    flat = rho.reshape(-1, n)
    taus = np.empty(flat.shape[0])
    for i, r in enumerate(flat):
        tau = 0.5
        for k in range(1, n):
            tau += r[k]
            if k >= c * tau:
                break
        taus[i] = max(tau, 0.5)
    return taus.reshape(x.shape[:-1])


def mean_and_sigma(power):
    """Per-gate mean of a pulse-power series power[x, g] and the standard
    deviation of that mean (speckle): sqrt(var 2 tau / n)."""
    p = np.asarray(power, dtype=np.float64)
    n = p.shape[0]
    mean = p.mean(axis=0)
    var = p.var(axis=0)
    tau = integrated_autocorrelation_time(p.T)
    return mean, np.sqrt(var * 2.0 * tau / n), tau


def iq_correlation(Y, max_lag):
    """|<Y[x + k] conj Y[x]>| / <|Y|^2> for k = 0 .. max_lag, power-weighted
    over the gates (the pulse-to-pulse coherence of the IQ)."""
    Y = np.asarray(Y)
    n = Y.shape[0]
    p = np.sum(np.abs(Y) ** 2) / n
    return np.array([abs(np.sum(Y[k:] * np.conj(Y[:n - k]))) / (n - k) / p
                     for k in range(max_lag + 1)])


# Mean over a segment of (sqrt(1 - tau) + sqrt(tau))^2 = 1 + pi/4: the power
# gain of the eq. (1) cross-fade when the long-time signals of two
# consecutive spectra are fully coherent (eq. (1) conserves the variance of
# independent signals only).
COHERENT_POWER_GAIN = 1.0 + np.pi / 4.0


def _normalized(p, s):
    """Waveform normalised to unit sum and the standard deviation of each
    normalised gate (first order in the per-gate deviations, gates taken as
    independent)."""
    S = p.sum()
    q = p / S
    var = (s / S) ** 2 * (1.0 - 2.0 * q) + q ** 2 * np.sum((s / S) ** 2)
    return q, np.sqrt(np.maximum(var, 0.0))


def compare_waveforms(Y_fast, Y_reg, gate_floor=0.01):
    """Fidelity of a fast-mode run against the regular mode over the same
    pulses.  The waveforms are compared as the paper's Fig. 6 does, normalised
    (unit sum here): per-gate difference in units of the combined speckle
    standard deviation (the two runs see one surface, so their speckle is
    positively correlated and this is conservative), over the gates holding
    at least gate_floor of the peak power, and the relative L2 difference of
    the normalised waveforms.  The total-power ratio is reported with its
    standard deviation; eq. (1) keeps it at 1 for independent consecutive
    signals and raises it up to 1 + pi/4 for coherent ones."""
    pf, sf, tf = mean_and_sigma(np.abs(np.asarray(Y_fast)) ** 2)
    pr, sr, tr = mean_and_sigma(np.abs(np.asarray(Y_reg)) ** 2)
    qf, uf = _normalized(pf, sf)
    qr, ur = _normalized(pr, sr)
    sig = np.sqrt(uf ** 2 + ur ** 2)
    keep = pr >= gate_floor * pr.max()
    z = np.where(keep & (sig > 0), (qf - qr) / np.where(sig > 0, sig, 1.0), 0.0)
    tot_f, tot_r = pf.sum(), pr.sum()
    # total power: the per-gate means are correlated across gates as well;
    # bound its deviation by the sum of the per-gate deviations
    s_tot = np.sqrt(np.sum(sf) ** 2 + np.sum(sr) ** 2)
    return {
        "waveform_fast": pf, "waveform_regular": pr,
        "z": z, "max_abs_z": float(np.max(np.abs(z))), "gates_compared": int(keep.sum()),
        "rms_z": float(np.sqrt(np.mean(z[keep] ** 2))) if keep.any() else 0.0,
        "waveform_rel_l2": float(np.linalg.norm(qf - qr) / np.linalg.norm(qr)),
        "power_ratio": float(tot_f / tot_r), "power_ratio_sigma": float(s_tot / tot_r),
        "tau_fast_median": float(np.median(tf[keep])) if keep.any() else 0.0,
        "tau_regular_median": float(np.median(tr[keep])) if keep.any() else 0.0,
    }


def sweep(scene, n_fasts, precision, torch, with_iq=False, max_lag=32, tune=False):
    """Run the regular mode and every n_fast on the scene; returns a dict per
    mode: time, speed-up over the regular mode, facet-updates/s and (fast
    modes) the fidelity against the regular mode over the mode's pulses.
    tune: each mode's launch parameters (row path, update lanes) from the
    autotuner first (its choice is recorded as "tuning")."""
    from . import inputs, simradar
    g = scene.grid
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, scene.sea.swh, scene.sea.peak_wavelength,
                               scene.sea.seed, scene.sea.swell)
    cdt = np.complex128 if precision == simradar.SIM_PREC_FP64 else np.complex64
    spec_t = torch.as_tensor(spec.astype(cdt), device="cuda")
    del spec
    out = {}
    Y_reg = None
    t_reg = None
    for nf in (1,) + tuple(n_fasts):
        wl = mode(scene, nf)
        sim = simradar.Simulator(g, wl.radar, precision)
        tuning = None
        if tune:
            from . import autotune
            e = autotune.tune(sim, spec_t, use_cache=False,
                              run_times=[wl.update_time(j) for j in range(wl.n_spec)])
            tuning = {"row_path": e["row_path"], "row_bands": e["row_bands"],
                      "update_lanes": e["update_lanes"]}
        prep = sim.prepare_spectrum(spec_t)
        run_mode(sim, prep, wl, torch)                 # warm-up (code objects, caches)
        t0 = time.perf_counter()
        T, Y, dt = run_mode(sim, prep, wl, torch)
        wall = time.perf_counter() - t0
        Yh = Y.cpu().numpy()
        rec = {"n_fast": nf, "n_doppler": wl.radar.n_doppler, "spectra": wl.n_spec,
               "pulses": wl.n_pulses, "gpu_s": dt, "wall_s": wall,
               "facet_updates_per_s": wl.n_facets * wl.n_spec / dt,
               "iq_pulses_per_s": wl.n_pulses / dt}
        if tuning is not None:
            rec["tuning"] = tuning
        if nf == 1:
            Y_reg, t_reg = Yh, dt
        else:
            n = wl.n_pulses
            c = compare_waveforms(Yh, Y_reg[:n])
            rec.update({"speedup": t_reg / dt,
                        "max_abs_z": c["max_abs_z"], "rms_z": c["rms_z"],
                        "gates_compared": c["gates_compared"],
                        "waveform_rel_l2": c["waveform_rel_l2"],
                        "power_ratio": c["power_ratio"],
                        "power_ratio_sigma": c["power_ratio_sigma"],
                        "tau_fast_median": c["tau_fast_median"],
                        "tau_regular_median": c["tau_regular_median"]})
            if with_iq:
                cf = iq_correlation(Yh, max_lag)
                cr = iq_correlation(Y_reg[:n], max_lag)
                rec["iq_correlation_fast"] = [round(float(v), 4) for v in cf]
                rec["iq_correlation_regular"] = [round(float(v), 4) for v in cr]
                rec["iq_correlation_max_diff"] = float(np.max(np.abs(cf - cr)))
        out[nf] = rec
        del T, Y, prep
        sim.close()
        torch.cuda.empty_cache()
    return out


def sigma_of_z_bound(n_gates: int, p_false: float = 1e-3) -> float:
    """Two-sided Gaussian bound that n_gates independent unit normals all
    stay under with probability 1 - p_false (Bonferroni)."""
    from statistics import NormalDist
    return NormalDist().inv_cdf(1.0 - p_false / (2.0 * max(1, n_gates)))


__all__ = ["SWEEP_NFAST", "doppler_bins", "sweep_scene", "mode", "run_mode",
           "integrated_autocorrelation_time", "mean_and_sigma", "iq_correlation",
           "compare_waveforms", "sweep", "sigma_of_z_bound"]
