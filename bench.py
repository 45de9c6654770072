"""Throughput of the fast-mode hot path on one MI355X.

One step = the whole path on the 4096 x 4096-facet nadir workload (16.8M
facets at 1 m, SWH 3 m, 128 gates x 256 Doppler bins, 65 spectra = 64 update
intervals of 256 pulses, 16384 IQ pulses): for each spectrum the surface is
synthesised and every facet rasterised (fused update+accumulate), then the
spectra are inverse transformed, cross-faded and overlap-added into IQ.

Prints one JSON line.  `value` is facet-updates/s of the FP32 context (range
and phase in FP64); the plain FP64 context is reported beside it, with the
FP32 context's relative L2 distance to it.  The along-track stress workload
(8192 x 16384 facets, 513 spectra) and the batch of 16 uneven realisations
are timed for a few steps each and reported as sub-objects.  Every spectrum is
generated on the host once and is resident in HBM before timing.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, GB/s
METRIC = "facet-updates/s + simulated IQ pulses/s (FP32+FP64-phase vs FP64, same GPU)"

# Algorithmic HBM bytes of one facet-update (one facet processed for one
# spectrum), FP32 context (FP64 doubles them): read the spectrum once (8 B)
# and one write plus one read of the six packed complex intermediates of the
# out-of-LDS 2-D transform (2 x 48 B).  Facet sets, scatterers and the
# per-update spectra and IQ are not algorithmic traffic.
ALG_BYTES_PER_FACET_UPDATE = 8 + 2 * 48
# Each kernel's share of those bytes: the column pass reads the spectrum and
# writes the intermediates, a row pass reads them back; the facet accumulate
# moves none (its facet fields are the split path's own round trip).
ALG_SHARE = {"surface_colpass": 8 + 48, "surface_rowpass": 48, "fused_rowpass": 48,
             "accumulate_facets": 0}
# What this layout actually has to move (eight half-width planes of the
# columns kx >= 0: 32 B written and 32 B read per facet), for reference.
LAYOUT_SHARE = {"surface_colpass": 8 + 32, "surface_rowpass": 32, "fused_rowpass": 32,
                "accumulate_facets": 0}

# HBM bytes per launch measured with rocprofv3 FETCH_SIZE (x2.000) and
# WRITE_SIZE (x1.000), scaled by a 1 GiB copy in the same runs
# (profiles/track_4096_hbm_counters.md; the autotuned launch shapes of the
# track: 256 accumulate bands in float, 512 in double), valid only for the
# kernel sources they were taken on.
KERNEL_SOURCES = ("kernels.hip", "device_common.hpp", "scatter.hpp", "launch.hpp")
MEASURED = {
    "source_sha": "8f63f3bf2156d9cf",
    "fp32": {"surface_colpass": 812e6, "surface_rowpass": 1141e6,
             "accumulate_facets": 606e6, "reduce_partials": 2e6},
    "fp64": {"surface_colpass": 1347e6, "surface_rowpass": 2283e6,
             "accumulate_facets": 1211e6, "reduce_partials": 3e6},
}
PER_UPDATE_KERNELS = ("surface_colpass", "surface_rowpass", "fused_rowpass", "accumulate_facets",
                      "reduce_partials")


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2408_11472_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--workload", default="track_4096")
    p.add_argument("--no-fp64", action="store_true", help="skip the FP64 context")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extra", action="store_true",
                   help="skip the stress and batched sub-objects of the default line")
    p.add_argument("--extra-steps", type=int, default=2,
                   help="timed steps of the stress and batched workloads in the default line")
    p.add_argument("--no-autotune", action="store_true",
                   help="skip the autotuner (row path and band count per shape, batch mode)")
    p.add_argument("--tuning-cache", action="store_true",
                   help="take the autotuner's choice from its cache file when it has one "
                        "(a profiled run then launches no candidate)")
    p.add_argument("--copy-calibration-mib", type=int, default=0,
                   help="before timing, copy a buffer of this size once (a plain copy kernel "
                        "of known traffic, to scale the HBM byte counters of a profiler run)")
    return p.parse_args()


def path_roofline(bytes_per_fu, facet_updates, seconds):
    """Whole path against the HBM peak: algorithmic bytes of the facet-updates
    of the timed region over its duration."""
    alg = bytes_per_fu * facet_updates
    achieved = alg / seconds / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4)}


def timed_steps(sim, spec_t, wl, steps, warmup, torch):
    """Warm-up steps, then `steps` timed steps for the throughput (HIP events
    on the launch stream around the timed region, plus the host clock), then
    as many again with the library's per-kernel HIP events (recorded on the
    launch stream around every kernel) for the kernel times.  The per-kernel
    events cost about 3 % of a step, so they are kept out of the throughput's
    timed region."""
    T = sim.empty_spectra(wl.n_spec)
    Y = torch.empty((wl.n_pulses, wl.radar.n_gates), dtype=sim.complex_dtype, device="cuda")
    prep = sim.prepare_spectrum(spec_t)

    def step():
        T.zero_()
        sim.run(spec_t, wl.n_updates, t_fast=T, y=Y, prepared=prep)

    def timed(n):
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(st)
        for _ in range(n):
            step()
        e1.record(st)
        torch.cuda.synchronize()
        return time.perf_counter() - t0, e0.elapsed_time(e1) / 1e3

    for _ in range(warmup):
        step()
    dt, dt_ev = timed(steps)
    sim.profile(True)
    dt_prof, _ = timed(steps)
    prof = sim.profile_read()
    sim.profile(False)
    return dt, dt_ev, dt_prof, prof, T, Y, prep


def dominant_kernel(prof, wl, scale, measured_ok, prec_name):
    """The per-update kernel with the most time, credited with its share of
    the algorithmic bytes only; measured HBM traffic per launch beside it."""
    best = max((k for k in ALG_SHARE if prof[k][1]), key=lambda k: prof[k][0])
    ms, n = prof[best]
    avg_s = ms / 1e3 / n
    alg = ALG_SHARE[best] * scale * wl.n_facets
    achieved = alg / avg_s / 1e9
    return {"kernel": best, "bound": "hbm", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "alg_bytes_per_facet": ALG_SHARE[best] * scale,
            "layout_bytes_per_facet": LAYOUT_SHARE[best] * scale,
            "avg_launch_us": round(avg_s * 1e6, 2), "alg_bytes_per_launch": alg,
            "traffic": MEASURED[prec_name].get(best) if measured_ok else None}


def copy_bandwidth(torch, mib=1024, reps=5):
    """GB/s of a plain device copy of `mib` MiB (read + write), HIP events on
    the current stream, best of `reps`."""
    n = mib * 1024 * 1024 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        s = e0.elapsed_time(e1) / 1e3
        best = s if best is None else min(best, s)
    del src, dst
    return {"bytes": 2 * n * 4, "gbs": round(2 * n * 4 / best / 1e9, 1)}


def _oracle_spectrum(args):
    """One spectrum of the oracle (worker process): seconds taken."""
    spec, grid, radar, j = args
    import oracle.fastmode as ofm
    t0 = time.perf_counter()
    ofm.doppler_spectrum(spec, grid, radar, j)
    return time.perf_counter() - t0


def cpu_baseline(spec, wl):
    """The oracle, as it stands, on the host's cores: one whole spectrum of
    the full workload per worker process (spectra are independent), as many
    workers as cores (at most the 16 of one GPU's share), plus one spectrum on
    a single core."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    ncpu = os.cpu_count() or 1
    workers = max(1, min(16, ncpu))
    t1 = _oracle_spectrum((spec, wl.grid, wl.radar, wl.n_updates // 2))
    js = [(spec, wl.grid, wl.radar, (wl.n_updates // 2 + k) % wl.n_spec) for k in range(workers)]
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                          "MKL_NUM_THREADS")}
    for k in env:
        os.environ[k] = "1"    # one thread per worker process
    try:
        t0 = time.perf_counter()
        with ProcessPoolExecutor(max_workers=workers,
                                 mp_context=multiprocessing.get_context("spawn")) as ex:
            list(ex.map(_oracle_spectrum, js))
        dt = time.perf_counter() - t0
    finally:
        for k, v in env.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return {"value": round(workers * wl.n_facets / dt, 1), "unit": "facet-updates/s",
            "cores": workers, "kind": "oracle",
            "single_core_value": round(wl.n_facets / t1, 1),
            "host_cpus": ncpu,
            "sample": f"{workers} whole spectra of the full {wl.grid.nx}x{wl.grid.ny} workload, "
                      f"one per worker process (numpy float64, one thread each), {dt:.1f} s "
                      f"wall including worker start-up; single core: one spectrum in {t1:.1f} s"}


def run_delay_doppler(sim, Y, torch, burst=64, reps=20):
    """Delay-Doppler processing (bursts of 64 pulses, centroid estimated per
    burst, range migration corrected, multi-look) of the step's IQ: time per
    call (HIP events on the launch stream), the HBM bytes it must move (the
    IQ read twice, the beams written and read back by the range pass and read
    by the multi-look).  Its agreement with the oracle is the tests' business
    (the oracle runs here only in the CPU-baseline leg)."""
    st = torch.cuda.current_stream()
    out = sim.delay_doppler(Y, burst=burst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        out = sim.delay_doppler(Y, burst=burst)
    e1.record(st)
    e1.synchronize()
    s = e0.elapsed_time(e1) / 1e3 / reps
    nb = Y.shape[0] // burst
    cs = Y.element_size()
    moved = 2 * Y.numel() * cs + 4 * nb * burst * Y.shape[1] * cs
    return {"burst": burst, "bursts": nb, "ms_per_call": round(s * 1e3, 4),
            "bytes_per_call": moved, "achieved_gbs": round(moved / s / 1e9, 1),
            "waveform_finite": bool(torch.isfinite(out["waveform"]).all().item())}


def run_batch(a, members, steps, warmup, torch):
    """The batched-realisations workload: all members on one context, replayed
    as one captured HIP graph per step (FP32 + FP64 phase)."""
    import numpy as np
    from paper_2408_11472_amd import inputs, simradar
    specs = []
    for w in members:
        g = w.grid
        s = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, w.sea.swh, w.sea.peak_wavelength,
                                w.sea.seed, w.sea.swell)
        specs.append(torch.as_tensor(s.astype(np.complex64), device="cuda"))
        del s
    batch = simradar.Batch([(w.grid, w.radar, w.n_updates) for w in members],
                           simradar.SIM_PREC_FP32_PHASE64)
    T, Y = batch.empty_outputs()
    tuning = None
    if not a.no_autotune:
        from paper_2408_11472_amd import autotune
        tuning = autotune.tune_batch(batch, specs, T, Y, repeats=1)
    batch.run(specs, T, Y, use_graph=False)
    torch.cuda.synchronize()
    batch.profile(True)
    batch.run(specs, T, Y, use_graph=False)
    torch.cuda.synchronize()
    prof = batch.profile_read()
    batch.profile(False)
    for _ in range(warmup):
        batch.run(specs, T, Y, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        batch.run(specs, T, Y, use_graph=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fu = sum(w.n_facets * w.n_spec for w in members)
    pulses = sum(w.n_pulses for w in members)
    out = {"workload": "batched_16", "realisations": len(members),
           "facets": sum(w.n_facets for w in members), "facet_updates_per_step": fu,
           "steps": steps, "warmup": warmup, "graph": True,
           "ms_per_step": round(dt / steps * 1e3, 3),
           "value": round(fu * steps / dt, 1), "unit": "facet-updates/s",
           "iq_pulses_per_s": round(pulses * steps / dt, 1),
           "roofline": path_roofline(ALG_BYTES_PER_FACET_UPDATE, fu * steps, dt),
           "mode": "persistent" if getattr(batch, "mode", 2) == 2 else "lanes",
           "tuning": tuning,
           "eager_kernels_ms": {k: round(v[0], 3) for k, v in prof.items() if v[1]}}
    batch.close()
    del specs, T, Y
    torch.cuda.empty_cache()
    return out


def run_single(a, wl, steps, warmup, torch, with_fp64=True, cpu=True):
    """The single-realisation line (both contexts on the same spectrum)."""
    import numpy as np
    from paper_2408_11472_amd import inputs, simradar
    g = wl.grid
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed, wl.sea.swell)
    measured_ok = kernel_source_sha() == MEASURED["source_sha"] and wl.name.startswith("track_4096")
    results, keep = {}, {}
    for name, prec, cdt, scale in (("fp32", simradar.SIM_PREC_FP32_PHASE64, np.complex64, 1),
                                   ("fp64", simradar.SIM_PREC_FP64, np.complex128, 2)):
        if name == "fp64" and not with_fp64:
            continue
        try:
            sim = simradar.Simulator(g, wl.radar, prec)
        except simradar.SimError as e:
            if name == "fp64" and e.status == simradar.SIM_ERR_UNSUPPORTED:
                results[name] = {"unsupported": str(e)}
                continue
            raise
        spec_t = torch.as_tensor(spec.astype(cdt), device="cuda")
        tuning = None
        if not a.no_autotune:
            from paper_2408_11472_amd import autotune
            tuning = autotune.tune(sim, spec_t, use_cache=a.tuning_cache,
                                   run_times=[wl.update_time(j) for j in range(wl.n_spec)])
        dt, dt_ev, dt_prof, prof, T, Y, prep = timed_steps(sim, spec_t, wl, steps, warmup, torch)
        fu = wl.n_facets * wl.n_spec * steps
        ms_step = dt / steps * 1e3
        upd = {k: prof[k] for k in PER_UPDATE_KERNELS if prof[k][1]}
        traffic = None
        if measured_ok and all(k in MEASURED[name] for k in upd):
            # measured HBM bytes of one update: every per-update kernel's
            # bytes per launch times its launches per update
            traffic = sum(MEASURED[name][k] * (n / (wl.n_spec * steps)) for k, (_, n) in upd.items())
        roof = path_roofline(ALG_BYTES_PER_FACET_UPDATE * scale, fu, dt_ev)
        roof.update({"scope": "whole path per step (all update kernels and the IQ "
                              "post-processing), HIP events on the launch stream",
                     "alg_bytes_per_facet_update": ALG_BYTES_PER_FACET_UPDATE * scale,
                     "facet_updates_per_step": wl.n_facets * wl.n_spec,
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per update (rocprofv3 counters)",
                     "alg_bytes_per_update": ALG_BYTES_PER_FACET_UPDATE * scale * wl.n_facets,
                     "dominant_kernel": dominant_kernel(prof, wl, scale, measured_ok, name)})
        # with several update lanes the launches of different updates overlap:
        # a launch's duration then includes the time it shares the CUs
        roof["dominant_kernel"].update({"update_lanes": sim.lanes,
                                        "launches_overlap": sim.lanes > 1})
        dd = (run_delay_doppler(sim, Y, torch)
              if name == "fp32" and wl.name.startswith("track_4096") else None)
        # one more update with per-facet codes (outside the timed region)
        code = torch.empty((g.ny, g.nx), dtype=torch.int32, device="cuda")
        cnt = sim.counters()
        Tc = sim.empty_spectra(wl.n_spec)
        jc = wl.n_updates // 2 + 1
        sim.update_and_accumulate_prepared(prep, wl.update_time(jc), jc, Tc, counters=cnt,
                                           facet_code=code)
        torch.cuda.synchronize()
        keep[name] = (T.cpu().numpy().astype(np.complex128), Y.cpu().numpy().astype(np.complex128),
                      code.cpu().numpy(), int(cnt.cpu()[0]))
        results[name] = {
            "ms_per_step": round(ms_step, 3),
            "event_ms_per_step": round(dt_ev / steps * 1e3, 3),
            "profiled_ms_per_step": round(dt_prof / steps * 1e3, 3),
            "ms_per_update": round(ms_step / wl.n_spec, 4),
            "facet_updates_per_s": fu / dt,
            "iq_pulses_per_s": wl.n_pulses * steps / dt,
            "kernels_ms_per_step": {k: round(v[0] / steps, 4) for k, v in prof.items() if v[1]},
            "roofline": roof,
            "finite": bool(torch.isfinite(torch.view_as_real(Y)).all().item()),
            "tuning": tuning,
            "delay_doppler": dd,
        }
        print(f"[bench] {wl.name} {name}: {ms_step:.2f} ms/step  "
              f"{results[name]['facet_updates_per_s']:.3e} facet-updates/s  "
              f"kernels {results[name]['kernels_ms_per_step']}", file=sys.stderr, flush=True)
        del T, Y, spec_t, prep, Tc, code
        sim.close()
        del sim
        torch.cuda.empty_cache()
    precision = None
    if "fp32" in keep and "fp64" in keep:
        def rl2(x, y):
            return float(np.linalg.norm(x - y) / np.linalg.norm(y))
        T32, Y32, c32, n_ill = keep["fp32"]
        T64, Y64, c64, _ = keep["fp64"]
        precision = {"reference": "FP64 context on the same GPU (pinned to the FP64 oracle)",
                     "T_fast_rel_l2": rl2(T32, T64), "Y_rel_l2": rl2(Y32, Y64),
                     "index_mismatches_per_update": int((c32 != c64).sum()),
                     "illuminated_per_update": n_ill}
    cpu_line = cpu_baseline(spec, wl) if cpu else None
    return results, precision, cpu_line


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {a.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2408_11472_amd import workloads
    if a.workload in workloads.BATCHES:
        out = run_batch(a, workloads.BATCHES[a.workload](), a.steps, a.warmup, torch)
        line = {"metric": METRIC, "value": out["value"], "unit": "facet-updates/s",
                "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
                "ms_per_step": out["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "f32", "data": "synthetic",
                "config": {"workload": "batched_16", "realisations": out["realisations"],
                           "facets": out["facets"], "range_phase": "f64",
                           "parallelism": "single-gpu"},
                "iq_pulses_per_s": out["iq_pulses_per_s"], "roofline": out["roofline"],
                "eager_kernels_ms": out["eager_kernels_ms"]}
        print(json.dumps(line), flush=True)
        return
    if a.workload == "gradient_2048":
        main_gradient(a, workloads.gradient_2048())
        return
    if a.workload == "nfast_sweep":
        out = run_nfast_sweep(torch, with_iq=True, tune=not a.no_autotune)
        line = {"metric": METRIC, "value": out["regular"]["facet_updates_per_s"],
                "unit": "facet-updates/s", "n_gpus": 1, "steps": 1, "warmup": 1,
                "ms_per_step": round(out["regular"]["gpu_s"] * 1e3, 3),
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "f32", "data": "synthetic",
                "config": {"workload": out["workload"], "range_phase": "f64",
                           "parallelism": "single-gpu"},
                "nfast_sweep": out}
        print(json.dumps(line), flush=True)
        return

    if a.copy_calibration_mib > 0:
        n = a.copy_calibration_mib * 1024 * 1024 // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    wl = workloads.ALL[a.workload]()
    copy = copy_bandwidth(torch)
    results, precision, cpu_line = run_single(a, wl, a.steps, a.warmup, torch,
                                              with_fp64=not a.no_fp64,
                                              cpu=not a.no_cpu_baseline)
    r32 = results["fp32"]
    line = {
        "metric": METRIC,
        "value": round(r32["facet_updates_per_s"], 1),
        "unit": "facet-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": r32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "facets": wl.n_facets, "spectra": wl.n_spec,
                   "n_gates": wl.radar.n_gates, "n_doppler": wl.radar.n_doppler,
                   "n_fast": wl.radar.n_fast, "pulses": wl.n_pulses,
                   "range_phase": "f64", "parallelism": "single-gpu"},
        "iq_pulses_per_s": round(r32["iq_pulses_per_s"], 1),
        "ms_per_update": r32["ms_per_update"],
        "kernels_ms_per_step": r32["kernels_ms_per_step"],
        "event_ms_per_step": r32["event_ms_per_step"],
        "profiled_ms_per_step": r32["profiled_ms_per_step"],
        "roofline": r32["roofline"],
        "copy_bandwidth": copy,
        "tuning": r32["tuning"],
        "delay_doppler": r32["delay_doppler"],
    }
    if "fp64" in results:
        r64 = results["fp64"]
        line["fp64"] = ({"value": round(r64["facet_updates_per_s"], 1),
                         "iq_pulses_per_s": round(r64["iq_pulses_per_s"], 1),
                         "ms_per_step": r64["ms_per_step"],
                         "ms_per_update": r64["ms_per_update"],
                         "profiled_ms_per_step": r64["profiled_ms_per_step"],
                         "kernels_ms_per_step": r64["kernels_ms_per_step"],
                         "roofline": r64["roofline"]} if "unsupported" not in r64 else r64)
    if precision is not None:
        line["precision"] = precision
    if not a.no_extra and a.workload == "track_4096":
        st, _, _ = run_single(a, workloads.stress_8192x16384(), a.extra_steps, 1, torch,
                              with_fp64=False, cpu=False)
        s32 = st["fp32"]
        sw = workloads.stress_8192x16384()
        line["stress_8192x16384"] = {
            "workload": sw.name, "facets": sw.n_facets, "spectra": sw.n_spec,
            "pulses": sw.n_pulses, "steps": a.extra_steps, "warmup": 1,
            "ms_per_step": s32["ms_per_step"], "ms_per_update": s32["ms_per_update"],
            "value": round(s32["facet_updates_per_s"], 1), "unit": "facet-updates/s",
            "iq_pulses_per_s": round(s32["iq_pulses_per_s"], 1),
            "kernels_ms_per_step": s32["kernels_ms_per_step"],
            "tuning": s32["tuning"],
            "roofline": {k: v for k, v in s32["roofline"].items() if k != "traffic"}}
        line["batched_16"] = run_batch(a, workloads.batched_16(), max(2, a.extra_steps), 1, torch)
        line["nfast_sweep"] = run_nfast_sweep(torch, tune=not a.no_autotune)
    # The paper gives only end-to-end wall times of its own scenario (Sec. IV:
    # 3.51e8 scatterers, 267379 pulses) on 4 GTX 1080; the rate they imply for
    # the fast mode at n_fast = 250 is quoted as context, not as a target.
    line["paper_context"] = {"facet_updates_per_s": 3.1e8, "hardware": "4 x GeForce GTX 1080",
                             "basis": "end-to-end wall time of the paper's scenario at "
                                      "n_fast = 250 (20 min), static costs included"}
    if cpu_line is not None:
        line["cpu_baseline"] = cpu_line
    print(json.dumps(line), flush=True)


def run_nfast_sweep(torch, with_iq=False, nx=1024, n_pulses=5000, tune=True):
    """Regular mode (a surface update at every pulse) and the fast mode at
    n_fast = 250 .. 1250 on one 1024^2-facet scene of 6.25 m^2 scatterers
    (wind sea + 4 m swell, CWM on), 5000 pulses, FP32 with double range and
    phase: GPU time and speed-up per mode (the paper's Fig. 4) and the
    fidelity of each fast-mode multi-look waveform against the regular mode's
    (the paper's Fig. 6), in units of the speckle standard deviation."""
    from paper_2408_11472_amd import nfast, simradar
    scene = nfast.sweep_scene(nx=nx, n_pulses=n_pulses)
    res = nfast.sweep(scene, nfast.SWEEP_NFAST, simradar.SIM_PREC_FP32_PHASE64, torch,
                      with_iq=with_iq, tune=tune)
    reg = res[1]

    def clean(r):
        return {k: (round(v, 6) if isinstance(v, float) else v) for k, v in r.items()}
    return {"workload": scene.name, "facets": scene.n_facets, "pulses": scene.n_pulses,
            "regular": clean(reg),
            "fast": [clean(res[nf]) for nf in nfast.SWEEP_NFAST]}


def main_gradient(a, wl):
    """The differentiable chain on its workload: facet fields of every update
    (from the surface update) as inputs, forward (scatterers, IQ, waveform,
    loss) and backward (hand adjoint to dL/dh, dL/dsx, dL/dsy) per step, FP32
    context with range and phase in double."""
    import numpy as np
    import torch

    from paper_2408_11472_amd import inputs, simradar
    from paper_2408_11472_amd.autograd import FIXED_FIELDS, waveform_loss
    g, r = wl.grid, wl.radar
    sim = simradar.Simulator(g, r, simradar.SIM_PREC_FP32_PHASE64)
    times = [wl.update_time(j) for j in range(wl.n_spec)]

    def fields(seed):
        spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                                   seed, wl.sea.swell)
        st = torch.as_tensor(spec.astype(np.complex64), device="cuda")
        out = {k: torch.empty((wl.n_spec, g.ny, g.nx), dtype=torch.float32, device="cuda")
               for k in simradar.FACET_FIELDS}
        for j, t in enumerate(times):
            sim.surface_update(st, t, 1.0 / r.prf_hz, out={k: out[k][j] for k in out})
        return out

    target_f = fields(wl.sea.seed + 1)
    T = sim.empty_spectra(wl.n_spec)
    for j, t in enumerate(times):
        sim.range_doppler_accumulate({k: target_f[k][j] for k in simradar.FACET_FIELDS}, t, j, T)
    target, _ = sim.waveform_loss(sim.segments_to_iq(T))
    del target_f, T
    f = fields(wl.sea.seed)
    fixed = {k: f[k] for k in FIXED_FIELDS}
    h = f["h"].requires_grad_(True)
    sx = f["sx"].requires_grad_(True)
    sy = f["sy"].requires_grad_(True)

    def step():
        L = waveform_loss(h, sx, sy, sim, fixed, times, target)
        gh, gsx, gsy = torch.autograd.grad(L, (h, sx, sy))
        return L, gh

    # update lanes of the run calls (forward accumulate, adjoint): a few
    # whole steps on each lane count, the fewest within 1 % of the fastest
    lanes_ms, bands_ms = {}, {}

    def step_ms():
        for _ in range(2):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / 5 * 1e3

    if not a.no_autotune:
        from paper_2408_11472_amd import autotune
        for lanes in autotune.CANDIDATE_LANES:
            sim.set_update_lanes(lanes)
            lanes_ms[lanes] = step_ms()
        sim.set_update_lanes(autotune.pick_lanes(lanes_ms, margin=0.01))
        # then the band count of the forward accumulate, on those lanes
        if sim.lanes > 1:
            for nb in autotune.CANDIDATE_ACC_BANDS:
                sim.set_acc_bands(nb)
                bands_ms[nb] = step_ms()
            sim.set_acc_bands(autotune.pick_acc_bands(bands_ms))
    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        L, gh = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fu = wl.n_facets * wl.n_spec
    line = {
        "metric": METRIC, "value": round(fu * a.steps / dt, 1), "unit": "facet-updates/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(dt / a.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "facets": wl.n_facets, "spectra": wl.n_spec,
                   "step": "forward + backward of the waveform loss", "range_phase": "f64",
                   "parallelism": "single-gpu"},
        "loss": float(L.detach()), "grad_h_finite": bool(torch.isfinite(gh).all().item()),
        "update_lanes": sim.lanes,
        "lanes_ms_per_step": {str(k): round(v, 3) for k, v in lanes_ms.items()} or None,
        "acc_bands": autotune.pick_acc_bands(bands_ms) if bands_ms else 0,
        "acc_bands_ms_per_step": {str(k): round(v, 3) for k, v in bands_ms.items()} or None,
    }
    print(json.dumps(line), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
