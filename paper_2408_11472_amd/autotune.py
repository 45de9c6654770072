"""Autotuner of the launch parameters that do not change results beyond
summation order.

For one (grid, radar, precision) it times the fused update+accumulate call
on each row path (fused row pass with each candidate band count, i.e. the
number of LDS windows and row-pass blocks per update; or the split facet
row pass + facet accumulate) using the library's HIP-event timing, keeps the
fastest (the split path on a tie within FUSED_MARGIN); then it times a short
run of updates (sim_run_updates) on 1 to 4 update lanes and keeps the
fastest (fewer lanes on a tie within LANES_MARGIN), and on more than one lane
the band count of the facet accumulate (ACC_BANDS_MARGIN).  The choice is cached in
a JSON file keyed by the shape and the library build (a rebuilt library is
tuned again).  Cache: $SIMRADAR_TUNING_CACHE or
~/.cache/simradar/tuning.json.
"""
from __future__ import annotations

import json
import os

CANDIDATE_BANDS = (64, 128, 256, 512)
# (row path, band count) pairs timed; the split path has no band count
PATH_FUSED, PATH_SPLIT = 1, 2
# The fused row pass is kept only when it beats the split path by more than
# this fraction: within it the two are a tie (timing noise decides), and the
# split path, whose kernels are timed one by one, is the stable choice.
FUSED_MARGIN = 0.02
CANDIDATE_LANES = (1, 2, 3, 4)
# More lanes are kept only when they beat fewer by more than this fraction.
# The tuner's short runs overstate the gain of lanes on large grids against a
# whole run (measured, 3 lanes against 1: 4096^2 track 7.5 % in the tuner,
# 6 % over the run; 8192 x 16384 stress 3 % in the tuner, 0.6 % slower over
# the run of 513 updates), so the margin is set between the two.
LANES_MARGIN = 0.04
# Bands of the facet accumulate tried once more than one lane is kept: fewer
# bands leave room on the CUs for the other lanes' kernels (measured on the
# 4096^2 track, whole runs on 3 lanes: 46.8 ms with 256 bands against 48.3
# with 512; on one lane 57.2 against 51.7), kept only when faster than the
# default by more than ACC_BANDS_MARGIN on the same sampled run.
CANDIDATE_ACC_BANDS = (512, 256)
ACC_BANDS_MARGIN = 0.01
# Runs of at most WHOLE_RUN_MAX updates (given their update times) are timed
# whole for the lanes and the band count, since short samples misjudge both:
# on the 4096^2 track (65 updates) a 24-update sample put 2 lanes within
# LANES_MARGIN of 3 in one run (50.7 ms per step instead of 48.5) and showed
# 0.8 % of the 3 % that 256 accumulate bands gain.  Whole runs there: 1 lane
# 51.9 ms, 2 lanes 50.5, 3 lanes 48.6, 4 lanes 48.0; the margin for whole
# runs keeps the choice away from those gaps (3 lanes).
WHOLE_RUN_MAX = 128
WHOLE_RUN_LANES_MARGIN = 0.025


def cache_path() -> str:
    p = os.environ.get("SIMRADAR_TUNING_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "simradar", "tuning.json")


_BUILD_ID = None


def library_build_id() -> str:
    """First 12 hex digits of the SHA-256 of the loaded library file: choices
    timed on one build of the kernels are not applied to another."""
    global _BUILD_ID
    if _BUILD_ID is None:
        import hashlib
        from . import simradar
        h = hashlib.sha256()
        with open(simradar.LIB_PATH, "rb") as f:
            for chunk in iter(lambda: f.read(1 << 20), b""):
                h.update(chunk)
        _BUILD_ID = h.hexdigest()[:12]
    return _BUILD_ID


def shape_key(sim) -> str:
    """Cache key of a shape: precision, grid sides, gates and bins, and the
    library build.  The cache file belongs to one machine (its path is per
    user or set by the caller); the device name is left out because some
    runtimes (a profiler's) report it empty."""
    g, r = sim.grid, sim.radar
    return (f"prec{sim.precision}|{g.nx}x{g.ny}|G{r.n_gates}|N{r.n_doppler}"
            f"|lib{library_build_id()}")


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(cache):
    p = cache_path()
    os.makedirs(os.path.dirname(p), exist_ok=True)
    tmp = p + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _apply(sim, entry):
    sim.set_row_path(entry["row_path"])
    sim.set_row_bands(entry["row_bands"])
    sim.set_update_lanes(entry.get("update_lanes", 1))
    sim.set_acc_bands(entry.get("acc_bands", 0))


def pick(times: dict) -> tuple:
    """The (row path, band count) to use from the times per update of every
    candidate: the fastest, except that a fused candidate must beat the split
    path by more than FUSED_MARGIN."""
    best = min(times, key=times.get)
    split = times.get((PATH_SPLIT, 0))
    if best[0] == PATH_FUSED and split is not None and split <= times[best] * (1 + FUSED_MARGIN):
        return (PATH_SPLIT, 0)
    return best


def pick_acc_bands(times: dict, margin: float = ACC_BANDS_MARGIN) -> int:
    """The accumulate band setting from the run time of each band count
    (512 the default): the fastest if it beats 512 by more than `margin`,
    else 0 (the default)."""
    if not times or 512 not in times:
        return 0
    best = min(times, key=times.get)
    if best != 512 and times[best] < times[512] * (1 - margin):
        return best
    return 0


def pick_lanes(times: dict, margin: float = LANES_MARGIN) -> int:
    """The lane count to use from the run time of each candidate: the
    fastest, unless fewer lanes are within `margin` of it (LANES_MARGIN for
    the tuner's short runs; a caller timing whole steps can use less)."""
    best = min(times, key=times.get)
    for n in sorted(times):
        if n < best and times[n] <= times[best] * (1 + margin):
            return n
    return best


def lane_run_updates(sim) -> int:
    """Updates per timed run of the lane tuning: about 4e8 facet-updates,
    between 24 and 192."""
    g = sim.grid
    return int(max(24, min(192, 4e8 // (g.nx * g.ny))))


def sample_times(times, n: int) -> list:
    """n of the run's update times, evenly spaced over the whole run (the
    first updates of a long track may light little of the grid, and an
    update's cost depends on how many facets it scatters)."""
    times = list(times)
    if len(times) <= n:
        return times
    return [times[(i * (len(times) - 1)) // (n - 1)] for i in range(n)]


def run_sample(sim, times):
    """The update times a tuning run uses, and whether they are the whole
    run: the run's own times when given and at most WHOLE_RUN_MAX, else
    lane_run_updates of them sampled evenly (default: the first updates at
    j n_fast / PRF)."""
    r = sim.radar
    n = lane_run_updates(sim)
    if times is None:
        return [(j * r.n_fast) / r.prf_hz for j in range(n)], False
    times = list(times)
    if len(times) <= WHOLE_RUN_MAX:
        return times, True
    return sample_times(times, n), False


def tune_lanes(sim, spec0, repeats: int = 3, times=None) -> dict:
    """Time a run of updates on each candidate lane count (HIP events on the
    launch stream, best of `repeats`); returns {lanes: ms}.  times: the
    run's update times (run_sample)."""
    times, _ = run_sample(sim, times)
    n = len(times)
    prep = sim.prepare_spectrum(spec0)
    T = sim.empty_spectra(n)
    out = {}
    for lanes in CANDIDATE_LANES:
        sim.set_update_lanes(lanes)
        out[lanes] = _time_run(sim, prep, times, T, repeats)
    return out


def _time_run(sim, prep, times, T, repeats):
    """Best of `repeats` timed runs (after one warm-up), in ms."""
    import torch
    sim.run_updates(prep, times, 0, T)                       # warm-up
    best = None
    for _ in range(repeats):
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        sim.run_updates(prep, times, 0, T)
        e1.record(st)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    return best


def tune_acc_bands(sim, spec0, repeats: int = 3, times=None) -> dict:
    """Time a run (run_sample) on the simulator's current lanes with each
    candidate accumulate band count; returns {bands: ms} ({} on one lane,
    where the default is kept).  Leaves the default set."""
    if sim.lanes <= 1:
        return {}
    times, _ = run_sample(sim, times)
    prep = sim.prepare_spectrum(spec0)
    T = sim.empty_spectra(len(times))
    out = {}
    for nb in CANDIDATE_ACC_BANDS:
        sim.set_acc_bands(nb)
        out[nb] = _time_run(sim, prep, times, T, repeats)
    sim.set_acc_bands(0)
    return out


def tune(sim, spec0, repeats: int = 6, use_cache: bool = True, run_times=None) -> dict:
    """Pick the row path and the band count of the fused row pass for this
    simulator's shape, then the update lanes (on the run's update times
    `run_times` when given) and on more than one lane the accumulate band
    count, and apply them.  Returns {"row_path": p, "row_bands": n,
    "times_us": {...}, "update_lanes": l, "lanes_ms": {...}, "acc_bands": b,
    "acc_bands_ms": {...}} (times per update of every row path candidate, run
    times of every lane count and accumulate band count; b = 0: default)."""
    import torch
    key = shape_key(sim)
    cache = _load() if use_cache else {}
    if key in cache and all(k in cache[key] for k in ("row_path", "update_lanes", "acc_bands")):
        _apply(sim, cache[key])
        return cache[key]
    T = sim.empty_spectra(2)
    times = {}
    r = sim.radar
    cands = [(PATH_FUSED, nb) for nb in CANDIDATE_BANDS] + [(PATH_SPLIT, 0)]
    for path, nb in cands:
        sim.set_row_path(path)
        sim.set_row_bands(nb)
        sim.update_and_accumulate(spec0, 0.0, 1, T)        # warm-up
        torch.cuda.synchronize()
        sim.profile(True)
        for i in range(repeats):
            sim.update_and_accumulate(spec0, (i * r.n_fast) / r.prf_hz, 1, T)
        prof = sim.profile_read()
        sim.profile(False)
        total = sum(ms for ms, n in prof.values())
        times[(path, nb)] = 1e3 * total / repeats
    best = pick(times)
    sim.set_row_path(best[0])
    sim.set_row_bands(best[1])
    lane_ms = tune_lanes(sim, spec0, times=run_times)
    whole = run_sample(sim, run_times)[1]
    lanes = pick_lanes(lane_ms, WHOLE_RUN_LANES_MARGIN if whole else LANES_MARGIN)
    sim.set_update_lanes(lanes)
    acc_ms = tune_acc_bands(sim, spec0, times=run_times)
    entry = {"row_path": best[0], "row_bands": best[1],
             "times_us": {("fused%d" % nb if p == PATH_FUSED else "split"): round(v, 1)
                          for (p, nb), v in times.items()},
             "update_lanes": lanes,
             "lanes_ms": {str(k): round(v, 3) for k, v in lane_ms.items()},
             "lanes_updates": len(run_sample(sim, run_times)[0]),
             "lanes_whole_run": whole,
             "acc_bands": pick_acc_bands(acc_ms),
             "acc_bands_ms": {str(k): round(v, 3) for k, v in acc_ms.items()}}
    _apply(sim, entry)
    if use_cache:
        cache = _load()
        cache[key] = entry
        _store(cache)
    return entry


def tune_batch(batch, specs, T, Y=None, repeats: int = 2, shapes: bool = True) -> dict:
    """Pick the batch mode (lanes or persistent launches) by timing replays of
    the captured graph of each, and, with shapes=True, tune the row path of
    every member shape first (lanes mode runs each member through the
    context's row path; the persistent launches use the split path).
    The lanes mode is also timed with 256 accumulate bands for every member,
    kept when it beats both modes by more than ACC_BANDS_MARGIN.  Returns
    {"mode": ..., "acc_bands": b, "times_ms": {...}, "shapes": {...}}."""
    import time

    import torch
    from . import simradar
    out = {"shapes": {}}
    if shapes:
        seen = {}
        for g, r, s in zip(batch.grids, batch.radars, specs):
            key = (g.nx, g.ny, r.n_gates, r.n_doppler)
            if key in seen:
                continue
            sim = simradar.Simulator(g, r, batch.precision, device=batch.device.index or 0)
            seen[key] = tune(sim, s)
            sim.close()
        out["shapes"] = {f"{k[0]}x{k[1]}_G{k[2]}_N{k[3]}": v for k, v in seen.items()}
        # every member runs (in the lanes mode) with its shape's values
        for i, (g, r) in enumerate(zip(batch.grids, batch.radars)):
            e = seen[(g.nx, g.ny, r.n_gates, r.n_doppler)]
            simradar.sim_batch_set_tuning(batch.batch, i, simradar.SIM_TUNE_ROW_PATH,
                                          e["row_path"])
            simradar.sim_batch_set_tuning(batch.batch, i, simradar.SIM_TUNE_ROW_BANDS,
                                          e["row_bands"])
    def set_acc_bands(nb):
        for i in range(len(batch.grids)):
            simradar.sim_batch_set_tuning(batch.batch, i, simradar.SIM_TUNE_ACC_BANDS, nb)

    times = {}
    # the lanes mode also with 256 accumulate bands for every member (members
    # on different streams overlap, as update lanes do)
    for name, mode, nb in (("lanes", simradar.SIM_BATCH_LANES, 0),
                           ("persistent", simradar.SIM_BATCH_PERSISTENT, 0),
                           ("lanes_acc256", simradar.SIM_BATCH_LANES, 256)):
        set_acc_bands(nb)
        batch.set_mode(mode)
        batch.run(specs, T, Y, use_graph=True)            # capture + warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(repeats):
            batch.run(specs, T, Y, use_graph=True)
        torch.cuda.synchronize()
        times[name] = (time.perf_counter() - t0) / repeats * 1e3
    best = min(("lanes", "persistent"), key=times.get)
    if times["lanes_acc256"] < times[best] * (1 - ACC_BANDS_MARGIN):
        best = "lanes_acc256"
    set_acc_bands(256 if best == "lanes_acc256" else 0)
    batch.set_mode(simradar.SIM_BATCH_PERSISTENT if best == "persistent"
                   else simradar.SIM_BATCH_LANES)
    out.update({"mode": "lanes" if best == "lanes_acc256" else best,
                "acc_bands": 256 if best == "lanes_acc256" else 0,
                "times_ms": {k: round(v, 3) for k, v in times.items()}})
    return out
