"""Autotuner of the launch parameters that do not change results beyond
summation order.

For one (grid, radar, precision) it times the fused update+accumulate call
with each candidate band count of the row pass (the number of LDS windows
per update, i.e. row-pass blocks) using the library's HIP-event timing, keeps
the fastest, and caches it in a JSON file keyed by the device name and the
shape.  Cache: $SIMRADAR_TUNING_CACHE or ~/.cache/simradar/tuning.json.
"""
from __future__ import annotations

import json
import os

CANDIDATE_BANDS = (64, 128, 256, 512)


def cache_path() -> str:
    p = os.environ.get("SIMRADAR_TUNING_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "simradar", "tuning.json")


def shape_key(sim) -> str:
    import torch
    g, r = sim.grid, sim.radar
    dev = torch.cuda.get_device_name(sim.device)
    return (f"{dev}|prec{sim.precision}|{g.nx}x{g.ny}|G{r.n_gates}|N{r.n_doppler}")


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


def tune(sim, spec0, repeats: int = 6, use_cache: bool = True) -> dict:
    """Pick the band count of the fused row pass for this simulator's shape
    and apply it.  Returns {"row_bands": n, "times_us": {...}}."""
    import torch
    key = shape_key(sim)
    cache = _load() if use_cache else {}
    if key in cache:
        sim.set_row_bands(cache[key]["row_bands"])
        return cache[key]
    T = sim.empty_spectra(2)
    times = {}
    r = sim.radar
    for nb in CANDIDATE_BANDS:
        sim.set_row_bands(nb)
        sim.update_and_accumulate(spec0, 0.0, 1, T)        # warm-up
        torch.cuda.synchronize()
        sim.profile(True)
        for i in range(repeats):
            sim.update_and_accumulate(spec0, (i * r.n_fast) / r.prf_hz, 1, T)
        prof = sim.profile_read()
        sim.profile(False)
        total = sum(ms for ms, n in prof.values())
        times[nb] = 1e3 * total / repeats
    best = min(times, key=times.get)
    sim.set_row_bands(best)
    entry = {"row_bands": best, "times_us": {str(k): round(v, 1) for k, v in times.items()}}
    if use_cache:
        cache = _load()
        cache[key] = entry
        _store(cache)
    return entry
