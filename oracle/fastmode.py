"""Oracle: Algorithm 1 end to end (FP64).  Test infrastructure only.

For every spectrum j = 0 .. U (Sec. III.B allocates 1 + n_pulses / n_fast
spectra), the surface and the platform are updated at the first pulse of the
pair, t_j = j n_fast / PRF, and at t_j + 1 / PRF; the scatterers are rasterised
into T_fast[j]; post-processing turns T_fast into Y.
"""
from __future__ import annotations

import numpy as np

from . import surface, scatter, iq


def update_time(j, radar):
    return (j * radar.n_fast) / radar.prf_hz


def doppler_spectrum(spec0, grid, radar, j):
    """T_fast[j] (shape G x N), the per-facet codes and the counters."""
    t = update_time(j, radar)
    fac = surface.facets(spec0, grid, t, 1.0 / radar.prf_hz)
    return scatter.accumulate(fac, grid, radar, t)


def doppler_spectra(spec0, grid, radar, n_updates):
    """T_fast of shape (U + 1, G, N)."""
    T = np.zeros((n_updates + 1, radar.n_gates, radar.n_doppler), dtype=complex)
    for j in range(n_updates + 1):
        T[j] = doppler_spectrum(spec0, grid, radar, j)[0]
    return T


def simulate(spec0, grid, radar, n_updates):
    """(T_fast, Y) for U update intervals."""
    T = doppler_spectra(spec0, grid, radar, n_updates)
    return T, iq.segments_to_iq(T, radar.n_fast, radar.window)
