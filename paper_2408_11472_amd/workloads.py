"""Named synthetic workloads (parameter records only, no method arithmetic).

Each workload fixes a facet grid, a sea state and a nadir radar geometry in the
shape of the paper's altimetry scenario (Sec. IV: Ku band at 13.575 GHz, PRF
about 18 kHz, metre-scale facets, wind sea plus swell with the Choppy Wave
Model on).  Geometry common to all workloads:

* flat Earth, straight track along +y at constant altitude, nadir boresight;
* the track runs over the centre line of the patch and the nadir point
  crosses the patch centre half-way through the run;
* the range window starts at H - (G/2 + 1/2) dr, so a flat sea at nadir falls
  in the middle of gate G/2.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math
import random

WIN_SQRT_TRIANGLE = 0        # weights of eq. (1)
WIN_SQRT_RAISED_COSINE = 1   # power-complementary raised-cosine cross-fade

SPEED_OF_LIGHT = 299792458.0


@dataclass
class Grid:
    nx: int
    ny: int
    dx: float
    dy: float
    x_origin: float = 0.0
    y_origin: float = 0.0
    gravity: float = 9.81
    cwm: int = 1


@dataclass
class Radar:
    altitude: float = 815.0e3
    velocity: float = 7.0e3
    sat_x: float = 0.0
    sat_y0: float = 0.0
    carrier_hz: float = 13.575e9
    prf_hz: float = 18.0e3
    gate_spacing: float = 0.43
    window_start: float = 0.0
    beamwidth_3db: float = math.radians(1.3)
    fresnel_sq: float = 0.62
    mss: float = 0.01
    n_gates: int = 128
    n_doppler: int = 256
    n_fast: int = 256
    window: int = WIN_SQRT_TRIANGLE


@dataclass
class Sea:
    swh: float
    peak_wavelength: float
    seed: int
    swell: dict | None = None


@dataclass
class Workload:
    name: str
    grid: Grid
    radar: Radar
    sea: Sea
    n_updates: int                 # update intervals U; U + 1 spectra
    notes: str = ""

    @property
    def n_spec(self) -> int:
        return self.n_updates + 1

    @property
    def n_pulses(self) -> int:
        return self.n_updates * self.radar.n_fast

    @property
    def n_facets(self) -> int:
        return self.grid.nx * self.grid.ny

    def pulse_time(self, pulse_index: int) -> float:
        return pulse_index / self.radar.prf_hz

    def update_time(self, j: int) -> float:
        """Time of the first pulse of pair j (pulse j * n_fast)."""
        return (j * self.radar.n_fast) / self.radar.prf_hz


def _place(grid: Grid, radar: Radar, n_pulses: int) -> Radar:
    """Centre the track on the patch and set the range-window start."""
    run_time = n_pulses / radar.prf_hz
    xc = grid.x_origin + 0.5 * grid.nx * grid.dx
    yc = grid.y_origin + 0.5 * grid.ny * grid.dy
    return replace(
        radar,
        sat_x=xc,
        sat_y0=yc - 0.5 * radar.velocity * run_time,
        window_start=radar.altitude - (radar.n_gates / 2 + 0.5) * radar.gate_spacing,
    )


def make(name: str, nx: int, ny: int, spacing: float, sea: Sea, n_gates: int,
         n_doppler: int, n_fast: int, n_updates: int,
         window: int = WIN_SQRT_TRIANGLE, cwm: int = 1, notes: str = "",
         **radar_kw) -> Workload:
    # the patch is centred on the origin so that grid coordinates stay small
    grid = Grid(nx=nx, ny=ny, dx=spacing, dy=spacing,
                x_origin=-0.5 * nx * spacing, y_origin=-0.5 * ny * spacing,
                cwm=cwm)
    radar = Radar(n_gates=n_gates, n_doppler=n_doppler, n_fast=n_fast,
                  window=window, **radar_kw)
    radar = _place(grid, radar, n_updates * n_fast)
    return Workload(name=name, grid=grid, radar=radar, sea=sea,
                    n_updates=n_updates, notes=notes)


def small_256() -> Workload:
    """256x256 facets at 2 m, JONSWAP SWH 2 m (peak 100 m), 64 gates x 64
    Doppler bins, 8 updates of 64 pulses, raised-cosine cross-fade."""
    return make("small_256sq_2m_g64_n64_u8", 256, 256, 2.0,
                Sea(swh=2.0, peak_wavelength=100.0, seed=1), 64, 64, 64, 8,
                window=WIN_SQRT_RAISED_COSINE)


def track_4096() -> Workload:
    """4096x4096 facets at 1 m (16.8M scatterers), JONSWAP SWH 3 m (peak
    150 m), 128 gates x 256 Doppler bins, one update every 256 pulses, 64
    updates -> 65 spectra and 16384 pulses."""
    return make("track_4096sq_1m_g128_n256_u64", 4096, 4096, 1.0,
                Sea(swh=3.0, peak_wavelength=150.0, seed=2), 128, 256, 256, 64)


def gradient_2048() -> Workload:
    """2048x2048 facets at 1 m, SWH 2 m, 128 gates, 16 updates."""
    return make("grad_2048sq_1m_g128_n256_u16", 2048, 2048, 1.0,
                Sea(swh=2.0, peak_wavelength=100.0, seed=7), 128, 256, 256, 16)


def stress_8192x16384() -> Workload:
    """8192 (x) by 16384 (y) facets at 1 m (134M), swell (2.5 m, 250 m,
    sigma_k 0.006) plus wind sea (3.12 m) for 4 m total, 128 gates x 512 bins,
    n_fast 128, 512 updates -> 65536 pulses."""
    return make("stress_8192x16384_1m_g128_n512_u512", 8192, 16384, 1.0,
                Sea(swh=3.12, peak_wavelength=156.0, seed=3,
                    swell=dict(swh=2.5, peak_wavelength=250.0,
                               sigma_kx=0.006, sigma_ky=0.006)),
                128, 512, 128, 512)


def batched_16() -> list:
    """Sixteen independent realisations of uneven size run as one batch:
    6 x 1024^2, 5 x 2048^2, 3 x 4096^2 and 2 x 8192^2 facets at 1 m (2.1e8 in
    all), seeds 100..115 with the SWH of each drawn uniformly in [1, 6] m from
    its seed (peak wavelength 50 SWH), 128 gates x 256 bins, n_fast 256,
    32 updates -> 33 spectra and 8192 pulses each."""
    sides = [1024] * 6 + [2048] * 5 + [4096] * 3 + [8192] * 2
    out = []
    for r, n in enumerate(sides):
        seed = 100 + r
        swh = random.Random(seed).uniform(1.0, 6.0)
        out.append(make(f"batch{r:02d}_{n}sq_1m_g128_n256_u32", n, n, 1.0,
                        Sea(swh=swh, peak_wavelength=50.0 * swh, seed=seed),
                        128, 256, 256, 32))
    return out


def tiny(nx=16, ny=16, spacing=2.0, n_gates=16, n_doppler=8, n_fast=8,
         n_updates=2, seed=11, swh=2.0, window=WIN_SQRT_TRIANGLE, cwm=1,
         **radar_kw) -> Workload:
    """Small workload for brute-force checks."""
    return make(f"tiny_{nx}x{ny}", nx, ny, spacing,
                Sea(swh=swh, peak_wavelength=max(8.0 * spacing, 0.25 * nx * spacing),
                    seed=seed),
                n_gates, n_doppler, n_fast, n_updates, window=window, cwm=cwm,
                **radar_kw)


ALL = {
    "small_256": small_256,
    "track_4096": track_4096,
    "gradient_2048": gradient_2048,
    "stress_8192x16384": stress_8192x16384,
}

BATCHES = {
    "batched_16": batched_16,
}
