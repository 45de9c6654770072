"""Negative control of the precision reading (the paper states no precision;
the satellite-to-facet range and the carrier phase are kept in double).

Planted in the oracle on the CPU: the same scatterers with the facet
positions, both pulse ranges, the gate and Doppler coordinates and the phase
evaluated in float32.  At ~815 km one float32 ulp of range is 0.0625 m, i.e.
~36 rad of Ku-band carrier phase:

* the phase taken as 4 pi R / lambda in float32 (a ~4.6e8 rad argument with a
  32 rad ulp) is unrelated to the true one; and since the float32 ranges
  take only a few dozen values over the patch, facets of one cell share
  their phases and add coherently, so the relative L2 error is far above 1
  (not the sqrt(2) of two independent random-phase spectra);
* the phase taken as the fraction of R 2 f_c / c in float32, as the double
  path does, is identically zero (the ~7.4e7 cycles have an ulp of 8), so
  every facet adds in phase and the error is larger still.

The pulse-pair Doppler fails the same way: R' - R is a multiple of the
0.0625 m ulp, ~5.7 cycles, for a true value of ~1e-3 m."""
import numpy as np

import oracle.scatter as osc
import oracle.surface as osurf
from paper_2408_11472_amd import inputs, workloads


def _scatterers_float32_range(fac, grid, radar, t, naive_phase):
    """oracle.scatter.scatterers with the range and phase in float32."""
    f32 = np.float32
    x0, y0 = osc.grid_coordinates(grid)
    px = x0.astype(f32) + fac["disp_x"].astype(f32)
    py = y0.astype(f32) + fac["disp_y"].astype(f32)
    pz = fac["h"].astype(f32)
    sy1 = f32(radar.sat_y0 + radar.velocity * t)
    sy2 = f32(radar.sat_y0 + radar.velocity * (t + 1.0 / radar.prf_hz))
    dx = f32(radar.sat_x) - px
    dy = sy1 - py
    dz = f32(radar.altitude) - pz
    r = np.sqrt((dx * dx + dy * dy) + dz * dz)
    ex = f32(radar.sat_x) - (px + fac["ddisp_x"].astype(f32))
    ey = sy2 - (py + fac["ddisp_y"].astype(f32))
    ez = f32(radar.altitude) - (pz + fac["dh"].astype(f32))
    r2 = np.sqrt((ex * ex + ey * ey) + ez * ez)
    k2 = f32(osc.doppler_constant(radar))
    xi = (r - f32(radar.window_start)) / f32(radar.gate_spacing)
    u_raw = -(r2 - r) * k2
    u = u_raw - np.floor(u_raw + f32(0.5))
    G, N = radar.n_gates, radar.n_doppler
    ok = (xi >= 0) & (xi < G) & (fac["jac"] > 0)
    g = np.floor(np.where(ok, xi, 0)).astype(np.int64)
    k = np.mod(np.floor(N * u + f32(0.5)).astype(np.int64), N)
    code = np.where(ok, g * N + k, osc.CODE_OUT_OF_WINDOW)
    a = osc.amplitude(fac, grid, radar, dx.astype(float), dy.astype(float), dz.astype(float),
                      r.astype(float))
    if naive_phase:
        phi = (f32(2.0 * np.pi) * k2) * r
        ph = (np.cos(phi) - 1j * np.sin(phi)).astype(complex)
    else:
        cyc = r * k2
        ph = np.exp(-2j * np.pi * (cyc - np.floor(cyc)).astype(float))
    return code, np.where(ok, a * ph, 0.0)


def test_float32_range_and_phase_decorrelate_the_spectrum():
    wl = workloads.small_256()
    g, r = wl.grid, wl.radar
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)
    t = wl.update_time(4)
    fac = osurf.facets(spec, g, t, 1.0 / r.prf_hz)
    T64 = osc.accumulate(fac, g, r, t)[0]
    errs, dist, corr = {}, {}, {}
    for naive in (True, False):
        code32, c32 = _scatterers_float32_range(fac, g, r, t, naive)
        T32 = osc.rasterize(code32, c32, r)
        errs[naive] = np.linalg.norm(T32 - T64) / np.linalg.norm(T64)
        a, b = T32 / np.linalg.norm(T32), T64 / np.linalg.norm(T64)
        dist[naive] = np.linalg.norm(a - b)
        corr[naive] = abs(np.vdot(a, b))
        label = "4 pi R / lambda" if naive else "fraction of R 2 f_c / c"
        print(f"PRECISION small_256 float32-range T_fast[j] {errs[naive]:.3e} "
              f"(negative control, phase {label} in float32; correlation {corr[naive]:.3f}, "
              f"normalised distance {dist[naive]:.3f})")
    assert errs[True] > 10.0 and errs[False] > 10.0, errs
