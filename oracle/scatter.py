"""Oracle: facet scatterers and rasterisation into Doppler spectra (FP64).
Test infrastructure only.

Follows Algorithm 1 (Sec. III.B) for one spectrum j: the complex amplitude of
every facet at the first pulse of the pair, its range, its pulse-pair Doppler
arg(C' conj(C)) PRF / (2 pi), and the sum of the amplitudes per (range gate,
Doppler interval) - the "rasterize" step.  The facet radar equation on complex
amplitudes follows Sec. II.A; the paper's look-up tables (SSA1 NRCS, u-v antenna
patterns) are not available, so closed forms stand in (see below).

Definitions (every step in float64, in this order, no fused multiply-add):

  satellite   S(t) = (sat_x, sat_y0 + v t, H); second pulse at t' = t + 1/PRF
  facet       P = (x_origin + ix dx + disp_x, y_origin + iy dy + disp_y, h),
              P' = (P_x + ddisp_x, P_y + ddisp_y, P_z + dh)
  range       d = S - P, R = sqrt((d_x d_x + d_y d_y) + d_z d_z); same for R'
  gate        xi = (R - R_w0) / dr, g = floor(xi), kept when 0 <= xi < G
  Doppler     k2 = 2 f_c / c, u_raw = -(R' - R) k2 (cycles per pulse, the
              pulse-pair phase step over 2 pi), u = u_raw - floor(u_raw + 1/2)
              in [-1/2, 1/2), bin = floor(N u + 1/2) mod N (FFT order, bin 0 is
              zero Doppler, u = +1/2 goes to bin N/2)
  facing      q = -sx d_x - sy d_y + d_z (n . d up to a positive factor);
              the facet is kept when q > 0
  amplitude   tan^2 = |d x m|^2 / (d . m)^2 with m = (-sx, -sy, 1);
              cos^2 = 1 / (1 + tan^2);
              sigma0 = |G0|^2 / (mss cos^4) exp(-tan^2 / mss)   (geometric optics)
              A = jac sqrt(1 + sx^2 + sy^2) dx dy                (facet area)
              gamma = (2 / ln 2) sin^2(theta_3dB / 2),
              Ga = exp(-(2 / gamma) (d_x^2 + d_y^2) / R^2)      (two-way beam)
              a = sqrt(sigma0 A) Ga (H / R)^2
  phase       cyc = R k2, frac = cyc - floor(cyc), C = a exp(-2 pi i frac)
              (= a exp(-i 4 pi R / lambda))

Drop rules, tested in this order, each dropped facet counted once:
  nonfinite (any input field not finite), folded (jac <= 0),
  out_of_window (xi outside [0, G)), backfacing (q <= 0).

Parity: the index rules and the phase are pinned by a point scatterer in
closed-form geometry and by the static flat sea (all power in bin 0, gate
populations equal to annulus counts).  The NRCS, beam and radar constant are
this build's stand-ins for tables the paper does not print: their values are
pinned by closed forms at special points (nadir, known tilt), not against the
paper (parity unpinned against the paper for those constants).
"""
from __future__ import annotations

import numpy as np

SPEED_OF_LIGHT = 299792458.0

CODE_NONFINITE = -1
CODE_FOLDED = -2
CODE_OUT_OF_WINDOW = -3
CODE_BACKFACING = -4

COUNTER_NAMES = ("illuminated", "out_of_window", "folded", "backfacing",
                 "nonfinite")


def doppler_constant(radar):
    """k2 = 2 f_c / c  [cycles of two-way phase per metre of range]."""
    return 2.0 * radar.carrier_hz / SPEED_OF_LIGHT


def grid_coordinates(grid):
    """Absolute x0, y0 of every grid point, shape (ny, nx)."""
    ix = np.arange(grid.nx, dtype=np.float64)
    iy = np.arange(grid.ny, dtype=np.float64)
    x0 = grid.x_origin + ix * grid.dx
    y0 = grid.y_origin + iy * grid.dy
    return np.broadcast_to(x0[None, :], (grid.ny, grid.nx)), \
        np.broadcast_to(y0[:, None], (grid.ny, grid.nx))


def pulse_pair_ranges(fac, grid, radar, t):
    """Facet-to-satellite vectors and ranges at the two pulses of the pair."""
    x0, y0 = grid_coordinates(grid)
    px = x0 + fac["disp_x"]
    py = y0 + fac["disp_y"]
    pz = fac["h"]
    sy = radar.sat_y0 + radar.velocity * t
    dx = radar.sat_x - px
    dy = sy - py
    dz = radar.altitude - pz
    r = np.sqrt((dx * dx + dy * dy) + dz * dz)
    t2 = t + 1.0 / radar.prf_hz
    sy2 = radar.sat_y0 + radar.velocity * t2
    px2 = px + fac["ddisp_x"]
    py2 = py + fac["ddisp_y"]
    pz2 = pz + fac["dh"]
    dx2 = radar.sat_x - px2
    dy2 = sy2 - py2
    dz2 = radar.altitude - pz2
    r2 = np.sqrt((dx2 * dx2 + dy2 * dy2) + dz2 * dz2)
    return dx, dy, dz, r, r2


def gate_coordinate(r, radar):
    """xi = (R - R_w0) / dr; the gate is floor(xi)."""
    return (r - radar.window_start) / radar.gate_spacing


def doppler_cycles(r, r2, radar):
    """Pulse-pair phase step in cycles, wrapped into [-1/2, 1/2)."""
    u_raw = -(r2 - r) * doppler_constant(radar)
    return u_raw - np.floor(u_raw + 0.5)


def doppler_bin(u, n_doppler):
    """Nearest Doppler bin (round half up) in FFT order."""
    kk = np.floor(n_doppler * u + 0.5).astype(np.int64)
    return np.mod(kk, n_doppler)


def amplitude_tables(fac, grid, radar, dx, dy, dz, r, tables):
    """Complex amplitude with the tabulated NRCS and/or antenna pattern
    (oracle.tables; a missing table falls back to its closed form):
    a = sqrt(sigma0 A) G (H / R)^2."""
    from . import tables as otab
    sx, sy, jac = fac["sx"], fac["sy"], fac["jac"]
    theta, tan2 = otab.local_incidence(fac, dx, dy, dz)
    if tables.nrcs is not None:
        sigma0 = otab.nrcs_lookup(theta, tables)
    else:
        cos2 = 1.0 / (1.0 + tan2)
        sigma0 = radar.fresnel_sq / (radar.mss * cos2 * cos2) * np.exp(-tan2 / radar.mss)
    area = jac * np.sqrt(1.0 + sx * sx + sy * sy) * grid.dx * grid.dy
    if tables.antenna is not None:
        u, v = otab.line_of_sight(dx, dy, r)
        ga = otab.antenna_lookup(u, v, tables)
    else:
        gamma = (2.0 / np.log(2.0)) * np.sin(0.5 * radar.beamwidth_3db) ** 2
        ga = np.exp(-(2.0 / gamma) * (dx * dx + dy * dy) / (r * r))
    hr = radar.altitude / r
    return np.sqrt(sigma0 * area) * ga * hr * hr


def amplitude(fac, grid, radar, dx, dy, dz, r):
    """Real amplitude a of each facet (see module header)."""
    sx, sy, jac = fac["sx"], fac["sy"], fac["jac"]
    # m = (-sx, -sy, 1) is the facet normal scaled by 1/jac
    dot = -sx * dx - sy * dy + dz
    cx = dy * 1.0 - dz * (-sy)
    cy = dz * (-sx) - dx * 1.0
    cz = dx * (-sy) - dy * (-sx)
    tan2 = (cx * cx + cy * cy + cz * cz) / (dot * dot)
    cos2 = 1.0 / (1.0 + tan2)
    sigma0 = radar.fresnel_sq / (radar.mss * cos2 * cos2) * np.exp(-tan2 / radar.mss)
    area = jac * np.sqrt(1.0 + sx * sx + sy * sy) * grid.dx * grid.dy
    gamma = (2.0 / np.log(2.0)) * np.sin(0.5 * radar.beamwidth_3db) ** 2
    sin2 = (dx * dx + dy * dy) / (r * r)
    ga = np.exp(-(2.0 / gamma) * sin2)
    hr = radar.altitude / r
    return np.sqrt(sigma0 * area) * ga * hr * hr


def carrier_phase(r, radar):
    """exp(-2 pi i frac(R k2)) = exp(-i 4 pi R / lambda)."""
    cyc = r * doppler_constant(radar)
    frac = cyc - np.floor(cyc)
    return np.exp(-2j * np.pi * frac)


def scatterers(fac, grid, radar, t, tables=None):
    """Per-facet code (g N + bin, or a negative drop code) and amplitude C
    (closed forms, or the look-up tables of oracle.tables when given)."""
    G, N = radar.n_gates, radar.n_doppler
    fac = {k: np.asarray(v, dtype=np.float64) for k, v in fac.items()}
    finite = np.ones(fac["h"].shape, dtype=bool)
    for v in fac.values():
        finite &= np.isfinite(v)
    safe = {k: np.where(finite, v, 0.0) for k, v in fac.items()}
    with np.errstate(all="ignore"):
        dx, dy, dz, r, r2 = pulse_pair_ranges(safe, grid, radar, t)
        xi = gate_coordinate(r, radar)
        u = doppler_cycles(r, r2, radar)
        q = -safe["sx"] * dx - safe["sy"] * dy + dz
        in_win = (xi >= 0.0) & (xi < G)
        folded = safe["jac"] <= 0.0
        code = np.full(xi.shape, CODE_NONFINITE, dtype=np.int64)
        ok = finite & ~folded & in_win & (q > 0.0)
        g = np.floor(np.where(in_win, xi, 0.0)).astype(np.int64)
        k = doppler_bin(u, N)
        code[ok] = (g * N + k)[ok]
        code[finite & folded] = CODE_FOLDED
        code[finite & ~folded & ~in_win] = CODE_OUT_OF_WINDOW
        code[finite & ~folded & in_win & ~(q > 0.0)] = CODE_BACKFACING
        if tables is None:
            a = amplitude(safe, grid, radar, dx, dy, dz, r)
        else:
            a = amplitude_tables(safe, grid, radar, dx, dy, dz, r, tables)
        c = np.where(ok, a * carrier_phase(r, radar), 0.0)
    return code, c


def rasterize(code, c, radar):
    """T[g, k] = sum of C over the facets whose code is g N + k (Algorithm 1,
    "rasterize": sum the data in the tensor by coordinates)."""
    G, N = radar.n_gates, radar.n_doppler
    ok = code >= 0
    idx = code[ok]
    re = np.bincount(idx, weights=np.real(c[ok]), minlength=G * N)
    im = np.bincount(idx, weights=np.imag(c[ok]), minlength=G * N)
    return (re + 1j * im).reshape(G, N)


def counters(code):
    """Counts of illuminated and dropped facets by reason."""
    return {
        "illuminated": int(np.count_nonzero(code >= 0)),
        "out_of_window": int(np.count_nonzero(code == CODE_OUT_OF_WINDOW)),
        "folded": int(np.count_nonzero(code == CODE_FOLDED)),
        "backfacing": int(np.count_nonzero(code == CODE_BACKFACING)),
        "nonfinite": int(np.count_nonzero(code == CODE_NONFINITE)),
    }


def accumulate(fac, grid, radar, t, tables=None):
    """One Doppler spectrum [G, N] from a facet set at pulse time t, plus the
    per-facet codes and the drop counters."""
    code, c = scatterers(fac, grid, radar, t, tables)
    return rasterize(code, c, radar), code, counters(code)
