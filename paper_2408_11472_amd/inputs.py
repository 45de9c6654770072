"""Seeded synthetic inputs: directional wave spectra and their random-phase
coefficients.

This module produces the *input* of the fast-mode path, the complex spectral
coefficients of the sea surface at t = 0 (the paper builds its surfaces from
prescribed spectra, Sec. II.A).  It holds none of the method's arithmetic: no
surface synthesis, no scattering, no Doppler processing.  Both the CPU oracle
(through the tests) and the HIP path consume the arrays it returns.

Spectral family (the paper names wind speed and a Gaussian swell, Sec. IV.A and
IV.D, but no wind-sea family): JONSWAP in frequency, converted to wavenumber
with the deep-water dispersion relation, times a cos^2 spreading on the half
plane around the wind direction.  Swell: a Gaussian in (kx, ky) as in the
S1/S2 sea states of Sec. IV.D.

Array convention: coefficients are returned as ``c[iy, ix]`` in FFT order, where
``ix`` indexes kx = 2 pi n_x / (nx dx), n_x = ix for ix < nx/2 and ix - nx
otherwise (same for y).  The zero mode and the Nyquist row and column are zero.
The support lies on the half plane ky > 0, so no +k/-k pair is populated and
the surface variance equals 1/2 sum |c|^2 exactly; the coefficients are scaled
so that 4 sqrt(1/2 sum |c|^2) equals the requested significant wave height.
"""
from __future__ import annotations

import numpy as np

GRAVITY = 9.81


def wavenumber_grid(nx: int, ny: int, dx: float, dy: float):
    """Return (KX, KY) of shape (ny, nx) in FFT order [rad/m]."""
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=dx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=dy)
    KX, KY = np.meshgrid(kx, ky)
    return KX, KY


def _support_mask(nx: int, ny: int) -> np.ndarray:
    """Half plane ky > 0 without the Nyquist row/column (FFT order)."""
    m = np.zeros((ny, nx), dtype=bool)
    m[1:ny // 2, :] = True          # n_y in [1, ny/2 - 1]
    if nx > 1:
        m[:, nx // 2] = False       # Nyquist column n_x = -nx/2
    return m


def jonswap_density(nx, ny, dx, dy, peak_wavelength, gamma=3.3,
                    wind_dir=0.5 * np.pi, g=GRAVITY) -> np.ndarray:
    """Directional variance density Psi(kx, ky) [m^4] (unnormalised level).

    JONSWAP S(w) ~ w^-5 exp(-5/4 (wp/w)^4) gamma^r, converted to k with
    dw/dk = g / (2 w), spread as (2/pi) cos^2(theta - wind_dir) on the half plane
    facing the wind, and divided by k for the polar-to-Cartesian Jacobian.
    Only the shape matters: the level is fixed later by the requested SWH.
    """
    KX, KY = wavenumber_grid(nx, ny, dx, dy)
    K = np.hypot(KX, KY)
    psi = np.zeros_like(K)
    pos = K > 0
    w = np.sqrt(g * K[pos])
    kp = 2.0 * np.pi / peak_wavelength
    wp = np.sqrt(g * kp)
    sigma = np.where(w <= wp, 0.07, 0.09)
    r = np.exp(-((w - wp) ** 2) / (2.0 * sigma ** 2 * wp ** 2))
    s_w = g ** 2 * w ** -5.0 * np.exp(-1.25 * (wp / w) ** 4) * gamma ** r
    f_k = s_w * g / (2.0 * w)
    theta = np.arctan2(KY[pos], KX[pos])
    c = np.cos(theta - wind_dir)
    spread = np.where(c > 0.0, (2.0 / np.pi) * c * c, 0.0)
    psi[pos] = f_k * spread / K[pos]
    return psi


def gaussian_swell_density(nx, ny, dx, dy, peak_wavelength, sigma_kx, sigma_ky,
                           direction=0.5 * np.pi) -> np.ndarray:
    """Gaussian swell density centred on k_p = 2 pi / peak_wavelength along
    ``direction`` with standard deviations (sigma_kx, sigma_ky) [rad/m]
    (the S1/S2 form of Sec. IV.D); unnormalised level."""
    KX, KY = wavenumber_grid(nx, ny, dx, dy)
    kp = 2.0 * np.pi / peak_wavelength
    kx0, ky0 = kp * np.cos(direction), kp * np.sin(direction)
    return np.exp(-0.5 * ((KX - kx0) / sigma_kx) ** 2
                  - 0.5 * ((KY - ky0) / sigma_ky) ** 2)


def coefficients(psi: np.ndarray, dx: float, dy: float, swh: float,
                 seed: int) -> np.ndarray:
    """Random-phase coefficients c = sqrt(2 Psi dkx dky) exp(i phi), restricted
    to the half-plane support and scaled to the requested SWH.  complex128."""
    ny, nx = psi.shape
    dkx = 2.0 * np.pi / (nx * dx)
    dky = 2.0 * np.pi / (ny * dy)
    mask = _support_mask(nx, ny)
    amp = np.sqrt(2.0 * np.where(mask, psi, 0.0) * dkx * dky)
    rng = np.random.default_rng(np.uint64(seed))
    phi = 2.0 * np.pi * rng.random((ny, nx))
    c = amp * np.exp(1j * phi)
    var = 0.5 * np.sum(np.abs(c) ** 2)
    if var <= 0.0:
        raise ValueError("spectrum has no energy on this grid")
    c *= (swh / 4.0) / np.sqrt(var)
    return c


def sea_spectrum(nx, ny, dx, dy, swh, peak_wavelength, seed, swell=None):
    """Spectral coefficients of a wind sea (JONSWAP, SWH ``swh``) plus an
    optional Gaussian swell ``swell = dict(swh, peak_wavelength, sigma_kx,
    sigma_ky)``; the two parts draw independent phases, so their variances add
    on average."""
    wind = coefficients(jonswap_density(nx, ny, dx, dy, peak_wavelength),
                        dx, dy, swh, seed)
    if swell is None:
        return wind
    sw = coefficients(gaussian_swell_density(nx, ny, dx, dy,
                                             swell["peak_wavelength"],
                                             swell["sigma_kx"],
                                             swell["sigma_ky"]),
                      dx, dy, swell["swh"], seed + 7919)
    return wind + sw


def random_facets(nx, ny, seed, slope_rms=0.1, height_rms=1.0,
                  disp_rms=0.5, dz_rms=1e-3, ddisp_rms=1e-5):
    """Synthetic facet fields (SoA dict of float64 arrays, shape (ny, nx)) used
    to exercise the scatterer/rasterisation step on its own."""
    rng = np.random.default_rng(np.uint64(seed))
    f = {
        "disp_x": disp_rms * rng.standard_normal((ny, nx)),
        "disp_y": disp_rms * rng.standard_normal((ny, nx)),
        "h": height_rms * rng.standard_normal((ny, nx)),
        "sx": slope_rms * rng.standard_normal((ny, nx)),
        "sy": slope_rms * rng.standard_normal((ny, nx)),
        "jac": 1.0 + 0.05 * rng.standard_normal((ny, nx)),
        "ddisp_x": ddisp_rms * rng.standard_normal((ny, nx)),
        "ddisp_y": ddisp_rms * rng.standard_normal((ny, nx)),
        "dh": dz_rms * rng.standard_normal((ny, nx)),
    }
    return f


def random_spectra(n_spec, n_gates, n_doppler, seed):
    """Random complex Doppler-spectrum tensor (n_spec, n_gates, n_doppler)."""
    rng = np.random.default_rng(np.uint64(seed))
    return (rng.standard_normal((n_spec, n_gates, n_doppler))
            + 1j * rng.standard_normal((n_spec, n_gates, n_doppler)))
