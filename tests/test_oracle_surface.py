"""Pins of the oracle's sea surface (Sec. II.A: spectral surfaces with the
Choppy Wave Model; Sec. II.B: facets with normals) against brute force,
closed forms and exact identities."""
import math

import numpy as np
import pytest

import oracle.surface as osurf
from paper_2408_11472_amd import inputs, workloads
from tests import brute


def _tiny(nx=16, ny=16, cwm=1, seed=3):
    wl = workloads.tiny(nx=nx, ny=ny, spacing=2.0, cwm=cwm, seed=seed)
    spec = inputs.sea_spectrum(nx, ny, wl.grid.dx, wl.grid.dy, wl.sea.swh,
                               wl.sea.peak_wavelength, wl.sea.seed)
    return wl, spec


@pytest.mark.parametrize("nx,ny", [(8, 8), (16, 16), (16, 8)])
@pytest.mark.parametrize("cwm", [0, 1])
def test_fields_match_direct_modal_sum(nx, ny, cwm):
    wl, spec = _tiny(nx, ny, cwm)
    g = wl.grid
    t = 0.37
    f = osurf.fields(spec, g, t)
    modes = brute.mode_list(spec, nx, ny, g.dx, g.dy)
    X, Y = np.meshgrid(np.arange(nx) * g.dx, np.arange(ny) * g.dy)
    h, Dx, Dy = brute.surface_at(modes, X, Y, t, cwm=bool(cwm))
    scale = max(1e-300, np.max(np.abs(h)))
    np.testing.assert_allclose(f["h"], h, atol=1e-12 * scale, rtol=0)
    np.testing.assert_allclose(f["disp_x"], Dx, atol=1e-12 * scale, rtol=0)
    np.testing.assert_allclose(f["disp_y"], Dy, atol=1e-12 * scale, rtol=0)


@pytest.mark.parametrize("nx,ny,rows", [(16, 32, [0, 5, 31]), (32, 16, [15, 2]), (8, 64, [63])])
def test_row_subset_fields_match_direct_modal_sum(nx, ny, rows):
    wl, spec = _tiny(nx, ny, 1, seed=nx + ny)
    g = wl.grid
    t = 1.91
    f = osurf.fields_rows(spec, g, t, rows)
    modes = brute.mode_list(spec, nx, ny, g.dx, g.dy)
    X, Y = np.meshgrid(np.arange(nx) * g.dx, np.asarray(rows) * g.dy)
    h, Dx, Dy = brute.surface_at(modes, X, Y, t)
    scale = np.max(np.abs(h))
    np.testing.assert_allclose(f["h"], h, atol=1e-12 * scale, rtol=0)
    np.testing.assert_allclose(f["disp_x"], Dx, atol=1e-12 * scale, rtol=0)
    np.testing.assert_allclose(f["disp_y"], Dy, atol=1e-12 * scale, rtol=0)
    # derivative fields and facets: the rows of the whole-grid evaluation
    # (whose derivatives are pinned by finite differences below)
    full = osurf.fields(spec, g, t)
    for k in osurf.FIELDS:
        s = max(1e-300, np.max(np.abs(full[k])))
        np.testing.assert_allclose(f[k], full[k][rows], atol=1e-12 * s, rtol=0)
    fr = osurf.facets_rows(spec, g, t, 1e-3, rows)
    ff = osurf.facets(spec, g, t, 1e-3)
    for k in osurf.FACET_FIELDS:
        s = max(1e-300, np.max(np.abs(ff[k])))
        np.testing.assert_allclose(fr[k], ff[k][rows], atol=1e-11 * s, rtol=0)


@pytest.mark.parametrize("cwm", [0, 1])
def test_derivative_fields_match_finite_differences(cwm):
    nx = ny = 16
    wl, spec = _tiny(nx, ny, cwm)
    g = wl.grid
    t = 1.1
    f = osurf.fields(spec, g, t)
    modes = brute.mode_list(spec, nx, ny, g.dx, g.dy)
    X, Y = np.meshgrid(np.arange(nx) * g.dx, np.arange(ny) * g.dy)
    eps = 1e-4

    def d(axis, comp):
        if axis == 0:
            p = brute.surface_at(modes, X + eps, Y, t, cwm=bool(cwm))[comp]
            m = brute.surface_at(modes, X - eps, Y, t, cwm=bool(cwm))[comp]
        else:
            p = brute.surface_at(modes, X, Y + eps, t, cwm=bool(cwm))[comp]
            m = brute.surface_at(modes, X, Y - eps, t, cwm=bool(cwm))[comp]
        return (p - m) / (2 * eps)

    tol = 1e-7
    np.testing.assert_allclose(f["h_x"], d(0, 0), atol=tol)
    np.testing.assert_allclose(f["h_y"], d(1, 0), atol=tol)
    np.testing.assert_allclose(f["dx_x"], d(0, 1), atol=tol)
    np.testing.assert_allclose(f["dx_y"], d(1, 1), atol=tol)
    np.testing.assert_allclose(f["dx_y"], d(0, 2), atol=tol)   # Dy_x = Dx_y
    np.testing.assert_allclose(f["dy_y"], d(1, 2), atol=tol)


def test_facet_normal_matches_tangent_plane_of_displaced_surface():
    nx = ny = 16
    wl, spec = _tiny(nx, ny, 1)
    g = wl.grid
    t, dt = 0.5, 1.0 / 18000.0
    fac = osurf.facets(spec, g, t, dt)
    modes = brute.mode_list(spec, nx, ny, g.dx, g.dy)
    X, Y = np.meshgrid(np.arange(nx) * g.dx, np.arange(ny) * g.dy)
    eps = 1e-4
    rx = (brute.displaced_point(modes, X + eps, Y, t)
          - brute.displaced_point(modes, X - eps, Y, t)) / (2 * eps)
    ry = (brute.displaced_point(modes, X, Y + eps, t)
          - brute.displaced_point(modes, X, Y - eps, t)) / (2 * eps)
    n = np.cross(rx, ry)
    np.testing.assert_allclose(fac["jac"], n[..., 2], atol=1e-7)
    np.testing.assert_allclose(fac["sx"], -n[..., 0] / n[..., 2], atol=1e-6)
    np.testing.assert_allclose(fac["sy"], -n[..., 1] / n[..., 2], atol=1e-6)
    # displacement over the pulse pair = direct difference of positions
    p0 = brute.displaced_point(modes, X, Y, t)
    p1 = brute.displaced_point(modes, X, Y, t + dt)
    np.testing.assert_allclose(fac["ddisp_x"], p1[..., 0] - p0[..., 0], atol=1e-12)
    np.testing.assert_allclose(fac["ddisp_y"], p1[..., 1] - p0[..., 1], atol=1e-12)
    np.testing.assert_allclose(fac["dh"], p1[..., 2] - p0[..., 2], atol=1e-12)


def test_single_mode_is_a_trochoid_travelling_at_phase_speed():
    # one mode along +y: h = a cos(th), y = y0 - a sin(th), th = k y0 - w t + phi
    nx, ny, d = 8, 32, 1.5
    grid = workloads.Grid(nx=nx, ny=ny, dx=d, dy=d, cwm=1)
    spec = np.zeros((ny, nx), dtype=complex)
    a, phi, m = 0.8, 0.3, 3
    spec[m, 0] = a * np.exp(1j * phi)
    k = 2 * math.pi * m / (ny * d)
    w = math.sqrt(9.81 * k)
    for t in (0.0, 0.7, 2.9):
        f = osurf.fields(spec, grid, t)
        y0 = np.arange(ny)[:, None] * d * np.ones((1, nx))
        th = k * y0 - w * t + phi
        np.testing.assert_allclose(f["h"], a * np.cos(th), atol=1e-13)
        np.testing.assert_allclose(f["disp_y"], -a * np.sin(th), atol=1e-13)
        np.testing.assert_allclose(f["disp_x"], 0.0, atol=1e-13)
        np.testing.assert_allclose(f["h_y"], -a * k * np.sin(th), atol=1e-12)
        np.testing.assert_allclose(f["dy_y"], -a * k * np.cos(th), atol=1e-12)
    # crest at th = 0 travels at c = w / k
    c = w / k
    assert abs(c - math.sqrt(9.81 / k)) < 1e-12


@pytest.mark.parametrize("cwm", [0, 1])
def test_variance_identities(cwm):
    nx, ny = 64, 32
    wl = workloads.tiny(nx=nx, ny=ny, spacing=1.0, cwm=cwm, seed=5, swh=2.6)
    g = wl.grid
    spec = inputs.sea_spectrum(nx, ny, g.dx, g.dy, 2.6, 16.0, 5)
    f = osurf.fields(spec, g, 0.81)
    # SWH = 4 sigma exactly for the half-plane spectrum
    assert abs(4 * math.sqrt(np.mean(f["h"] ** 2)) - 2.6) < 1e-12
    # every field has zero mean
    for name, v in f.items():
        assert abs(np.mean(v)) < 1e-13, name
    # slope variance = 1/2 sum |k|^2 |c|^2
    KX, KY = inputs.wavenumber_grid(nx, ny, g.dx, g.dy)
    mss = 0.5 * np.sum((KX ** 2 + KY ** 2) * np.abs(spec) ** 2)
    assert abs(np.mean(f["h_x"] ** 2 + f["h_y"] ** 2) - mss) < 1e-12 * max(1.0, mss)
    if cwm:
        # |D|^2 has the variance of h; the Lagrangian map preserves mean area
        assert abs(np.mean(f["disp_x"] ** 2 + f["disp_y"] ** 2)
                   - np.mean(f["h"] ** 2)) < 1e-12
        fac = osurf.facets(spec, g, 0.81, 1e-4)
        assert abs(np.mean(fac["jac"]) - 1.0) < 1e-12
    else:
        assert np.all(f["disp_x"] == 0) and np.all(f["disp_y"] == 0)


def test_flat_sea_facets():
    grid = workloads.Grid(nx=8, ny=8, dx=1.0, dy=1.0)
    fac = osurf.facets(np.zeros((8, 8), complex), grid, 0.3, 1e-4)
    for k in ("disp_x", "disp_y", "h", "sx", "sy", "ddisp_x", "ddisp_y", "dh"):
        assert np.all(fac[k] == 0.0), k
    assert np.all(fac["jac"] == 1.0)
