"""Oracle: Choppy-Wave-Model sea surface and facets (FP64).  Test
infrastructure only.

The paper builds surrogate 3-D surfaces from prescribed spectra and adds the
Choppy Wave Model (CWM) for asymmetric, non-Gaussian profiles (Sec. II.A); the
scene is a set of facets described by vertices and normals (Sec. II.B).

Definitions used here (linear deep-water waves plus the CWM horizontal
Lagrangian displacement):

    F(x0, t) = Re sum_k M_F(k) c(k) exp(i (k . x0 - w(k) t)),  w = sqrt(g |k|)

with x0 = (ix dx, iy dy) measured from facet (0, 0) (spectral phases are
referenced to the first facet; the absolute position of facet (ix, iy) is
(x_origin + ix dx, y_origin + iy dy)).  Field multipliers M_F:

    h   : 1                    Dx  : i kx/|k|      Dy  : i ky/|k|
    h_x : i kx                 h_y : i ky
    Dx_x: -kx^2/|k|            Dx_y = Dy_x: -kx ky/|k|      Dy_y: -ky^2/|k|

(each d/dx multiplies by i kx).  With the CWM switched off the displacement
multipliers are zero.  The facet of grid point x0 sits at
P = (x0 + Dx, y0 + Dy, h); its tangents are r_x = dP/dx0 = (1 + Dx_x, Dy_x, h_x)
and r_y = dP/dy0 = (Dx_y, 1 + Dy_y, h_y); its normal n = r_x x r_y, its Jacobian
J = n_z and its slopes sx = -n_x/n_z, sy = -n_y/n_z.  The displacement of the
facet over the pulse pair is P(t + dt) - P(t), both surfaces evaluated in full
as Algorithm 1 does.

Parity: pinned by a direct (non-FFT) modal sum on small grids (the row-subset
evaluation as well), finite differences of that sum for every derivative
field and for the facet normal,
the closed-form single-mode CWM (trochoid) profile and phase speed, and the
exact variance identities of the half-plane spectrum.
"""
from __future__ import annotations

import numpy as np

FIELDS = ("h", "disp_x", "disp_y", "h_x", "h_y", "dx_x", "dx_y", "dy_y")
FACET_FIELDS = ("disp_x", "disp_y", "h", "sx", "sy", "jac",
                "ddisp_x", "ddisp_y", "dh")


def wavenumbers(grid):
    """(KX, KY) on the FFT-ordered grid of ``grid`` (shape ny, nx)."""
    kx = 2.0 * np.pi * np.fft.fftfreq(grid.nx, d=grid.dx)
    ky = 2.0 * np.pi * np.fft.fftfreq(grid.ny, d=grid.dy)
    return np.meshgrid(kx, ky)


def multipliers(grid, names=FIELDS):
    """Spectral multiplier M_F(k) of each named field (dict of complex arrays)."""
    make = _multiplier_makers(grid)
    return {n: make[n]() for n in names}


def _multiplier_makers(grid):
    """One callable per field that builds its multiplier on demand."""
    KX, KY = wavenumbers(grid)
    K = np.hypot(KX, KY)
    inv_k = np.zeros_like(K)
    np.divide(1.0, K, out=inv_k, where=K > 0)
    d = 1.0 if grid.cwm else 0.0
    make = {
        "h": lambda: np.ones_like(K, dtype=complex),
        "disp_x": lambda: d * 1j * KX * inv_k,
        "disp_y": lambda: d * 1j * KY * inv_k,
        "h_x": lambda: 1j * KX,
        "h_y": lambda: 1j * KY,
        "dx_x": lambda: d * (-(KX * KX) * inv_k) + 0j,
        "dx_y": lambda: d * (-(KX * KY) * inv_k) + 0j,
        "dy_y": lambda: d * (-(KY * KY) * inv_k) + 0j,
    }
    return make


def evolved(spec0, grid, t):
    """c(k) exp(-i w(k) t) with the deep-water dispersion relation.

    The zero mode and the Nyquist row and column carry no wave (the input
    convention of the coefficients; the generator never fills them), so they
    are cleared here."""
    KX, KY = wavenumbers(grid)
    w = np.sqrt(grid.gravity * np.hypot(KX, KY))
    c = np.array(spec0, dtype=complex)
    c[0, 0] = 0.0
    c[grid.ny // 2, :] = 0.0
    c[:, grid.nx // 2] = 0.0
    return c * np.exp(-1j * w * t)


def fields(spec0, grid, t, names=FIELDS):
    """Real fields F(x0, t) on the Lagrangian grid, shape (ny, nx) each.

    numpy's ifft2 carries a 1/(nx ny) factor and the + sign in the exponent,
    so the modal sum is ifft2(.) * nx * ny."""
    c = evolved(spec0, grid, t)
    m = multipliers(grid, names)
    scale = grid.nx * grid.ny
    return {n: np.real(np.fft.ifft2(m[n] * c)) * scale for n in names}


def fields_rows(spec0, grid, t, rows, names=FIELDS):
    """The same fields evaluated only on the grid rows ``rows`` (shape
    (len(rows), nx) each), for sampling grids too large to transform whole.

    The modal sum is taken along y by its definition, a sum over ky of
    M_F c exp(i ky y0) with the exponent reduced exactly as
    2 pi ((n_y iy) mod ny) / ny, and then along x by numpy's inverse FFT."""
    rows = np.asarray(rows, dtype=np.int64)
    c = evolved(spec0, grid, t)
    n_y = np.fft.fftfreq(grid.ny, d=1.0 / grid.ny).round().astype(np.int64)
    e = np.exp(2j * np.pi * (np.outer(rows, n_y) % grid.ny) / grid.ny)    # (r, ny)
    make = _multiplier_makers(grid)
    out = {}
    for n in names:
        part = e @ (make[n]() * c)                                          # (r, nx)
        out[n] = np.real(np.fft.ifft(part, axis=1)) * grid.nx
    return out


def facet_normal(f):
    """Normal n = r_x x r_y of the displaced facet from the field dict."""
    rx = (1.0 + f["dx_x"], f["dx_y"], f["h_x"])        # dP/dx0 (Dy_x = Dx_y)
    ry = (f["dx_y"], 1.0 + f["dy_y"], f["h_y"])        # dP/dy0
    nx = rx[1] * ry[2] - rx[2] * ry[1]
    ny = rx[2] * ry[0] - rx[0] * ry[2]
    nz = rx[0] * ry[1] - rx[1] * ry[0]
    return nx, ny, nz


def facets(spec0, grid, t, dt):
    """Facet set at time t and its displacement over the pulse pair.

    Returns the SoA dict (float64 arrays, shape (ny, nx)):
    disp_x, disp_y, h      facet position relative to its grid point
    sx, sy                 slopes -n_x/n_z, -n_y/n_z
    jac                    n_z (<= 0 marks a folded CWM facet)
    ddisp_x, ddisp_y, dh   P(t + dt) - P(t)
    """
    f0 = fields(spec0, grid, t)
    f1 = fields(spec0, grid, t + dt, names=("h", "disp_x", "disp_y"))
    return _facets_from_fields(f0, f1)


def facets_rows(spec0, grid, t, dt, rows):
    """``facets`` restricted to the grid rows ``rows`` (shape (len(rows), nx))."""
    f0 = fields_rows(spec0, grid, t, rows)
    f1 = fields_rows(spec0, grid, t + dt, rows, names=("h", "disp_x", "disp_y"))
    return _facets_from_fields(f0, f1)


def _facets_from_fields(f0, f1):
    nx, ny, nz = facet_normal(f0)
    with np.errstate(divide="ignore", invalid="ignore"):
        sx = -nx / nz
        sy = -ny / nz
    return {
        "disp_x": f0["disp_x"], "disp_y": f0["disp_y"], "h": f0["h"],
        "sx": sx, "sy": sy, "jac": nz,
        "ddisp_x": f1["disp_x"] - f0["disp_x"],
        "ddisp_y": f1["disp_y"] - f0["disp_y"],
        "dh": f1["h"] - f0["h"],
    }
