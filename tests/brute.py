"""Brute-force references for tiny inputs, written independently of the
oracle: direct modal sums evaluated at arbitrary points (no FFT), finite
differences, explicit per-facet loops."""
from __future__ import annotations

import math

import numpy as np


def mode_list(spec0, nx, ny, dx, dy):
    """Explicit list of (kx, ky, c) for every nonzero coefficient."""
    out = []
    for iy in range(ny):
        ny_ = iy if iy < ny // 2 else iy - ny
        for ix in range(nx):
            nx_ = ix if ix < nx // 2 else ix - nx
            c = complex(spec0[iy, ix])
            if c != 0:
                out.append((2 * math.pi * nx_ / (nx * dx),
                            2 * math.pi * ny_ / (ny * dy), c))
    return out


def surface_at(modes, x, y, t, g=9.81, cwm=True):
    """(h, Dx, Dy) at Lagrangian coordinates (x, y) (arrays), time t, by
    direct summation over the modes:
        h  = sum |c| cos(theta),  D = -sum (k/|k|) |c| sin(theta),
        theta = kx x + ky y - w t + arg c."""
    x = np.asarray(x, dtype=float)
    y = np.asarray(y, dtype=float)
    h = np.zeros(np.broadcast(x, y).shape)
    Dx = np.zeros_like(h)
    Dy = np.zeros_like(h)
    for kx, ky, c in modes:
        k = math.hypot(kx, ky)
        w = math.sqrt(g * k)
        th = kx * x + ky * y - w * t + math.atan2(c.imag, c.real)
        a = abs(c)
        h += a * np.cos(th)
        if cwm and k > 0:
            Dx -= (kx / k) * a * np.sin(th)
            Dy -= (ky / k) * a * np.sin(th)
    return h, Dx, Dy


def displaced_point(modes, x, y, t, **kw):
    """P(x0) = (x0 + Dx, y0 + Dy, h) with x0 measured from facet (0,0)."""
    h, Dx, Dy = surface_at(modes, x, y, t, **kw)
    return np.stack([x + Dx, y + Dy, h], axis=-1)
