"""Oracle: tabulated antenna pattern and NRCS (FP64).  Test infrastructure
only.

Sec. II.A: all antenna patterns needed by a simulation are computed once,
recorded on a u-v grid, and their complex value at each facet is obtained by
interpolation in that grid; the NRCS of the resolved facets comes from
look-up tables (computed offline with SSA1) as a function of the local
scattering geometry.  The paper prints neither table nor the interpolation
rule, so this build reads them as follows:

* antenna: a two-way complex amplitude pattern ant[iv][iu] sampled at
  u = u0 + iu du, v = v0 + iv dv, where (u, v) are the direction cosines
  along x and y of the line of sight from the platform to the facet,
  u = (P_x - S_x) / R, v = (P_y - S_y) / R (boresight at nadir);
  bilinear interpolation in the cell holding (u, v), the last row and
  column belonging to the cell before them; zero outside [u0, u0 + (nu-1) du]
  x [v0, v0 + (nv-1) dv];
* NRCS: sigma0[i] at local incidence theta_l = i dtheta (theta_l the angle
  between the facet normal and the line of sight, tan^2 theta_l as in the
  closed form), linear interpolation, zero beyond (n - 1) dtheta;
* with tables, a = sqrt(sigma0(theta_l) A) ant(u, v) (H / R)^2 is complex
  (the pattern's phase rides on the carrier phase), and stands in for the
  closed-form sqrt(sigma0_GO A) Ga (H / R)^2.

Parity: bilinear and linear interpolation are pinned by functions they
reproduce exactly (bilinear ones, node values), by the interpolation error
bound h^2 / 8 max|f''| against the closed-form beam and NRCS sampled finely,
and by the amplitude with tables of the closed forms against the closed-form
amplitude.  The tables' content is the caller's: no table of the paper is
available, so parity against the paper's SSA1 and SRAL tables is unpinned.
"""
from __future__ import annotations

import numpy as np


class Tables:
    """Antenna table ant[nv][nu] (complex) with its grid, and/or NRCS table
    sigma0[n] (real) over theta_l = i dtheta; either may be None."""

    def __init__(self, antenna=None, u0=0.0, du=1.0, v0=0.0, dv=1.0, nrcs=None, dtheta=1.0):
        self.antenna = None if antenna is None else np.asarray(antenna, dtype=complex)
        self.u0, self.du, self.v0, self.dv = float(u0), float(du), float(v0), float(dv)
        self.nrcs = None if nrcs is None else np.asarray(nrcs, dtype=np.float64)
        self.dtheta = float(dtheta)


def _cell(f, n):
    """Cell index and weight of a fractional grid coordinate f on n nodes
    (inside: 0 <= f <= n - 1; the last node belongs to cell n - 2)."""
    inside = (f >= 0.0) & (f <= n - 1)
    i = np.clip(np.floor(np.where(inside, f, 0.0)), 0, max(n - 2, 0)).astype(np.int64)
    return i, f - i, inside


def antenna_lookup(u, v, tab: Tables):
    """Bilinear interpolation of the antenna table at (u, v); 0 outside."""
    a = tab.antenna
    nv, nu = a.shape
    iu, wu, inu = _cell((np.asarray(u, dtype=np.float64) - tab.u0) / tab.du, nu)
    iv, wv, inv_ = _cell((np.asarray(v, dtype=np.float64) - tab.v0) / tab.dv, nv)
    iu1 = np.minimum(iu + 1, nu - 1)
    iv1 = np.minimum(iv + 1, nv - 1)
    val = ((1.0 - wv) * ((1.0 - wu) * a[iv, iu] + wu * a[iv, iu1])
           + wv * ((1.0 - wu) * a[iv1, iu] + wu * a[iv1, iu1]))
    return np.where(inu & inv_, val, 0.0)


def nrcs_lookup(theta, tab: Tables):
    """Linear interpolation of the NRCS table at theta; 0 outside."""
    s = tab.nrcs
    n = s.shape[0]
    i, w, inside = _cell(np.asarray(theta, dtype=np.float64) / tab.dtheta, n)
    i1 = np.minimum(i + 1, n - 1)
    return np.where(inside, (1.0 - w) * s[i] + w * s[i1], 0.0)


def line_of_sight(dx, dy, r):
    """Direction cosines (u, v) of the platform-to-facet line of sight from
    d = S - P."""
    return -dx / r, -dy / r


def local_incidence(fac, dx, dy, dz):
    """theta_l = atan(sqrt(tan^2)) with tan^2 = |d x m|^2 / (d . m)^2,
    m = (-sx, -sy, 1) (the closed-form NRCS's own incidence)."""
    sx, sy = fac["sx"], fac["sy"]
    dot = -sx * dx - sy * dy + dz
    cx = dy * 1.0 - dz * (-sy)
    cy = dz * (-sx) - dx * 1.0
    cz = dx * (-sy) - dy * (-sx)
    tan2 = (cx * cx + cy * cy + cz * cz) / (dot * dot)
    return np.arctan(np.sqrt(tan2)), tan2
