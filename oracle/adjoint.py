"""Oracle: multi-look waveform, L2 waveform loss and its gradient with respect
to the facet heights and slopes (FP64).  Test infrastructure only.

The paper multi-looks the echoes to reduce speckle before retracking
(Sec. IV.B) and aims at inverting sea-state parameters from simulated data
(Sec. V).  Here the differentiable chain is

    facets (h, sx, sy per update) -> C_f -> T_fast (rasterize, Algorithm 1)
      -> Y (post-processing, Sec. III.B) -> P[g] = mean_x |Y[x, g]|^2
      -> L = sum_g (P[g] - P_target[g])^2.

Gate and Doppler-bin indices are piecewise constant (zero derivative); the
pulse-pair displacement and the other facet fields are held fixed, so a
change of h moves both pulses of a pair and the bin stays put.

Gradient convention for a real loss of complex z = x + i y: the complex
gradient is dL/dx + i dL/dy.  For a complex-linear map Y = A T it transforms
as T_bar = A^H Y_bar, and for C = C(theta) with theta real,
dL/dtheta = Re(conj(C_bar) dC/dtheta).

Parity: the IQ adjoint is pinned by the dot-product identity
<A T, Y> = <T, A^H Y>; the whole gradient by central finite differences of
the forward oracle on facets away from gate and bin edges.
"""
from __future__ import annotations

import numpy as np

from . import iq, scatter


def waveform(Y):
    """P[g] = (1 / n_pulses) sum_x |Y[x, g]|^2 (multi-look over the run)."""
    Y = np.asarray(Y)
    return np.mean(np.abs(Y) ** 2, axis=0)


def loss(P, target):
    return float(np.sum((np.asarray(P) - np.asarray(target)) ** 2))


def loss_grad_y(Y, target):
    """Y_bar = dL/dRe(Y) + i dL/dIm(Y) = 2 (P - target)[g] * 2 Y / n_pulses."""
    Y = np.asarray(Y)
    P = waveform(Y)
    dP = 2.0 * (P - np.asarray(target))
    return dP[None, :] * 2.0 * Y / Y.shape[0]


def segments_to_iq_adjoint(Ybar, n_spec, n_doppler, n_fast, kind=iq.WIN_SQRT_TRIANGLE):
    """T_bar[j, g, k] = sum_x W(x - c_j) Y_bar[x, g] exp(-2 pi i k ((x - c_j) mod N) / N)
    over the pulses x of the run that spectrum j reaches (the transpose of
    the overlap-add, written as its definition)."""
    Ybar = np.asarray(Ybar, dtype=complex)
    n_pulses, G = Ybar.shape
    N = n_doppler
    Tbar = np.zeros((n_spec, G, N), dtype=complex)
    k = np.arange(N)
    for j in range(n_spec):
        c = j * n_fast
        for x in range(max(0, c - n_fast + 1), min(n_pulses, c + n_fast)):
            d = x - c
            w = iq.window_weight(d, n_fast, kind)
            if w == 0.0:
                continue
            ph = np.exp(-2j * np.pi * k * (d % N) / N)
            Tbar[j] += w * Ybar[x, :, None] * ph[None, :]
    return Tbar


def facet_gradients(fac, grid, radar, t, Tbar_j):
    """dL/dh, dL/dsx, dL/dsy of every facet of one update from T_bar[j].

    C = a exp(i phi) with phi = -2 pi frac(R k2); for theta in (h, sx, sy):
    dC/dtheta = C (d ln a / dtheta + i d phi / dtheta), where
      ln a = 1/2 ln(|G0|^2 A / mss) + ln(1 + tan^2) - tan^2 / (2 mss)
             - (2 / gamma) sin^2 + 2 ln H - 2 ln R,
      tan^2 = |c|^2 / q^2, c = d x m, q = d . m, m = (-sx, -sy, 1),
      d = S - P, dd/dh = (0, 0, -1), dm/dsx = (-1, 0, 0), dm/dsy = (0, -1, 0),
      A = jac sqrt(1 + sx^2 + sy^2) dx dy, dR/dh = -d_z / R.
    Dropped facets have zero gradient."""
    code, C = scatter.scatterers(fac, grid, radar, t)
    f = {k: np.asarray(v, dtype=np.float64) for k, v in fac.items()}
    ok = code >= 0
    safe = {k: np.where(ok, v, 0.0) for k, v in f.items()}
    dx, dy, dz, r, _ = scatter.pulse_pair_ranges(safe, grid, radar, t)
    sx, sy = safe["sx"], safe["sy"]
    mx, my, mz = -sx, -sy, 1.0
    cx = dy * mz - dz * my
    cy = dz * mx - dx * mz
    cz = dx * my - dy * mx
    q = dx * mx + dy * my + dz * mz
    c2 = cx * cx + cy * cy + cz * cz
    with np.errstate(all="ignore"):
        tan2 = c2 / (q * q)
        gamma = (2.0 / np.log(2.0)) * np.sin(0.5 * radar.beamwidth_3db) ** 2
        rho2 = dx * dx + dy * dy
        sin2 = rho2 / (r * r)
        s2 = 1.0 + sx * sx + sy * sy

        def dtan2(dcx, dcy, dcz, dq):
            return 2.0 * (cx * dcx + cy * dcy + cz * dcz) / (q * q) - 2.0 * c2 * dq / (q ** 3)

        def dlna(dtan, dlnA, dsin2, dlnR):
            return 0.5 * dlnA + dtan / (1.0 + tan2) - dtan / (2.0 * radar.mss) \
                - (2.0 / gamma) * dsin2 - 2.0 * dlnR

        k2 = scatter.doppler_constant(radar)
        # theta = h
        dR_h = -dz / r
        t_h = dtan2(-sy, sx, 0.0 * sx, -1.0)
        dsin2_h = -2.0 * sin2 * dR_h / r
        g_h = dlna(t_h, 0.0, dsin2_h, dR_h / r) + 1j * (-2.0 * np.pi * k2 * dR_h)
        # theta = sx: dc = d x (-1, 0, 0) = (0, -dz, dy), dq = -dx
        t_sx = dtan2(0.0 * dz, -dz, dy, -dx)
        g_sx = dlna(t_sx, sx / s2, 0.0, 0.0) + 0j
        # theta = sy: dc = d x (0, -1, 0) = (dz, 0, -dx), dq = -dy
        t_sy = dtan2(dz, 0.0 * dz, -dx, -dy)
        g_sy = dlna(t_sy, sy / s2, 0.0, 0.0) + 0j
    N = radar.n_doppler
    Cbar = np.zeros(C.shape, dtype=complex)
    idx = np.where(ok)
    cc = code[ok]
    Cbar[idx] = Tbar_j[cc // N, cc % N]
    out = {}
    for name, g in (("h", g_h), ("sx", g_sx), ("sy", g_sy)):
        out[name] = np.where(ok, np.real(np.conj(Cbar) * C * g), 0.0)
    return out


def forward_loss(facet_list, times, grid, radar, target):
    """L for a list of facet sets (one per spectrum) and their pulse times."""
    G, N = radar.n_gates, radar.n_doppler
    T = np.zeros((len(facet_list), G, N), dtype=complex)
    for j, (fac, t) in enumerate(zip(facet_list, times)):
        T[j] = scatter.accumulate(fac, grid, radar, t)[0]
    Y = iq.segments_to_iq(T, radar.n_fast, radar.window)
    return loss(waveform(Y), target), T, Y


def gradients(facet_list, times, grid, radar, target):
    """(L, [grads per spectrum]) by the hand adjoint."""
    L, T, Y = forward_loss(facet_list, times, grid, radar, target)
    Ybar = loss_grad_y(Y, target)
    Tbar = segments_to_iq_adjoint(Ybar, len(facet_list), radar.n_doppler, radar.n_fast,
                                  radar.window)
    grads = [facet_gradients(f, grid, radar, t, Tbar[j])
             for j, (f, t) in enumerate(zip(facet_list, times))]
    return L, grads
