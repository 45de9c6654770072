"""Oracle: Doppler spectra to range-azimuth IQ (FP64).  Test infrastructure
only.

Post-processing of Sec. III.B: allocate Y, run a batch of 1-D inverse FFTs on
the Doppler axis of T_fast, weight the long-time signals with eq. (1) and sum
them into the cells of Y.

Readings of points the paper leaves open:
* the inverse DFT is unnormalised, s_j[g, m] = sum_k T[j, g, k] exp(+2 pi i k m / N);
* spectrum j is centred on pulse c_j = j n_fast; with U + 1 spectra there are
  n_pulses = U n_fast pulses, and pulse x receives the spectra j = floor(x /
  n_fast) and j + 1;
* the offset d = x - c_j indexes the IDFT periodically, s_j[g, d mod N] (the
  exact IDFT value at any integer offset), which matters when N < 2 n_fast;
* eq. (1): W(d) = sqrt(1 - |d| / n_fast) for |d| <= n_fast, else 0;
  the alternative raised-cosine cross-fade is W(d) = cos(pi d / (2 n_fast)).
  Both satisfy sum_j W(x - c_j)^2 = 1 at every pulse (variance conservation).

Parity: pinned by sum W^2 = 1, W(0) = 1, W(+-n_fast) = 0, the centre identity
Y[j n_fast, g] = sum_k T[j, g, k], the single-bin closed form, Parseval for the
transform, and n_fast = 1 reducing to the per-pulse coherent sum.
"""
from __future__ import annotations

import numpy as np

WIN_SQRT_TRIANGLE = 0
WIN_SQRT_RAISED_COSINE = 1


def window_weight(d, n_fast, kind=WIN_SQRT_TRIANGLE):
    """Cross-fade weight of a spectrum at pulse offset d from its centre."""
    d = np.asarray(d, dtype=np.float64)
    inside = np.abs(d) <= n_fast
    if kind == WIN_SQRT_TRIANGLE:
        w = np.sqrt(np.clip(1.0 - np.abs(d) / n_fast, 0.0, None))
    elif kind == WIN_SQRT_RAISED_COSINE:
        w = np.cos(np.pi * d / (2.0 * n_fast))
    else:
        raise ValueError(f"unknown window {kind}")
    return np.where(inside, w, 0.0)


def long_time_signals(T):
    """s[j, g, m] = sum_k T[j, g, k] exp(+2 pi i k m / N) (numpy's ifft has the
    + sign and a 1/N factor)."""
    N = T.shape[-1]
    return np.fft.ifft(T, axis=-1) * N


def segments_to_iq(T, n_fast, kind=WIN_SQRT_TRIANGLE):
    """Y[x, g] for x in [0, (n_spec - 1) n_fast), shape (n_pulses, G)."""
    T = np.asarray(T, dtype=complex)
    n_spec, G, N = T.shape
    s = long_time_signals(T)
    n_pulses = (n_spec - 1) * n_fast
    Y = np.zeros((n_pulses, G), dtype=complex)
    for x in range(n_pulses):
        j0 = x // n_fast
        for j in (j0, j0 + 1):
            d = x - j * n_fast
            Y[x, :] += window_weight(d, n_fast, kind) * s[j, :, d % N]
    return Y
