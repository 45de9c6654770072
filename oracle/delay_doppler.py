"""Oracle: Delay-Doppler processing of the range-azimuth IQ (FP64).  Test
infrastructure only.

Sec. IV.C focuses the simulated IQ with a Delay-Doppler algorithm: the pulses
are cut into bursts of 64, and for each burst

1. the Doppler-centroid shift is removed (the trajectory is not exactly
   tangent to the surface);
2. an along-track FFT over the pulses of the burst forms Doppler beams
   (finer azimuth resolution);
3. the range migration of the scatterers of each Doppler beam is undone with
   delay phase coefficients;

and the Doppler strips are averaged (multi-look) to reduce the speckle.

Readings of points the paper leaves open (listed in the design notes):
* IQ convention of this build: a scatterer of Doppler u cycles per pulse has
  Y[x] ~ exp(+2 pi i u x) (the inverse DFT of the spectra, Sec. III.B), and a
  scatterer ahead of the platform by dy has u = 2 v dy / (lambda R PRF).
* Centroid: either given (u_c cycles per pulse, 0 for the level, straight
  track of the scenes here) or estimated per burst with the pulse-pair
  estimator u_c = arg(sum_{x,g} Y[x+1, g] conj Y[x, g]) / (2 pi); the burst
  is multiplied by exp(-2 pi i u_c x), x counted from the burst's first pulse.
* Along-track FFT: unnormalised forward DFT over the M pulses of a burst,
  Z[f, g] = sum_x Y'[x, g] exp(-2 pi i f x / M), beams in FFT order, beam f
  at Doppler u_f = f_s / M relative to the removed centroid, with f_s = f for
  f < M/2 and f - M otherwise (after the centroid is removed, beam 0 looks at
  the point under the platform).
* Range migration: a scatterer seen in beam f lies dy_f = u_f PRF lambda H /
  (2 v) along track and is late by dR_f = dy_f^2 / (2 H) (flat Earth, range
  from the platform at the burst centre), delta_f = dR_f / dr gates.  The
  delay phase coefficients exp(+2 pi i q delta_f / G) (q the range frequency,
  FFT order) applied between a forward and an inverse DFT over the G gates
  move the beam's echo delta_f gates earlier.
* Output: the power |Z|^2 of every beam of every burst, [n_bursts][M][G], and
  its multi-look average over bursts and beams, [G].  Trailing pulses that do
  not fill a burst are not used.

Parity: pinned by a single point scatterer (its tone falls in one beam with
power M^2 |a|^2; a known centroid is removed exactly), a delay applied to a
band-limited echo moved back by the coefficients, Parseval of the azimuth DFT
and the multi-look of a stationary speckle-free signal.
"""
from __future__ import annotations

import numpy as np

SPEED_OF_LIGHT = 299792458.0


def centroid_cycles(burst):
    """Pulse-pair centroid of one burst [M][G]: arg(sum Y[x+1] conj Y[x]) / 2 pi."""
    b = np.asarray(burst, dtype=complex)
    s = np.sum(b[1:] * np.conj(b[:-1]))
    return float(np.angle(s) / (2.0 * np.pi)) if s != 0 else 0.0


def beam_cycles(M):
    """Doppler of every beam of an M-point along-track DFT (FFT order), in
    cycles per pulse."""
    f = np.arange(M)
    return np.where(f < M // 2, f, f - M) / M


def migration_gates(u, radar):
    """Range migration in gates of a scatterer at Doppler u cycles/pulse."""
    lam = SPEED_OF_LIGHT / radar.carrier_hz
    dy = u * radar.prf_hz * lam * radar.altitude / (2.0 * radar.velocity)
    return dy * dy / (2.0 * radar.altitude) / radar.gate_spacing


def process_burst(burst, radar, centroid=None, migration=True):
    """One burst [M][G] -> beam powers [M][G] (steps 1-3 and |.|^2)."""
    b = np.asarray(burst, dtype=complex)
    M, G = b.shape
    uc = centroid_cycles(b) if centroid is None else float(centroid)
    x = np.arange(M)
    b = b * np.exp(-2j * np.pi * uc * x)[:, None]
    # step 2: along-track DFT, written out as the sum over pulses
    f = np.arange(M)
    E = np.exp(-2j * np.pi * np.outer(f, x) / M)
    Z = E @ b
    if migration:
        # step 3: delay phase coefficients over the gates
        q = np.arange(G)
        qs = np.where(q < G // 2, q, q - G)
        for fi in range(M):
            d = migration_gates(beam_cycles(M)[fi], radar)
            Zq = np.fft.fft(Z[fi])
            Z[fi] = np.fft.ifft(Zq * np.exp(2j * np.pi * qs * d / G))
    return np.abs(Z) ** 2


def delay_doppler(Y, radar, burst=64, centroid=None, migration=True):
    """Beam powers of every burst [n_bursts][burst][G] and the multi-looked
    waveform [G] (mean over bursts and beams)."""
    Y = np.asarray(Y, dtype=complex)
    nb = Y.shape[0] // burst
    P = np.stack([process_burst(Y[i * burst:(i + 1) * burst], radar, centroid, migration)
                  for i in range(nb)])
    return P, P.mean(axis=(0, 1))
