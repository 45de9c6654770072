"""Pins of the Delay-Doppler oracle (Sec. IV.C) on signals whose processed
form is known in closed form."""
import numpy as np
import pytest

import oracle.delay_doppler as odd
from paper_2408_11472_amd import workloads


def _radar(G=32, **kw):
    return workloads.Radar(n_gates=G, **kw)


def test_point_scatterer_falls_in_one_beam():
    # a bin-centred tone at gate g0: all energy in beam f0 with |Z|^2 = M^2 |a|^2
    M, G, g0, f0 = 64, 32, 11, 5
    a = 0.7 - 0.2j
    x = np.arange(M)
    Y = np.zeros((M, G), complex)
    Y[:, g0] = a * np.exp(2j * np.pi * f0 * x / M)
    P = odd.process_burst(Y, _radar(G), centroid=0.0, migration=False)
    assert np.isclose(P[f0, g0], M * M * abs(a) ** 2, rtol=1e-12)
    P[f0, g0] = 0.0
    assert np.max(P) < 1e-20
    # negative Doppler lands at beam M + f (FFT order)
    Y[:, g0] = a * np.exp(-2j * np.pi * 3 * x / M)
    P = odd.process_burst(Y, _radar(G), centroid=0.0, migration=False)
    assert np.argmax(P[:, g0]) == M - 3


def test_centroid_estimate_removes_a_known_tone():
    M, G = 32, 16
    u0 = 0.0731
    x = np.arange(M)
    rng = np.random.default_rng(1)
    amp = rng.standard_normal(G) + 1j * rng.standard_normal(G)
    Y = np.exp(2j * np.pi * u0 * x)[:, None] * amp[None, :]
    assert abs(odd.centroid_cycles(Y) - u0) < 1e-14
    P = odd.process_burst(Y, _radar(G), centroid=None, migration=False)
    # after the centroid is removed every gate's tone is at zero Doppler
    assert np.allclose(P[0], M * M * np.abs(amp) ** 2, rtol=1e-12)
    assert np.max(P[1:]) < 1e-18 * np.max(P[0])


def test_migration_constant_closed_form():
    r = _radar(G=64)
    lam = 299792458.0 / r.carrier_hz
    # a scatterer 300 m ahead: Doppler 2 v dy / (lambda H), late by dy^2 / (2 H)
    dy = 300.0
    u = 2.0 * r.velocity * dy / (lam * r.altitude) / r.prf_hz
    assert np.isclose(odd.migration_gates(u, r), dy * dy / (2.0 * r.altitude) / r.gate_spacing,
                      rtol=1e-12)
    assert odd.migration_gates(0.0, r) == 0.0


def test_delay_coefficients_move_a_band_limited_echo_back():
    # beam f carries an echo centred delta_f gates late; with migration on its
    # range profile becomes the same echo at g0
    M, G, g0 = 64, 64, 20
    r = _radar(G=G)    # beam 3 of 64 at 18 kHz lies ~1.1 km ahead: ~1.7 gates late
    q = np.arange(G)
    qs = np.where(q < G // 2, q, q - G)
    band = np.abs(qs) < G // 4

    def echo(pos):
        return np.fft.ifft(np.where(band, np.exp(-2j * np.pi * qs * pos / G), 0.0))
    x = np.arange(M)
    f = 3
    d = odd.migration_gates(f / M, r)
    assert 0.5 < d < G / 4
    Y = np.exp(2j * np.pi * f * x / M)[:, None] * echo(g0 + d)[None, :]
    P = odd.process_burst(Y, r, centroid=0.0, migration=True)
    want = M * M * np.abs(echo(g0)) ** 2
    assert np.allclose(P[f], want, rtol=0, atol=1e-12 * want.max())
    assert np.argmax(P[f]) == g0
    # without the correction the peak sits delta_f late
    P0 = odd.process_burst(Y, r, centroid=0.0, migration=False)
    assert np.argmax(P0[f]) == g0 + int(round(d))


@pytest.mark.parametrize("migration", [False, True])
def test_parseval_and_multilook(migration):
    rng = np.random.default_rng(4)
    M, G, nb = 16, 32, 5
    Y = rng.standard_normal((nb * M + 7, G)) + 1j * rng.standard_normal((nb * M + 7, G))
    r = _radar(G=G)
    P, w = odd.delay_doppler(Y, r, burst=M, centroid=0.0, migration=migration)
    assert P.shape == (nb, M, G) and w.shape == (G,)
    for b in range(nb):
        # energy: M times the burst's energy (the range step is unitary)
        e_in = np.sum(np.abs(Y[b * M:(b + 1) * M]) ** 2)
        assert np.isclose(P[b].sum(), M * e_in, rtol=1e-12)
    assert np.allclose(w, P.mean(axis=(0, 1)), rtol=1e-14)
    # per gate without migration: Parseval along the pulses
    if not migration:
        e_g = np.sum(np.abs(Y[:M]) ** 2, axis=0)
        assert np.allclose(P[0].sum(axis=0), M * e_g, rtol=1e-12)
