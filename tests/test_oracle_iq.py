"""Pins of the oracle's post-processing (Sec. III.B steps 1-4, eq. (1))."""
import math

import numpy as np
import pytest

import oracle.iq as oiq
from paper_2408_11472_amd import inputs


@pytest.mark.parametrize("kind", [oiq.WIN_SQRT_TRIANGLE, oiq.WIN_SQRT_RAISED_COSINE])
@pytest.mark.parametrize("n_fast", [1, 2, 7, 64, 250])
def test_weights_conserve_power_at_every_pulse(kind, n_fast):
    # the 1/2 power keeps the total variance: sum_j W(x - c_j)^2 = 1
    x = np.arange(0, 5 * n_fast)
    total = np.zeros(x.shape)
    for j in range(0, 7):
        total += oiq.window_weight(x - j * n_fast, n_fast, kind) ** 2
    np.testing.assert_allclose(total, 1.0, atol=1e-14)
    assert oiq.window_weight(0, n_fast, kind) == 1.0
    assert abs(oiq.window_weight(n_fast, n_fast, kind)) < 1e-15
    assert abs(oiq.window_weight(-n_fast, n_fast, kind)) < 1e-15
    assert oiq.window_weight(n_fast + 1, n_fast, kind) == 0.0


def test_eq1_values():
    # W_i(x) = (1 - |i - x| / n_fast)^(1/2)
    n = 500
    for d, w in [(0, 1.0), (125, math.sqrt(0.75)), (-250, math.sqrt(0.5)), (499, math.sqrt(1 / 500))]:
        assert abs(oiq.window_weight(d, n) - w) < 1e-15


def test_parseval_of_the_long_time_signals():
    T = inputs.random_spectra(3, 5, 64, seed=4)
    s = oiq.long_time_signals(T)
    np.testing.assert_allclose(np.sum(np.abs(s) ** 2, axis=-1),
                               64 * np.sum(np.abs(T) ** 2, axis=-1), rtol=1e-12)


def test_long_time_signal_is_the_direct_idft():
    T = inputs.random_spectra(2, 3, 16, seed=9)
    s = oiq.long_time_signals(T)
    k = np.arange(16)
    for m in (0, 1, 5, 15):
        direct = np.sum(T * np.exp(2j * np.pi * k * m / 16), axis=-1)
        np.testing.assert_allclose(s[..., m], direct, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("N,n_fast", [(64, 64), (128, 32), (16, 24)])
def test_centre_identity(N, n_fast):
    T = inputs.random_spectra(5, 4, N, seed=1)
    Y = oiq.segments_to_iq(T, n_fast)
    for j in range(4):
        np.testing.assert_allclose(Y[j * n_fast], T[j].sum(axis=-1), rtol=1e-12)


@pytest.mark.parametrize("N,n_fast", [(32, 32), (64, 16), (16, 24)])
def test_single_bin_closed_form(N, n_fast):
    T = np.zeros((4, 2, N), complex)
    k_star, Cv = 3, 0.7 - 0.2j
    T[1, 1, k_star] = Cv
    Y = oiq.segments_to_iq(T, n_fast)
    for x in range(Y.shape[0]):
        d = x - n_fast
        expect = 0.0
        if abs(d) < n_fast:
            expect = math.sqrt(1 - abs(d) / n_fast) * Cv * np.exp(2j * np.pi * k_star * d / N)
        assert abs(Y[x, 1] - expect) < 1e-13
        assert Y[x, 0] == 0


def test_regular_mode_limit_of_post_processing():
    # n_fast = 1: each pulse is its own spectrum, Y[x] = sum_k T[x]
    T = inputs.random_spectra(9, 3, 8, seed=2)
    Y = oiq.segments_to_iq(T, 1)
    np.testing.assert_allclose(Y, T[:-1].sum(axis=-1), rtol=1e-12)


def test_variance_of_independent_spectra_is_conserved():
    # E|Y|^2 = E|s|^2 for independent spectra (statistical form of the 1/2 power)
    N, n_fast = 32, 32
    T = inputs.random_spectra(400, 8, N, seed=12)
    Y = oiq.segments_to_iq(T, n_fast)
    ratio = np.mean(np.abs(Y) ** 2) / (N * 2.0)     # E|s|^2 = N E|T|^2 = 2N
    assert abs(ratio - 1.0) < 0.02
