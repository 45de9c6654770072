"""Host statistics of the n_fast sweep, pinned on series whose answer is
known in closed form (no GPU).

* An AR(1) series x[n] = phi x[n-1] + e[n] has rho(k) = phi^k, so its
  integrated autocorrelation time is 1/2 + phi / (1 - phi) = (1 + phi) /
  (2 (1 - phi)); white noise has 1/2.
* The standard deviation of a mean from mean_and_sigma must match the spread
  of the means of many independent series (AR(1) and speckle-like squared
  complex AR(1) series).
* The per-gate z statistic of two independent runs of the same process is
  N(0, 1): its rms is near 1 and Bonferroni bound holds.
* iq_correlation of a complex AR(1) series is |phi|^k.
* Regular mode is n_fast = 1 with 2 bins; fast modes get the smallest power
  of two covering 2 n_fast, capped at 2048.
"""
import numpy as np

from paper_2408_11472_amd import nfast


def _ar1(phi, n, m, rng, complex_=False):
    e = rng.standard_normal((m, n))
    if complex_:
        e = (e + 1j * rng.standard_normal((m, n))) / np.sqrt(2.0)
    x = np.empty_like(e)
    x[:, 0] = e[:, 0] / np.sqrt(1.0 - phi * phi)
    for k in range(1, n):
        x[:, k] = phi * x[:, k - 1] + e[:, k]
    return x


def test_integrated_autocorrelation_time_of_ar1():
    rng = np.random.default_rng(3)
    # the estimate of tau over a window of M ~ 5 tau lags has a relative
    # standard deviation of about sqrt(2 (2M + 1) / n); with n = 1e5 that is
    # 6 % at phi = 0.95: each series within 30 %, their mean within 10 %
    for phi in (0.0, 0.5, 0.8, 0.95):
        x = _ar1(phi, 100000, 8, rng)
        tau = nfast.integrated_autocorrelation_time(x)
        exact = (1.0 + phi) / (2.0 * (1.0 - phi))
        assert np.all(np.abs(tau / exact - 1.0) < 0.3), (phi, tau, exact)
        assert abs(tau.mean() / exact - 1.0) < 0.1, (phi, tau, exact)


def test_sigma_of_the_mean_matches_the_spread_of_means():
    rng = np.random.default_rng(5)
    for complex_ in (False, True):
        x = _ar1(0.9, 4000, 400, rng, complex_=complex_)
        p = np.abs(x) ** 2 if complex_ else x
        means = p.mean(axis=1)
        # mean_and_sigma takes [pulse][gate]: one series per "gate"
        _, sig, _ = nfast.mean_and_sigma(p.T)
        ratio = np.median(sig) / np.std(means)
        assert 0.85 < ratio < 1.15, ratio


def test_z_of_independent_runs_is_unit_normal():
    rng = np.random.default_rng(9)
    G, n = 200, 3000
    a = _ar1(0.8, n, G, rng, complex_=True).T
    b = _ar1(0.8, n, G, rng, complex_=True).T
    c = nfast.compare_waveforms(a, b, gate_floor=0.0)
    assert 0.8 < c["rms_z"] < 1.2, c["rms_z"]
    assert c["max_abs_z"] < nfast.sigma_of_z_bound(G, 1e-3)
    assert abs(c["power_ratio"] - 1.0) < 4.0 * c["power_ratio_sigma"]
    # a 10 % bias in one gate group is detected
    b2 = b.copy()
    b2[:, :50] *= np.sqrt(1.2)
    c2 = nfast.compare_waveforms(a, b2, gate_floor=0.0)
    assert c2["max_abs_z"] > nfast.sigma_of_z_bound(G, 1e-3)


def test_iq_correlation_of_complex_ar1():
    rng = np.random.default_rng(13)
    phi = 0.9
    x = _ar1(phi, 50000, 4, rng, complex_=True).T
    r = nfast.iq_correlation(x, 10)
    assert abs(r[0] - 1.0) < 1e-12
    assert np.all(np.abs(r - phi ** np.arange(11)) < 0.03), r


def test_mode_bins_and_pulses():
    assert nfast.doppler_bins(1) == 2
    assert nfast.doppler_bins(250) == 512
    assert nfast.doppler_bins(500) == 1024
    assert nfast.doppler_bins(750) == 2048
    assert nfast.doppler_bins(1250) == 2048
    scene = nfast.sweep_scene(nx=64, n_pulses=5000)
    assert scene.radar.n_fast == 1 and scene.n_spec == 5001
    for nf in nfast.SWEEP_NFAST:
        m = nfast.mode(scene, nf)
        assert m.n_pulses == (5000 // nf) * nf and m.n_pulses <= 5000
        # same track and range window as the regular mode
        assert m.radar.sat_y0 == scene.radar.sat_y0
        assert m.radar.window_start == scene.radar.window_start


def test_coherent_power_gain_of_the_cross_fade():
    """Eq. (1) keeps the variance of independent consecutive signals and
    raises coherent ones by the segment mean of (sqrt(1 - tau) + sqrt(tau))^2
    = 1 + pi/4 (the oracle's post-processing, a static scatterer in one
    bin), which is the bound nfast.COHERENT_POWER_GAIN states."""
    import oracle.iq as oiq
    nf, U, G, N = 400, 6, 1, 1024
    T = np.zeros((U + 1, G, N), complex)
    T[:, 0, 0] = 0.8 - 0.3j
    Y = oiq.segments_to_iq(T, nf)
    gain = np.mean(np.abs(Y) ** 2) / abs(T[0, 0, 0]) ** 2
    assert abs(gain - nfast.COHERENT_POWER_GAIN) < 2.0 / nf, gain
    # independent spectra: the gain averages to 1
    rng = np.random.default_rng(17)
    T = rng.standard_normal((U + 1, 256, 64)) + 1j * rng.standard_normal((U + 1, 256, 64))
    Y = oiq.segments_to_iq(T, 32)
    s = oiq.long_time_signals(T)
    gain = np.mean(np.abs(Y) ** 2) / np.mean(np.abs(s) ** 2)
    assert abs(gain - 1.0) < 0.02, gain
