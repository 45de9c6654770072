"""Consistency of the paper's printed scenario figures with the readings used
by the oracle (tensor shape of Sec. III.B, tile count of Sec. IV)."""
import json
import os

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_scenario.json")


def test_scenario_figures_are_consistent():
    s = json.load(open(GOLDEN))
    # 335 tiles of 1024 x 1024 scatterers make the stated 3.51e8 scatterers
    assert abs(s["n_tiles"] * s["tile_side"] ** 2 / s["n_scatterers"] - 1) < 0.005
    # 267 379 pulses at 17.8 kHz span ~15 s; a 100 km track then implies a
    # ground speed of ~6.7 km/s, a LEO platform (sanity of the units)
    v = s["track_km"] * 1e3 / (s["n_pulses"] / s["prf_hz"])
    assert 6.0e3 < v < 7.5e3
    # T_fast holds 1 + n_pulses / n_fast spectra (integer division for a
    # final partial interval)
    shapes = {n: 1 + s["n_pulses"] // n for n in s["n_fast_tested"]}
    assert shapes[250] == 1070 and shapes[500] == 535 and shapes[1250] == 214


def test_oracle_tensor_shapes_follow_the_paper():
    """The oracle allocates the tensor of Sec. III.B: 1 + n_pulses / n_fast
    spectra, spectrum j taken at pulse j n_fast (its update time j n_fast /
    PRF), and post-processing returns one IQ row per pulse."""
    import numpy as np

    import oracle.fastmode as ofm
    from paper_2408_11472_amd import inputs, workloads
    s = json.load(open(GOLDEN))
    wl = workloads.tiny(nx=16, ny=16, n_gates=8, n_doppler=8, n_fast=5, n_updates=3)
    g, r = wl.grid, wl.radar
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)
    n_pulses = 3 * r.n_fast
    T, Y = ofm.simulate(spec, g, r, n_pulses // r.n_fast)
    assert T.shape == (1 + n_pulses // r.n_fast, r.n_gates, r.n_doppler)
    assert Y.shape == (n_pulses, r.n_gates)
    # at the scenario's PRF, updates every 250 pulses are 250 / 17.8 kHz apart
    radar = type("R", (), {"n_fast": 250, "prf_hz": s["prf_hz"]})()
    assert np.isclose(ofm.update_time(1, radar), 250 / 17.8e3, rtol=1e-15)
    assert ofm.update_time(s["n_pulses"] // 250, radar) <= s["n_pulses"] / s["prf_hz"]
