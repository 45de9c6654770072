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
