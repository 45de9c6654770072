"""Host logic of the autotuner's choice (no GPU): the fastest candidate,
with ties between the fused and the split row path going to the split path."""
from paper_2408_11472_amd import autotune as at

F, S = at.PATH_FUSED, at.PATH_SPLIT


def test_fastest_wins_when_clearly_faster():
    assert at.pick({(F, 256): 700.0, (F, 64): 900.0, (S, 0): 800.0}) == (F, 256)
    assert at.pick({(F, 256): 820.0, (S, 0): 700.0}) == (S, 0)


def test_tie_within_margin_goes_to_split():
    # 839.9 (split) vs 840.9 (fused): split already fastest
    assert at.pick({(F, 256): 840.9, (S, 0): 839.9}) == (S, 0)
    # fused 1 % faster: within the margin, split kept
    assert at.pick({(F, 256): 825.0, (F, 512): 826.0, (S, 0): 833.0}) == (S, 0)
    # just beyond the margin: fused kept
    t = 800.0
    assert at.pick({(F, 128): t, (S, 0): t * (1 + at.FUSED_MARGIN) * 1.001}) == (F, 128)


def test_without_split_candidate():
    assert at.pick({(F, 128): 2.0, (F, 256): 1.0}) == (F, 256)


def test_lanes_fastest_unless_fewer_within_margin():
    assert at.pick_lanes({1: 458.0, 2: 283.0, 3: 224.0, 4: 226.0}) == 3
    # the tuner's times on the 4096^2 track and the 8192 x 16384 stress runs
    assert at.pick_lanes({1: 19.163, 2: 18.646, 3: 17.726, 4: 17.671}) == 3
    assert at.pick_lanes({1: 194.263, 2: 194.622, 3: 188.512, 4: 193.235}) == 1
    # 3 and 4 lanes within the margin of each other: the fewer kept
    assert at.pick_lanes({1: 100.0, 2: 80.0, 3: 70.5, 4: 70.0}) == 3
    # no lane count beats one by more than the margin
    assert at.pick_lanes({1: 100.0, 2: 99.0, 3: 97.0, 4: 99.5}) == 1


def test_sample_times_spread_over_the_run():
    t = [0.1 * j for j in range(513)]
    s = at.sample_times(t, 24)
    assert len(s) == 24 and s[0] == t[0] and s[-1] == t[-1]
    assert all(b > a for a, b in zip(s, s[1:]))
    assert at.sample_times(t[:10], 24) == t[:10]


def test_lanes_margin_of_whole_steps():
    t = {1: 2.942, 2: 2.779, 3: 2.715, 4: 2.739}
    assert at.pick_lanes(t) == 2                     # the short-run margin
    assert at.pick_lanes(t, margin=0.01) == 3


def test_cache_key_names_the_shape_and_the_library_build():
    """A cached choice applies to one shape on one build of the library."""
    import types
    g = types.SimpleNamespace(nx=4096, ny=2048)
    r = types.SimpleNamespace(n_gates=128, n_doppler=256)
    sim = types.SimpleNamespace(grid=g, radar=r, precision=1)
    key = at.shape_key(sim)
    assert key.startswith("prec1|4096x2048|G128|N256|lib")
    bid = at.library_build_id()
    assert key.endswith(bid) and len(bid) == 12 and int(bid, 16) >= 0
    sim.precision = 0
    assert at.shape_key(sim) != key


def test_accumulate_bands_kept_only_when_clearly_faster():
    # measured on the 4096^2 track, 3 lanes: 256 bands 3 % faster -> kept
    assert at.pick_acc_bands({512: 48.3, 256: 46.8}) == 256
    # within the margin, or slower (one lane): the default (0)
    assert at.pick_acc_bands({512: 48.3, 256: 47.9}) == 0
    assert at.pick_acc_bands({512: 51.7, 256: 57.2}) == 0
    assert at.pick_acc_bands({}) == 0                    # one lane: not timed
    t = 100.0
    assert at.pick_acc_bands({512: t, 256: t * (1 - at.ACC_BANDS_MARGIN) * 0.999}) == 256


def test_short_runs_are_tuned_whole_long_ones_on_a_sample():
    import types
    g = types.SimpleNamespace(nx=4096, ny=4096)
    r = types.SimpleNamespace(n_fast=256, prf_hz=17800.0)
    sim = types.SimpleNamespace(grid=g, radar=r)
    track = [j * 256 / 17800.0 for j in range(65)]
    times, whole = at.run_sample(sim, track)
    assert whole and times == track
    long_run = [j * 128 / 17800.0 for j in range(513)]
    times, whole = at.run_sample(sim, long_run)
    assert not whole and len(times) == at.lane_run_updates(sim)
    assert times[0] == long_run[0] and times[-1] == long_run[-1]
    times, whole = at.run_sample(sim, None)
    assert not whole and len(times) == at.lane_run_updates(sim)


def test_whole_run_margin_keeps_three_lanes_on_the_track():
    # whole runs of the 4096^2 track (65 updates): 3 lanes, away from the
    # 1.2 % to 4 lanes and the 4 % to 2 lanes
    whole = {1: 51.87, 2: 50.48, 3: 48.55, 4: 47.96}
    assert at.pick_lanes(whole, at.WHOLE_RUN_LANES_MARGIN) == 3
    assert at.pick_lanes({k: v * (1.003 if k == 3 else 1.0) for k, v in whole.items()},
                         at.WHOLE_RUN_LANES_MARGIN) == 3
