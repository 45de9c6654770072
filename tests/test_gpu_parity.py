"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (relative L2 over all complex entries unless stated):
* same inputs, FP64 context: indices bit-exact, values <= 1e-12;
* same inputs, FP32 context with FP64 range/phase: indices bit-exact, values
  <= 1e-5 (float amplitudes, float sums of ~1e3 terms, float transforms);
* end to end from the spectrum, FP64: values <= 1e-9, index mismatches only
  for facets within 1e-6 of a gate/bin edge (or of the fold and facing
  thresholds);
* end to end, FP32: values <= 5e-3 (float surface heights move the carrier
  phase by ~1e-4 rad and flip facets that sit on gate/bin edges), mismatching
  indices only for facets within 1e-4 of an edge, their count bounded by the
  measured coordinate error.
"""
import numpy as np
import pytest

import oracle.fastmode as ofm
import oracle.iq as oiq
import oracle.scatter as osc
import oracle.surface as osurf
from paper_2408_11472_amd import inputs, workloads
from tests.gpu_helpers import (continuous_coordinates, expected_flips, explain_mismatches,
                               print_case, print_precision, rel_l2, rounded_facets,
                               to_torch_facets)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _sim():
    from paper_2408_11472_amd import simradar
    return simradar


PRECS = [("fp64", 0, np.float64), ("fp32", 1, np.float32)]


def _spec(wl):
    g = wl.grid
    return inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed, wl.sea.swell)


# ---------------------------------------------------------------- post-processing

@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
@pytest.mark.parametrize("G,N,n_fast,n_spec,window", [
    (5, 8, 8, 3, 0), (64, 64, 64, 9, 1), (128, 256, 256, 4, 0), (3, 16, 24, 4, 0),
    (7, 64, 16, 5, 1), (1, 2, 1, 6, 0), (130, 512, 128, 3, 0), (4, 2048, 512, 3, 1),
    (2, 2048, 2048, 2, 0)])
def test_segments_to_iq_matches_oracle(prec, pcode, npdt, G, N, n_fast, n_spec, window):
    simradar = _sim()
    print_case("segments_to_iq", prec, G, N, n_fast, n_spec, window)
    wl = workloads.tiny(n_gates=G, n_doppler=N, n_fast=n_fast, window=window)
    sim = simradar.Simulator(wl.grid, wl.radar, pcode)
    T = inputs.random_spectra(n_spec, G, N, seed=G * 1000 + N)
    T = T.astype(np.complex64 if npdt == np.float32 else np.complex128)
    Tt = torch.as_tensor(T, device="cuda")
    Y = sim.segments_to_iq(Tt).cpu().numpy()
    ref = oiq.segments_to_iq(T.astype(np.complex128), n_fast, window)
    err = rel_l2(Y, ref)
    tol = 1e-12 if prec == "fp64" else 2e-6
    assert err <= tol, err


# ---------------------------------------------------------------- scatterers

def _surface_facets(wl, j):
    spec = _spec(wl)
    t = wl.update_time(j)
    return osurf.facets(spec, wl.grid, t, 1.0 / wl.radar.prf_hz), t


@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
def test_accumulate_same_facets_small(prec, pcode, npdt):
    simradar = _sim()
    print_case("accumulate small_256", prec)
    wl = workloads.small_256()
    fac, t = _surface_facets(wl, 3)
    fac_r = rounded_facets(fac, npdt)
    T_ref, code_ref, cnt_ref = osc.accumulate(fac_r, wl.grid, wl.radar, t)
    sim = simradar.Simulator(wl.grid, wl.radar, pcode)
    Tt = sim.empty_spectra(wl.n_spec)
    cnt = sim.counters()
    code = torch.empty((wl.grid.ny, wl.grid.nx), dtype=torch.int32, device="cuda")
    sim.range_doppler_accumulate(to_torch_facets(fac_r, sim.real_dtype, "cuda"), t, 3, Tt,
                                 counters=cnt, facet_code=code)
    torch.cuda.synchronize()
    code = code.cpu().numpy()
    assert np.array_equal(code, code_ref), int(np.count_nonzero(code != code_ref))
    T = Tt.cpu().numpy()
    err = rel_l2(T[3], T_ref)
    assert err <= (1e-12 if prec == "fp64" else 1e-5), err
    for j in (0, 1, 2, 4, 8):
        assert np.all(T[j] == 0)
    c = cnt.cpu().numpy()
    assert [int(x) for x in c[:5]] == [cnt_ref[n] for n in osc.COUNTER_NAMES]
    assert c[5] == 0


@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
def test_accumulate_wide_doppler_windows_and_drop_rules(prec, pcode, npdt):
    # random facet motion spreads every chunk over all Doppler bins: the band
    # windows re-centre, split and overflow their slots; NaN, folded,
    # out-of-window and back-facing facets are all present.
    simradar = _sim()
    print_case("accumulate wide", prec)
    nx, ny = 64, 128
    grid = workloads.Grid(nx=nx, ny=ny, dx=1.0, dy=1.0, x_origin=-32.0, y_origin=-64.0)
    radar = workloads.Radar(n_gates=128, n_doppler=256, n_fast=256)
    radar.sat_x, radar.sat_y0 = 0.0, 0.0
    radar.gate_spacing = 0.05
    radar.window_start = radar.altitude - 64.5 * radar.gate_spacing
    fac = inputs.random_facets(nx, ny, seed=5, height_rms=1.0, dz_rms=0.01, disp_rms=0.3)
    fac["h"][0, :5] = np.nan
    fac["jac"][1, :7] = -0.5
    fac["sx"][2, :3] = 1e7          # facets at x < 0: normal turned away from the radar
    fac_r = rounded_facets(fac, npdt)
    t = 0.0123
    T_ref, code_ref, cnt_ref = osc.accumulate(fac_r, grid, radar, t)
    assert cnt_ref["out_of_window"] > 0 and cnt_ref["backfacing"] >= 3
    sim = simradar.Simulator(grid, radar, pcode)
    Tt = sim.empty_spectra(2)
    cnt = sim.counters()
    code = torch.empty((ny, nx), dtype=torch.int32, device="cuda")
    sim.range_doppler_accumulate(to_torch_facets(fac_r, sim.real_dtype, "cuda"), t, 1, Tt,
                                 counters=cnt, facet_code=code)
    torch.cuda.synchronize()
    assert np.array_equal(code.cpu().numpy(), code_ref)
    err = rel_l2(Tt.cpu().numpy()[1], T_ref)
    assert err <= (1e-12 if prec == "fp64" else 1e-5), err
    c = cnt.cpu().numpy()
    assert [int(x) for x in c[:5]] == [cnt_ref[n] for n in osc.COUNTER_NAMES]


@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
@pytest.mark.parametrize("which", ["bins", "gates"])
def test_accumulate_at_the_largest_sizes(prec, pcode, npdt, which):
    """The largest Doppler-bin count (2048, facets over most of them) and the
    largest gate count a band window holds (one bin of all gates in 32 KiB:
    4096 gates in float, 2048 in double, so the windows are one bin wide).
    Twice those gates are refused before any launch."""
    simradar = _sim()
    gmax = 4096 if prec == "fp32" else 2048
    G, N = (128, 2048) if which == "bins" else (gmax, 16)
    print_case("accumulate largest", prec, which, G, N)
    nx, ny = 64, 64
    grid = workloads.Grid(nx=nx, ny=ny, dx=1.0, dy=1.0, x_origin=-32.0, y_origin=-32.0)

    def radar_of(n_gates, spacing):
        r = workloads.Radar(n_gates=n_gates, n_doppler=N, n_fast=N)
        r.sat_x, r.sat_y0 = 0.0, 0.0
        r.gate_spacing = spacing
        r.window_start = r.altitude - (n_gates / 2 + 0.5) * spacing
        return r

    radar = radar_of(G, 0.05 if which == "bins" else 0.002)
    fac = inputs.random_facets(nx, ny, seed=11, height_rms=1.0, dz_rms=0.01, disp_rms=0.3)
    fac_r = rounded_facets(fac, npdt)
    t = 0.0071
    T_ref, code_ref, cnt_ref = osc.accumulate(fac_r, grid, radar, t)
    kept = code_ref[code_ref >= 0]
    lg = N.bit_length() - 1
    if which == "bins":
        assert len(np.unique(kept & (N - 1))) > N // 2
    else:
        assert len(np.unique(kept >> lg)) > 256
    sim = simradar.Simulator(grid, radar, pcode)
    Tt = sim.empty_spectra(2)
    cnt = sim.counters()
    code = torch.empty((ny, nx), dtype=torch.int32, device="cuda")
    ft = to_torch_facets(fac_r, sim.real_dtype, "cuda")
    sim.range_doppler_accumulate(ft, t, 1, Tt, counters=cnt, facet_code=code)
    torch.cuda.synchronize()
    assert np.array_equal(code.cpu().numpy(), code_ref)
    err = rel_l2(Tt.cpu().numpy()[1], T_ref)
    assert err <= (1e-12 if prec == "fp64" else 1e-5), err
    assert [int(x) for x in cnt.cpu().numpy()[:5]] == [cnt_ref[n] for n in osc.COUNTER_NAMES]
    if which == "gates":
        # twice the gates: no workspace size, and an accumulate call on this
        # context with such a radar returns before any launch
        with pytest.raises(simradar.SimError) as e:
            simradar.Simulator(grid, radar_of(2 * gmax, 0.002), pcode)
        assert e.value.status == simradar.SIM_ERR_UNSUPPORTED
        rr = simradar.sim_radar.from_buffer_copy(sim.radar)
        rr.n_gates = 2 * gmax
        T2 = torch.zeros((2, 2 * gmax, N), dtype=sim.complex_dtype, device="cuda")
        with pytest.raises(simradar.SimError) as e:
            simradar.sim_range_doppler_accumulate(sim.ctx, sim.grid, sim._facets_struct(ft), rr,
                                                  t, 1, T2.data_ptr(), 2, None, None,
                                                  sim._stream(None))
        assert e.value.status == simradar.SIM_ERR_UNSUPPORTED
        torch.cuda.synchronize()
        assert not T2.cpu().numpy().any()
    sim.close()


@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
@pytest.mark.parametrize("G", [1, 37, 130])
def test_accumulate_gate_counts_not_powers_of_two(prec, pcode, npdt, G):
    """Gate counts that are not powers of two (one gate, 37, 130): band
    windows of G rows and one reduce block per gate, against the oracle."""
    simradar = _sim()
    print_case("accumulate gates", prec, G)
    nx, ny, N = 64, 64, 64
    grid = workloads.Grid(nx=nx, ny=ny, dx=1.0, dy=1.0, x_origin=-32.0, y_origin=-32.0)
    radar = workloads.Radar(n_gates=G, n_doppler=N, n_fast=N)
    radar.sat_x, radar.sat_y0 = 0.0, 0.0
    radar.gate_spacing = 0.02
    radar.window_start = radar.altitude - (G / 2 + 0.5) * radar.gate_spacing
    fac = inputs.random_facets(nx, ny, seed=G, height_rms=0.5, dz_rms=0.002, disp_rms=0.2)
    fac_r = rounded_facets(fac, npdt)
    t = 0.0031
    T_ref, code_ref, cnt_ref = osc.accumulate(fac_r, grid, radar, t)
    assert cnt_ref["illuminated"] > 0 and cnt_ref["out_of_window"] > 0
    sim = simradar.Simulator(grid, radar, pcode)
    Tt = sim.empty_spectra(2)
    cnt = sim.counters()
    code = torch.empty((ny, nx), dtype=torch.int32, device="cuda")
    sim.range_doppler_accumulate(to_torch_facets(fac_r, sim.real_dtype, "cuda"), t, 1, Tt,
                                 counters=cnt, facet_code=code)
    torch.cuda.synchronize()
    assert np.array_equal(code.cpu().numpy(), code_ref)
    err = rel_l2(Tt.cpu().numpy()[1], T_ref)
    assert err <= (1e-12 if prec == "fp64" else 1e-5), err
    assert not Tt.cpu().numpy()[0].any()
    assert [int(x) for x in cnt.cpu().numpy()[:5]] == [cnt_ref[n] for n in osc.COUNTER_NAMES]
    sim.close()


@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
@pytest.mark.parametrize("reason", ["window", "nonfinite", "folded"])
def test_every_facet_dropped(prec, pcode, npdt, reason):
    """Degenerate updates where no facet reaches a spectrum (all out of the
    range window, all non-finite, all folded): the band windows stay empty,
    the ordered reduce finds no slot, T_fast stays exactly zero and every
    facet is counted once, as the oracle counts it; out of the window also
    end to end from the spectrum on both row paths."""
    simradar = _sim()
    print_case("every facet dropped", prec, reason)
    wl = workloads.tiny(nx=64, ny=32, spacing=1.5, n_gates=16, n_doppler=16, n_fast=16)
    g, r = wl.grid, wl.radar
    if reason == "window":
        r.window_start = r.altitude + 1000.0          # every range is before the window
    fac = inputs.random_facets(g.nx, g.ny, seed=3, height_rms=0.5, dz_rms=0.001,
                               disp_rms=0.1)
    if reason == "nonfinite":
        fac["h"][:] = np.nan
    elif reason == "folded":
        fac["jac"][:] = -0.25
    fac_r = rounded_facets(fac, npdt)
    t = 0.004
    T_ref, code_ref, cnt_ref = osc.accumulate(fac_r, g, r, t)
    assert not np.any(T_ref) and cnt_ref["illuminated"] == 0
    sim = simradar.Simulator(g, r, pcode)
    T = sim.empty_spectra(2)
    cnt = sim.counters()
    code = torch.empty((g.ny, g.nx), dtype=torch.int32, device="cuda")
    sim.range_doppler_accumulate(to_torch_facets(fac_r, sim.real_dtype, "cuda"), t, 1, T,
                                 counters=cnt, facet_code=code)
    torch.cuda.synchronize()
    assert not T.cpu().numpy().any()
    assert np.array_equal(code.cpu().numpy(), code_ref)
    assert [int(x) for x in cnt.cpu().numpy()[:5]] == [cnt_ref[n] for n in osc.COUNTER_NAMES]
    if reason == "window":
        spec = torch.as_tensor(_spec(wl).astype(np.complex128 if prec == "fp64"
                                                else np.complex64), device="cuda")
        for path in (simradar.SIM_ROW_PATH_SPLIT, simradar.SIM_ROW_PATH_FUSED):
            sim.set_row_path(path)
            T2, c2 = sim.empty_spectra(2), sim.counters()
            sim.update_and_accumulate(spec, t, 0, T2, counters=c2)
            torch.cuda.synchronize()
            assert not T2.cpu().numpy().any(), path
            c2 = c2.cpu().numpy()
            assert int(c2[0]) == 0 and int(c2[:5].sum()) == g.nx * g.ny, (path, c2)
    sim.close()


@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
def test_accumulate_adds_and_repeats(prec, pcode, npdt):
    # accumulate semantics: a second call adds the same spectrum again
    simradar = _sim()
    print_case("accumulate twice", prec)
    wl = workloads.tiny(nx=32, ny=16, n_gates=16, n_doppler=8)
    fac, t = _surface_facets(wl, 1)
    fac_r = rounded_facets(fac, npdt)
    T_ref = osc.accumulate(fac_r, wl.grid, wl.radar, t)[0]
    sim = simradar.Simulator(wl.grid, wl.radar, pcode)
    Tt = sim.empty_spectra(3)
    ft = to_torch_facets(fac_r, sim.real_dtype, "cuda")
    sim.range_doppler_accumulate(ft, t, 1, Tt)
    sim.range_doppler_accumulate(ft, t, 1, Tt)
    err = rel_l2(Tt.cpu().numpy()[1], 2 * T_ref)
    assert err <= (1e-12 if prec == "fp64" else 1e-5), err


# ---------------------------------------------------------------- surface

@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
@pytest.mark.parametrize("nx,ny,cwm", [(16, 16, 1), (64, 32, 1), (32, 128, 0), (256, 256, 1),
                                       (1024, 64, 1), (4096, 64, 0), (8192, 32, 1),
                                       (32, 16384, 1)])
def test_surface_update_matches_oracle(prec, pcode, npdt, nx, ny, cwm):
    if prec == "fp64" and ny > 8192:
        pytest.skip("ny > 8192 is float-only (LDS of one column)")
    simradar = _sim()
    print_case("surface", prec, nx, ny, cwm)
    wl = workloads.tiny(nx=nx, ny=ny, spacing=1.5, cwm=cwm, seed=nx + ny)
    # a sea of moderate steepness (SWH / peak wavelength <= 1/60): at the
    # default 2 m on the 12 m peak of the narrow grids the CWM surface is
    # near folding everywhere and the slopes are ill-conditioned in any
    # float evaluation
    wl.sea.swh = min(wl.sea.swh, wl.sea.peak_wavelength / 60.0)
    spec = _spec(wl)
    t, dt = 0.731, 1.0 / 18000.0
    ref = osurf.facets(spec, wl.grid, t, dt)
    sim = simradar.Simulator(wl.grid, wl.radar, pcode)
    spec_t = torch.as_tensor(spec.astype(np.complex64 if npdt == np.float32 else np.complex128),
                             device="cuda")
    out = sim.surface_update(spec_t, t, dt)
    torch.cuda.synchronize()
    tol = 1e-11 if prec == "fp64" else 2e-5
    for k in osurf.FACET_FIELDS:
        got = out[k].cpu().numpy().astype(np.float64)
        scale = np.sqrt(np.mean(ref[k] ** 2)) if k != "jac" else 1.0
        if scale == 0:
            # CWM off: the displacements are zero in the oracle and rounding
            # residue of the packed transform on the GPU (relative to h)
            scale = np.sqrt(np.mean(ref["h"] ** 2)) if k in ("disp_x", "disp_y") else \
                np.sqrt(np.mean(ref["dh"] ** 2))
        err = np.sqrt(np.mean((got - ref[k]) ** 2)) / scale
        assert err <= tol, (k, err)


@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
def test_surface_update_long_pair_interval(prec, pcode, npdt):
    """A pair interval long enough that w dt leaves the small-angle range of
    the increment multiplier (the other branch of the same formula)."""
    simradar = _sim()
    print_case("surface long dt", prec)
    wl = workloads.tiny(nx=64, ny=64, spacing=1.0, seed=5)
    wl.sea.swh = min(wl.sea.swh, wl.sea.peak_wavelength / 60.0)
    spec = _spec(wl)
    t, dt = 3.25, 0.2
    ref = osurf.facets(spec, wl.grid, t, dt)
    sim = simradar.Simulator(wl.grid, wl.radar, pcode)
    spec_t = torch.as_tensor(spec.astype(np.complex64 if npdt == np.float32 else np.complex128),
                             device="cuda")
    out = sim.surface_update(spec_t, t, dt)
    torch.cuda.synchronize()
    tol = 1e-11 if prec == "fp64" else 2e-5
    for k in ("ddisp_x", "ddisp_y", "dh"):
        got = out[k].cpu().numpy().astype(np.float64)
        err = np.sqrt(np.mean((got - ref[k]) ** 2)) / np.sqrt(np.mean(ref[k] ** 2))
        assert err <= tol, (k, err)


@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
@pytest.mark.parametrize("t", [3600.37, 86400.77])
def test_surface_update_late_in_a_long_track(prec, pcode, npdt, t):
    """An hour and a day into a track: the evolution phase w t reaches ~1e4 and
    ~6e5 rad, which only a reduction in double keeps exact enough for the
    float context's 2e-5 on the fields.  In double both sides round w t
    independently, so the bound grows by a few ulp of the largest w t.  The
    oracle forms the pair displacement as the difference of two evaluations
    (its definition), whose rounding of w t is relative to the fields, not to
    their small difference: the difference fields are held to that bound
    scaled by |P| / |dP| (the GPU applies the per-mode increment instead)."""
    simradar = _sim()
    print_case("surface late", prec, t)
    wl = workloads.tiny(nx=64, ny=64, spacing=1.0, seed=9)
    wl.sea.swh = min(wl.sea.swh, wl.sea.peak_wavelength / 60.0)
    spec = _spec(wl)
    dt = 1.0 / 18000.0
    ref = osurf.facets(spec, wl.grid, t, dt)
    sim = simradar.Simulator(wl.grid, wl.radar, pcode)
    spec_t = torch.as_tensor(spec.astype(np.complex64 if npdt == np.float32 else np.complex128),
                             device="cuda")
    out = sim.surface_update(spec_t, t, dt)
    torch.cuda.synchronize()
    w_max = np.sqrt(wl.grid.gravity * np.pi * np.sqrt(2.0) / wl.grid.dx)
    tol = (1e-11 + 8 * np.finfo(np.float64).eps * w_max * t) if prec == "fp64" else 2e-5
    phase = 8 * np.finfo(np.float64).eps * w_max * t
    base = {"ddisp_x": "disp_x", "ddisp_y": "disp_y", "dh": "h"}
    for k in osurf.FACET_FIELDS:
        got = out[k].cpu().numpy().astype(np.float64)
        scale = np.sqrt(np.mean(ref[k] ** 2)) if k != "jac" else 1.0
        err = np.sqrt(np.mean((got - ref[k]) ** 2)) / scale
        tk = tol + (phase * np.sqrt(np.mean(ref[base[k]] ** 2)) / scale if k in base else 0.0)
        assert err <= tk, (k, err, tk)
    sim.close()


# ---------------------------------------------------------------- end to end

def _mismatch_check(code, code_ref, fac_ref, fac_gpu, wl, t, fp64):
    """Every index mismatch sits on a threshold of the oracle's decision
    (gate or bin edge within 1e-4 in float / 1e-6 in double, |J| < 1e-4 /
    1e-9, |q|/R < 1e-6 / 1e-12), and the count stays within a bound computed
    from the measured coordinate error of the GPU facets."""
    coords = continuous_coordinates(fac_ref, wl.grid, wl.radar, t)
    n_bad = explain_mismatches(code, code_ref, coords, 1e-6 if fp64 else 1e-4,
                               1e-9 if fp64 else 1e-4, 1e-12 if fp64 else 1e-6)
    coords_gpu = continuous_coordinates(fac_gpu, wl.grid, wl.radar, t)
    n_exp = expected_flips(coords_gpu, coords, code_ref >= 0)
    print(f"index mismatches {n_bad}, expected {n_exp:.2f}", flush=True)
    assert n_bad <= 2 + 3.0 * n_exp, (n_bad, n_exp)
    return n_bad


@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
@pytest.mark.parametrize("which", ["tiny", "small_256", "wide_8192"])
def test_update_and_accumulate_end_to_end(prec, pcode, npdt, which):
    simradar = _sim()
    print_case("fused", prec, which)
    if which == "small_256":
        wl = workloads.small_256()
    elif which == "wide_8192":
        wl = workloads.tiny(nx=8192, ny=64, spacing=1.0, n_gates=64, n_doppler=64, n_fast=64,
                            n_updates=3)
    else:
        wl = workloads.tiny(nx=64, ny=64, spacing=2.0, n_gates=32, n_doppler=16, n_fast=16,
                            n_updates=3)
    spec = _spec(wl)
    sim = simradar.Simulator(wl.grid, wl.radar, pcode)
    spec_t = torch.as_tensor(spec.astype(np.complex64 if npdt == np.float32 else np.complex128),
                             device="cuda")
    j = 2
    t = wl.update_time(j)
    Tt = sim.empty_spectra(wl.n_spec)
    code = torch.empty((wl.grid.ny, wl.grid.nx), dtype=torch.int32, device="cuda")
    cnt = sim.counters()
    sim.update_and_accumulate(spec_t, t, j, Tt, counters=cnt, facet_code=code)
    torch.cuda.synchronize()
    fac = osurf.facets(spec, wl.grid, t, 1.0 / wl.radar.prf_hz)
    T_ref, code_ref, cnt_ref = osc.accumulate(fac, wl.grid, wl.radar, t)
    code = code.cpu().numpy()
    # the facets of the same kernels (the fused call's split row path writes
    # exactly these) give the measured coordinate error
    fg = sim.surface_update(spec_t, t, 1.0 / wl.radar.prf_hz)
    fac_gpu = {k: v.cpu().numpy().astype(np.float64) for k, v in fg.items()}
    _mismatch_check(code, code_ref, fac, fac_gpu, wl, t, prec == "fp64")
    err = rel_l2(Tt.cpu().numpy()[j], T_ref)
    assert err <= (1e-9 if prec == "fp64" else 5e-3), err
    assert int(cnt.cpu().numpy()[:5].sum()) == wl.n_facets


@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
def test_full_run_small_256(prec, pcode, npdt):
    simradar = _sim()
    print_case("run small_256", prec)
    wl = workloads.small_256()
    spec = _spec(wl)
    sim = simradar.Simulator(wl.grid, wl.radar, pcode)
    spec_t = torch.as_tensor(spec.astype(np.complex64 if npdt == np.float32 else np.complex128),
                             device="cuda")
    T, Y = sim.run(spec_t, wl.n_updates)
    torch.cuda.synchronize()
    T_ref, Y_ref = ofm.simulate(spec, wl.grid, wl.radar, wl.n_updates)
    eT, eY = rel_l2(T.cpu().numpy(), T_ref), rel_l2(Y.cpu().numpy(), Y_ref)
    # the multi-look waveform of the run (the GPU kernel) against the oracle's
    import oracle.adjoint as oad
    P, _ = sim.waveform_loss(Y)
    torch.cuda.synchronize()
    eP = rel_l2(P.cpu().numpy(), oad.waveform(Y_ref))
    for name, v in (("T_fast", eT), ("Y", eY), ("P", eP)):
        print_precision("small_256", f"{prec} end to end", name, v)
    assert eT <= (1e-9 if prec == "fp64" else 5e-3)
    assert eY <= (1e-9 if prec == "fp64" else 5e-3)
    assert eP <= (1e-9 if prec == "fp64" else 1e-3)
    # the three-call path gives the same spectra as the fused call
    T3 = sim.empty_spectra(wl.n_spec)
    for j in range(wl.n_spec):
        t = wl.update_time(j)
        fac = sim.surface_update(spec_t, t, 1.0 / wl.radar.prf_hz)
        sim.range_doppler_accumulate(fac, t, j, T3)
    torch.cuda.synchronize()
    assert rel_l2(T3.cpu().numpy(), T.cpu().numpy()) <= (1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("prec,pcode,npdt", PRECS)
@pytest.mark.parametrize("nx,ny", [(16, 16), (64, 32), (256, 256), (4096, 64), (8192, 32),
                                   (32, 16384), (1024, 64)])
def test_prepared_spectrum_gives_the_same_update(prec, pcode, npdt, nx, ny):
    """The column pass reading the prepared spectrum computes exactly what it
    computes from the FFT-order spectrum."""
    if prec == "fp64" and ny > 8192:
        pytest.skip("ny > 8192 is float-only (LDS of one column)")
    simradar = _sim()
    print_case("prepared", prec, nx, ny)
    wl = workloads.tiny(nx=nx, ny=ny, spacing=1.0, n_gates=32, n_doppler=16, n_fast=16,
                        n_updates=3, seed=nx * 3 + ny)
    wl.sea.swh = min(wl.sea.swh, wl.sea.peak_wavelength / 60.0)
    spec = _spec(wl)
    sim = simradar.Simulator(wl.grid, wl.radar, pcode)
    spec_t = torch.as_tensor(spec.astype(np.complex64 if npdt == np.float32 else np.complex128),
                             device="cuda")
    prep = sim.prepare_spectrum(spec_t)
    out = []
    for use_prep in (False, True):
        T = sim.empty_spectra(wl.n_spec)
        code = torch.empty((ny, nx), dtype=torch.int32, device="cuda")
        if use_prep:
            sim.update_and_accumulate_prepared(prep, wl.update_time(2), 2, T, facet_code=code)
        else:
            sim.update_and_accumulate(spec_t, wl.update_time(2), 2, T, facet_code=code)
        torch.cuda.synchronize()
        out.append((T.cpu().numpy(), code.cpu().numpy()))
    np.testing.assert_array_equal(out[0][1], out[1][1])
    # identical scatterers; only the order of the window atomics differs
    # (cells of up to ~1e3 nearly coherent terms: eps * n_cell)
    assert rel_l2(out[1][0], out[0][0]) <= (1e-13 if prec == "fp64" else 1e-5)
