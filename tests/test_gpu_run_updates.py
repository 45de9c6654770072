"""sim_run_updates: the updates of a run enqueued by the library in one call
(Algorithm 1's loop over spectra), against the same updates called one by
one on the same context (identical launches: counters equal, T_fast equal up
to the summation order of the window atomics), a partial range, and the
argument checks that return before any launch."""
import ctypes

import numpy as np
import pytest

from paper_2408_11472_amd import inputs, workloads
from tests.gpu_helpers import print_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("nx,ny,cwm", [(64, 64, 1), (128, 32, 0)])
def test_run_updates_equals_per_update_calls(prec, nx, ny, cwm):
    from paper_2408_11472_amd import simradar
    print_case("run_updates", prec, nx, ny, cwm)
    fp64 = prec == "fp64"
    wl = workloads.tiny(nx=nx, ny=ny, spacing=2.0, n_gates=32, n_doppler=16, n_fast=16,
                        n_updates=6, cwm=cwm)
    g, r = wl.grid, wl.radar
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)
    sim = simradar.Simulator(g, r, simradar.SIM_PREC_FP64 if fp64 else
                             simradar.SIM_PREC_FP32_PHASE64)
    spec_t = torch.as_tensor(spec.astype(np.complex128 if fp64 else np.complex64), device="cuda")
    prep = sim.prepare_spectrum(spec_t)
    times = [(j * r.n_fast) / r.prf_hz for j in range(wl.n_spec)]

    T1, c1 = sim.empty_spectra(wl.n_spec), sim.counters()
    for j, t in enumerate(times):
        sim.update_and_accumulate_prepared(prep, t, j, T1, counters=c1)
    T2, c2 = sim.empty_spectra(wl.n_spec), sim.counters()
    sim.run_updates(prep, times, 0, T2, counters=c2)
    # a partial range: spectra 2 .. 4 only
    T3 = sim.empty_spectra(wl.n_spec)
    sim.run_updates(prep, times[2:5], 2, T3)
    torch.cuda.synchronize()
    a, b, p = T1.cpu().numpy(), T2.cpu().numpy(), T3.cpu().numpy()
    assert np.array_equal(c1.cpu().numpy(), c2.cpu().numpy())
    assert int(c2.cpu().numpy()[0]) > 0
    tol = 1e-13 if fp64 else 1e-6
    assert rel_l2(b, a) <= tol, rel_l2(b, a)
    assert rel_l2(p[2:5], a[2:5]) <= tol
    assert not p[:2].any() and not p[5:].any()
    sim.close()


def test_run_updates_rejects_bad_arguments_before_launch():
    from paper_2408_11472_amd import simradar as s
    print_case("run_updates errors")
    wl = workloads.tiny(nx=32, ny=32, n_gates=8, n_doppler=16, n_fast=16, n_updates=2)
    sim = s.Simulator(wl.grid, wl.radar, s.SIM_PREC_FP32_PHASE64)
    prep = sim.prepare_spectrum(torch.zeros((32, 32), dtype=torch.complex64, device="cuda"))
    T = sim.empty_spectra(wl.n_spec)
    lib = s._lib

    def call(j0, times, n_spec=wl.n_spec, t_fast=T.data_ptr(), times_ptr=True):
        arr = (ctypes.c_double * max(1, len(times)))(*times)
        return lib.sim_run_updates(sim.ctx, ctypes.byref(sim.grid), prep.data_ptr(),
                                   ctypes.byref(sim.radar), j0, len(times),
                                   arr if times_ptr else None, t_fast, n_spec, None,
                                   torch.cuda.current_stream().cuda_stream)

    assert call(0, []) == s.SIM_ERR_SHAPE                       # count < 1
    assert call(-1, [0.0]) == s.SIM_ERR_SHAPE                   # j0 < 0
    assert call(2, [0.0, 1e-3]) == s.SIM_ERR_SHAPE              # past the last spectrum
    assert call(0, [0.0, float("nan")]) == s.SIM_ERR_ARG        # a time not finite
    assert call(0, [0.0], times_ptr=False) == s.SIM_ERR_ARG     # no times
    assert call(0, [0.0], t_fast=None) == s.SIM_ERR_ARG
    torch.cuda.synchronize()
    assert not T.cpu().numpy().any()                            # nothing launched
    assert call(1, [1e-3, 2e-3]) == s.SIM_OK
    torch.cuda.synchronize()
    # more lanes without a workspace re-sized for them: refused before launch
    T.zero_()
    assert lib.sim_set_tuning(sim.ctx, s.SIM_TUNE_UPDATE_LANES, 3) == s.SIM_OK
    assert lib.sim_set_tuning(sim.ctx, s.SIM_TUNE_UPDATE_LANES, 5) == s.SIM_ERR_ARG
    assert lib.sim_set_tuning(sim.ctx, s.SIM_TUNE_UPDATE_LANES, 0) == s.SIM_ERR_ARG
    assert call(0, [0.0, 1e-3, 2e-3]) == s.SIM_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert not T.cpu().numpy().any()
    sim.close()


def _lane_case(prec, nx=128, ny=64):
    from paper_2408_11472_amd import simradar
    fp64 = prec == "fp64"
    wl = workloads.tiny(nx=nx, ny=ny, spacing=2.0, n_gates=32, n_doppler=16, n_fast=16,
                        n_updates=8, cwm=1)
    g, r = wl.grid, wl.radar
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)
    sim = simradar.Simulator(g, r, simradar.SIM_PREC_FP64 if fp64 else
                             simradar.SIM_PREC_FP32_PHASE64)
    spec_t = torch.as_tensor(spec.astype(np.complex128 if fp64 else np.complex64), device="cuda")
    prep = sim.prepare_spectrum(spec_t)
    times = [(j * r.n_fast) / r.prf_hz for j in range(wl.n_spec)]
    return sim, prep, times, wl


@pytest.mark.parametrize("path", ["split", "fused"])
@pytest.mark.parametrize("lanes", [2, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_run_updates_on_lanes_equals_one_lane(prec, lanes, path):
    """Updates dealt to several streams, each with its own workspace slice
    (facet SoA on the split row path, band windows on both): the same spectra
    and counters as on the caller's stream alone."""
    from paper_2408_11472_amd import simradar
    print_case("run_updates lanes", prec, lanes, path)
    sim, prep, times, wl = _lane_case(prec)
    if path == "fused":
        sim.set_row_path(simradar.SIM_ROW_PATH_FUSED)
        sim.set_row_bands(16)
    else:
        sim.set_row_path(simradar.SIM_ROW_PATH_SPLIT)
    T1, c1 = sim.empty_spectra(wl.n_spec), sim.counters()
    sim.run_updates(prep, times, 0, T1, counters=c1)
    torch.cuda.synchronize()
    sim.set_update_lanes(lanes)
    T2, c2 = sim.empty_spectra(wl.n_spec), sim.counters()
    sim.run_updates(prep, times, 0, T2, counters=c2)
    # an odd range on the lanes (fewer updates than lanes at the end)
    T3 = sim.empty_spectra(wl.n_spec)
    sim.run_updates(prep, times[1:1 + lanes + 1], 1, T3)
    torch.cuda.synchronize()
    a, b, p = T1.cpu().numpy(), T2.cpu().numpy(), T3.cpu().numpy()
    assert np.array_equal(c1.cpu().numpy(), c2.cpu().numpy())
    tol = 1e-13 if prec == "fp64" else 1e-6
    assert rel_l2(b, a) <= tol, rel_l2(b, a)
    k = lanes + 1
    assert rel_l2(p[1:1 + k], a[1:1 + k]) <= tol
    assert not p[0].any() and not p[1 + k:].any()
    sim.close()


def test_run_updates_on_lanes_replayed_from_a_graph():
    """The forked lanes are captured with the caller's stream; every replay
    (with eager work between replays) gives the eager result."""
    print_case("run_updates lanes graph")
    sim, prep, times, wl = _lane_case("fp32", 64, 64)
    sim.set_update_lanes(3)
    T_ref = sim.empty_spectra(wl.n_spec)
    sim.run_updates(prep, times, 0, T_ref)
    torch.cuda.synchronize()
    ref = T_ref.cpu().numpy()
    T = sim.empty_spectra(wl.n_spec)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):                       # warm-up on the capture stream
        T.zero_()
        sim.run_updates(prep, times, 0, T)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        T.zero_()
        sim.run_updates(prep, times, 0, T)
    other = sim.empty_spectra(wl.n_spec)
    for rep in range(3):
        graph.replay()
        torch.cuda.synchronize()
        got = T.cpu().numpy()
        err = rel_l2(got, ref)
        print(f"replay {rep}: rel L2 {err:.2e}", flush=True)
        assert err <= 1e-6, (rep, err)
        other.zero_()
        sim.run_updates(prep, times, 0, other)            # eager work between replays
        torch.cuda.synchronize()
    assert rel_l2(other.cpu().numpy(), ref) <= 1e-6
    del graph
    sim.close()


@pytest.mark.parametrize("lanes", [1, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_accumulate_runs_equal_per_update_calls(prec, lanes):
    """sim_range_doppler_accumulate_run and its adjoint on stacked facet sets
    against one call per update: spectra (to the window-atomic order) and
    counters of the forward, the adjoint's gradients bit for bit."""
    from paper_2408_11472_amd import simradar
    print_case("accumulate runs", prec, lanes)
    sim, prep, times, wl = _lane_case(prec, 64, 32)
    g = wl.grid
    n = wl.n_spec
    stack = {k: torch.empty((n, g.ny, g.nx), dtype=sim.real_dtype, device="cuda")
             for k in simradar.FACET_FIELDS}
    for j in range(n):
        sim.surface_update(sim_spec(sim, wl), times[j], 1.0 / wl.radar.prf_hz,
                           out={k: stack[k][j] for k in stack})
    sim.set_update_lanes(lanes)
    T1, c1 = sim.empty_spectra(n), sim.counters()
    for j in range(n):
        sim.range_doppler_accumulate({k: stack[k][j] for k in stack}, times[j], j, T1,
                                     counters=c1)
    T2, c2 = sim.empty_spectra(n), sim.counters()
    sim.range_doppler_accumulate_run(stack, times, 0, T2, counters=c2)
    torch.cuda.synchronize()
    assert np.array_equal(c1.cpu().numpy(), c2.cpu().numpy())
    tol = 1e-13 if prec == "fp64" else 1e-6
    assert rel_l2(T2.cpu().numpy(), T1.cpu().numpy()) <= tol
    # adjoint on a seeded T-bar, updates 1 .. n - 1
    rng = np.random.default_rng(5)
    tb = rng.standard_normal(T1.shape) + 1j * rng.standard_normal(T1.shape)
    Tb = torch.as_tensor(tb.astype(np.complex128 if prec == "fp64" else np.complex64),
                         device="cuda")
    g1 = [torch.zeros((n, g.ny, g.nx), dtype=sim.real_dtype, device="cuda") for _ in range(3)]
    for j in range(1, n):
        sim.range_doppler_accumulate_adjoint({k: stack[k][j] for k in stack}, times[j], j, Tb,
                                             out=(g1[0][j], g1[1][j], g1[2][j]))
    g2 = [torch.zeros((n - 1, g.ny, g.nx), dtype=sim.real_dtype, device="cuda")
          for _ in range(3)]
    sim.range_doppler_accumulate_adjoint_run({k: v[1:] for k, v in stack.items()}, times[1:], 1,
                                             Tb, g2)
    torch.cuda.synchronize()
    for a, b in zip(g1, g2):
        assert torch.equal(a[1:], b)
        assert bool(torch.isfinite(b).all())
    with pytest.raises(ValueError):                 # a field that is not [count][ny][nx]
        sim.range_doppler_accumulate_run({k: v[0] for k, v in stack.items()}, times[:1], 0, T2)
    sim.close()


def sim_spec(sim, wl):
    g = wl.grid
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)
    return torch.as_tensor(spec.astype(np.complex128 if sim.precision == 0 else np.complex64),
                           device="cuda")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_accumulate_band_count_changes_only_summation_order(prec):
    """SIM_TUNE_ACC_BANDS: 64 bands against the default on a grid where they
    differ (bands hold at least 1024 facets): counters equal, spectra equal
    up to the order of the window sums; values outside the set are refused."""
    from paper_2408_11472_amd import simradar
    print_case("accumulate bands", prec)
    sim, prep, times, wl = _lane_case(prec, nx=512, ny=512)
    lib = simradar._lib
    for bad in (3, 32, 1024, -1):
        assert lib.sim_set_tuning(sim.ctx, simradar.SIM_TUNE_ACC_BANDS, bad) == \
            simradar.SIM_ERR_ARG
    T1, c1 = sim.empty_spectra(wl.n_spec), sim.counters()
    sim.run_updates(prep, times, 0, T1, counters=c1)
    sim.set_acc_bands(64)
    T2, c2 = sim.empty_spectra(wl.n_spec), sim.counters()
    sim.run_updates(prep, times, 0, T2, counters=c2)
    sim.set_acc_bands(0)
    torch.cuda.synchronize()
    assert np.array_equal(c1.cpu().numpy(), c2.cpu().numpy())
    err = rel_l2(T2.cpu().numpy(), T1.cpu().numpy())
    assert err <= (1e-13 if prec == "fp64" else 1e-5), err
    sim.close()
