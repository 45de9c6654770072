"""Batched realisations: a batch run (eager and as a replayed HIP graph)
gives the same spectra and IQ as running each realisation alone, and matches
the oracle."""
import numpy as np
import pytest

import oracle.fastmode as ofm
from paper_2408_11472_amd import inputs, workloads
from tests.gpu_helpers import print_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _members():
    # uneven grids, different sea states and window sizes
    # three members share a shape (one persistent class, with different
    # update counts: the class launch of update j holds only members with
    # j <= U)
    spec = [(64, 64, 2.0, 8, 16, 16, 2, 1.5), (128, 32, 1.0, 16, 8, 8, 3, 2.5),
            (32, 256, 2.0, 8, 32, 32, 1, 3.0), (64, 64, 2.0, 8, 16, 16, 4, 2.0),
            (64, 64, 2.0, 8, 16, 16, 1, 1.0)]
    out = []
    for i, (nx, ny, d, G, N, nf, U, swh) in enumerate(spec):
        wl = workloads.tiny(nx=nx, ny=ny, spacing=d, n_gates=G, n_doppler=N, n_fast=nf,
                            n_updates=U, seed=60 + i, swh=swh)
        out.append(wl)
    return out


def _spec(wl):
    g = wl.grid
    return inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)


MODES = [1, 2]      # SIM_BATCH_LANES, SIM_BATCH_PERSISTENT


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec,pcode,cdt,tol", [("fp64", 0, np.complex128, 1e-9),
                                                ("fp32", 1, np.complex64, 5e-3)])
def test_batch_matches_single_runs_and_oracle(prec, pcode, cdt, tol, mode):
    from paper_2408_11472_amd import simradar
    print_case("batch", prec, "mode", mode)
    wls = _members()
    specs_np = [_spec(w) for w in wls]
    batch = simradar.Batch([(w.grid, w.radar, w.n_updates) for w in wls], pcode)
    batch.set_mode(mode)
    specs = [torch.as_tensor(s.astype(cdt), device="cuda") for s in specs_np]
    T, Y = batch.empty_outputs()
    batch.run(specs, T, Y, use_graph=False)
    torch.cuda.synchronize()
    for w, s_np, s_t, Tb, Yb in zip(wls, specs_np, specs, T, Y):
        sim = simradar.Simulator(w.grid, w.radar, pcode)
        T1, Y1 = sim.run(s_t, w.n_updates)
        torch.cuda.synchronize()
        # same kernels, same order: equal up to the summation order of the
        # LDS window atomics
        assert rel_l2(Tb.cpu().numpy(), T1.cpu().numpy()) <= (1e-13 if prec == "fp64" else 1e-6)
        T_ref, Y_ref = ofm.simulate(s_np, w.grid, w.radar, w.n_updates)
        assert rel_l2(Tb.cpu().numpy(), T_ref) <= tol
        assert rel_l2(Yb.cpu().numpy(), Y_ref) <= tol
        sim.close()
    batch.close()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("prec,pcode,cdt", [("fp64", 0, np.complex128), ("fp32", 1, np.complex64)])
def test_graph_replays_match_eager(prec, pcode, cdt, mode):
    from paper_2408_11472_amd import simradar
    print_case("graph", prec, "mode", mode)
    wls = _members()
    batch = simradar.Batch([(w.grid, w.radar, w.n_updates) for w in wls], pcode)
    batch.set_mode(mode)
    specs = [torch.as_tensor(_spec(w).astype(cdt), device="cuda") for w in wls]
    T, Y = batch.empty_outputs()
    batch.run(specs, T, Y, use_graph=False)
    torch.cuda.synchronize()
    T_eager = [t.cpu().numpy() for t in T]
    Y_eager = [y.cpu().numpy() for y in Y]
    for rep in range(3):
        # eager work between replays dirties the outputs
        for t in T:
            t.fill_(complex(1.0, -2.0))
        for y in Y:
            y.fill_(complex(3.0, 4.0))
        torch.cuda.synchronize()
        batch.run(specs, T, Y, use_graph=True)
        torch.cuda.synchronize()
        for a, b in zip(T, T_eager):
            assert rel_l2(a.cpu().numpy(), b) <= (1e-13 if prec == "fp64" else 1e-6), rep
        for a, b in zip(Y, Y_eager):
            assert rel_l2(a.cpu().numpy(), b) <= (1e-13 if prec == "fp64" else 1e-6), rep
    batch.close()


# Band counts regroup the window partial sums: a summation-order change over
# cells of up to ~1e3 nearly coherent terms (eps * n_cell relative).
@pytest.mark.parametrize("prec,pcode,cdt,tol", [("fp64", 0, np.complex128, 1e-13),
                                                ("fp32", 1, np.complex64, 1e-5)])
def test_band_count_changes_only_summation_order(prec, pcode, cdt, tol, tmp_path, monkeypatch):
    from paper_2408_11472_amd import autotune, simradar
    print_case("bands", prec)
    monkeypatch.setenv("SIMRADAR_TUNING_CACHE", str(tmp_path / "tuning.json"))
    wl = workloads.small_256()
    spec = torch.as_tensor(_spec(wl).astype(cdt), device="cuda")
    sim = simradar.Simulator(wl.grid, wl.radar, pcode)
    outs = []
    with pytest.raises(simradar.SimError):
        sim.set_row_bands(3)                     # band counts are powers of two
    for nb in (0, 8, 32, 2, 64):
        sim.set_row_bands(nb)
        T = sim.empty_spectra(wl.n_spec)
        cnt = sim.counters()
        sim.update_and_accumulate(spec, wl.update_time(4), 4, T, counters=cnt)
        torch.cuda.synchronize()
        assert int(cnt.cpu()[:5].sum()) == wl.n_facets, nb     # every row walked once
        outs.append(T.cpu().numpy())
    for o in outs[1:]:
        assert rel_l2(o, outs[0]) <= tol
    entry = autotune.tune(sim, spec, repeats=2,
                          run_times=[wl.update_time(j) for j in range(wl.n_spec)])
    assert entry["row_path"] in (autotune.PATH_FUSED, autotune.PATH_SPLIT)
    if entry["row_path"] == autotune.PATH_FUSED:
        assert entry["row_bands"] in autotune.CANDIDATE_BANDS
    assert entry["update_lanes"] in autotune.CANDIDATE_LANES
    assert sim.lanes == entry["update_lanes"]
    again = autotune.tune(sim, spec)                                       # cached
    assert (again["row_path"], again["row_bands"], again["update_lanes"]) == \
        (entry["row_path"], entry["row_bands"], entry["update_lanes"])
    # the tuned context still computes the same spectrum
    T = sim.empty_spectra(wl.n_spec)
    sim.run(None, wl.n_updates, t_fast=T, prepared=sim.prepare_spectrum(spec))
    torch.cuda.synchronize()
    T_one = sim.empty_spectra(wl.n_spec)
    for j in range(wl.n_spec):
        sim.update_and_accumulate(spec, wl.update_time(j), j, T_one)
    torch.cuda.synchronize()
    assert rel_l2(T.cpu().numpy(), T_one.cpu().numpy()) <= tol
    sim.close()


@pytest.mark.parametrize("prec,pcode,cdt", [("fp64", 0, np.complex128), ("fp32", 1, np.complex64)])
@pytest.mark.parametrize("which", ["tiny", "small_256"])
def test_row_paths_agree(prec, pcode, cdt, which):
    """The fused row pass and the split facet row pass + facet accumulate give
    the same spectra and the same facet indices."""
    from paper_2408_11472_amd import simradar
    print_case("row paths", prec, which)
    wl = workloads.small_256() if which == "small_256" else workloads.tiny(
        nx=64, ny=32, spacing=2.0, n_gates=32, n_doppler=16, n_fast=16, n_updates=3)
    spec = torch.as_tensor(_spec(wl).astype(cdt), device="cuda")
    sim = simradar.Simulator(wl.grid, wl.radar, pcode)
    out = {}
    for path in (simradar.SIM_ROW_PATH_FUSED, simradar.SIM_ROW_PATH_SPLIT):
        sim.set_row_path(path)
        T = sim.empty_spectra(wl.n_spec)
        code = torch.empty((wl.grid.ny, wl.grid.nx), dtype=torch.int32, device="cuda")
        cnt = sim.counters()
        sim.update_and_accumulate(spec, wl.update_time(2), 2, T, counters=cnt, facet_code=code)
        torch.cuda.synchronize()
        out[path] = (T.cpu().numpy(), code.cpu().numpy(), cnt.cpu().numpy())
    (Tf, cf, nf), (Ts, cs_, ns) = out[simradar.SIM_ROW_PATH_FUSED], out[simradar.SIM_ROW_PATH_SPLIT]
    n_diff = int((cf != cs_).sum())
    assert n_diff <= (0 if prec == "fp64" else max(2, cf.size // 10000)), n_diff
    assert rel_l2(Tf, Ts) <= (1e-12 if prec == "fp64" else 1e-5 + 3 * np.sqrt(2 * n_diff / cf.size))
    assert int(nf[:5].sum()) == int(ns[:5].sum()) == wl.n_facets
    sim.close()


@pytest.mark.parametrize("prec,pcode,cdt", [("fp64", 0, np.complex128), ("fp32", 1, np.complex64)])
def test_persistent_mode_equals_lanes_mode_on_new_buffers(prec, pcode, cdt):
    """Both batch modes on one batch object, then the persistent mode again
    on another set of output buffers (its descriptors are rebuilt)."""
    from paper_2408_11472_amd import simradar
    print_case("batch modes", prec)
    wls = _members()
    batch = simradar.Batch([(w.grid, w.radar, w.n_updates) for w in wls], pcode)
    specs = [torch.as_tensor(_spec(w).astype(cdt), device="cuda") for w in wls]
    out = {}
    for mode in (simradar.SIM_BATCH_LANES, simradar.SIM_BATCH_PERSISTENT,
                 simradar.SIM_BATCH_PERSISTENT):
        batch.set_mode(mode)
        T, Y = batch.empty_outputs()
        batch.run(specs, T, Y)
        torch.cuda.synchronize()
        out.setdefault(mode, []).append(([t.cpu().numpy() for t in T],
                                         [y.cpu().numpy() for y in Y]))
    tol = 1e-13 if prec == "fp64" else 1e-6
    ref_T, ref_Y = out[simradar.SIM_BATCH_LANES][0]
    for T, Y in out[simradar.SIM_BATCH_PERSISTENT]:
        for a, b in zip(T + Y, ref_T + ref_Y):
            assert rel_l2(a, b) <= tol
    with pytest.raises(simradar.SimError):
        batch.set_mode(7)
    batch.close()



@pytest.mark.parametrize("prec,pcode,cdt", [("fp64", 0, np.complex128), ("fp32", 1, np.complex64)])
def test_member_accumulate_bands_change_only_summation_order(prec, pcode, cdt):
    """SIM_TUNE_ACC_BANDS per member of the lanes mode (a 512^2 member, where
    64 bands and the default differ): the same spectra up to the order of the
    window sums, eager and from a recaptured graph; bad values refused."""
    from paper_2408_11472_amd import simradar
    print_case("batch acc bands", prec)
    wls = _members()[:2] + [workloads.tiny(nx=512, ny=512, spacing=2.0, n_gates=16,
                                           n_doppler=16, n_fast=16, n_updates=2, seed=77)]
    batch = simradar.Batch([(w.grid, w.radar, w.n_updates) for w in wls], pcode)
    batch.set_mode(simradar.SIM_BATCH_LANES)
    specs = [torch.as_tensor(_spec(w).astype(cdt), device="cuda") for w in wls]
    T1, Y1 = batch.empty_outputs()
    batch.run(specs, T1, Y1, use_graph=False)
    lib = simradar._lib
    for bad in (3, 32, 1024):
        assert lib.sim_batch_set_tuning(batch.batch, 2, simradar.SIM_TUNE_ACC_BANDS, bad) == \
            simradar.SIM_ERR_ARG
    for i in range(len(wls)):
        simradar.sim_batch_set_tuning(batch.batch, i, simradar.SIM_TUNE_ACC_BANDS, 64)
    T2, Y2 = batch.empty_outputs()
    batch.run(specs, T2, Y2, use_graph=False)
    T3, Y3 = batch.empty_outputs()
    batch.run(specs, T3, Y3, use_graph=True)
    torch.cuda.synchronize()
    tol = 1e-13 if prec == "fp64" else 1e-5
    for a, b, c in zip(T1, T2, T3):
        assert rel_l2(b.cpu().numpy(), a.cpu().numpy()) <= tol
        assert rel_l2(c.cpu().numpy(), a.cpu().numpy()) <= tol
    batch.close()
