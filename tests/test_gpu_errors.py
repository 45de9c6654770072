"""Error paths of the C ABI with a live context: every rejected call returns
its status synchronously and launches nothing, and the context stays usable."""
import ctypes

import numpy as np
import pytest

from paper_2408_11472_amd import workloads
from tests.gpu_helpers import print_case

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _structs(s, wl):
    return s.grid_struct(wl.grid), s.radar_struct(wl.radar)


def test_rejected_calls_return_their_status_and_leave_the_context_usable():
    from paper_2408_11472_amd import simradar as s
    print_case("errors")
    lib = s._lib
    wl = workloads.tiny(nx=64, ny=32, spacing=2.0, n_gates=16, n_doppler=16, n_fast=16,
                        n_updates=2)
    sim = s.Simulator(wl.grid, wl.radar, s.SIM_PREC_FP32_PHASE64)
    g, r = _structs(s, wl)
    n = ctypes.c_size_t()

    def ws_status(**kw):
        gg = s.sim_grid.from_buffer_copy(g)
        rr = s.sim_radar.from_buffer_copy(r)
        for k, v in kw.items():
            setattr(gg if hasattr(gg, k) and k in dict(s.sim_grid._fields_) else rr, k, v)
        return lib.sim_workspace_size(sim.ctx, ctypes.byref(gg), ctypes.byref(rr), ctypes.byref(n))

    # sizes outside the supported set
    assert ws_status(nx=48) == s.SIM_ERR_UNSUPPORTED
    assert ws_status(ny=32768) == s.SIM_ERR_UNSUPPORTED
    assert ws_status(nx=8) == s.SIM_ERR_UNSUPPORTED
    assert ws_status(n_doppler=24) == s.SIM_ERR_UNSUPPORTED
    assert ws_status(n_doppler=4096) == s.SIM_ERR_UNSUPPORTED
    # invalid values
    assert ws_status(dx=0.0) == s.SIM_ERR_ARG
    assert ws_status(gravity=float("nan")) == s.SIM_ERR_ARG
    assert ws_status(prf_hz=-1.0) == s.SIM_ERR_ARG
    assert ws_status(n_gates=0) == s.SIM_ERR_ARG
    assert ws_status(n_fast=0) == s.SIM_ERR_ARG
    assert ws_status(window=7) == s.SIM_ERR_ARG
    assert ws_status() == s.SIM_OK

    spec = torch.zeros((32, 64), dtype=torch.complex64, device="cuda")
    T = sim.empty_spectra(wl.n_spec)
    st = torch.cuda.current_stream().cuda_stream
    # update index outside [0, n_spec)
    for j in (-1, wl.n_spec):
        assert lib.sim_update_and_accumulate(sim.ctx, ctypes.byref(g), spec.data_ptr(),
                                             ctypes.byref(r), 0.0, j, T.data_ptr(), wl.n_spec,
                                             None, None, st) == s.SIM_ERR_SHAPE
    # non-finite time, missing buffers
    assert lib.sim_update_and_accumulate(sim.ctx, ctypes.byref(g), spec.data_ptr(),
                                         ctypes.byref(r), float("inf"), 0, T.data_ptr(),
                                         wl.n_spec, None, None, st) == s.SIM_ERR_ARG
    assert lib.sim_update_and_accumulate(sim.ctx, ctypes.byref(g), None, ctypes.byref(r), 0.0,
                                         0, T.data_ptr(), wl.n_spec, None, None,
                                         st) == s.SIM_ERR_ARG
    # post-processing needs two spectra at least
    Y = torch.empty((16, 16), dtype=torch.complex64, device="cuda")
    assert lib.sim_segments_to_iq(sim.ctx, ctypes.byref(r), T.data_ptr(), 1, Y.data_ptr(),
                                  st) == s.SIM_ERR_SHAPE
    # prepared spectrum: misaligned buffer
    prep = torch.empty(2 * 64 * 32 + 1, dtype=torch.complex64, device="cuda")
    assert lib.sim_prepare_spectrum(sim.ctx, ctypes.byref(g), spec.data_ptr(),
                                    prep.data_ptr() + 4, st) == s.SIM_ERR_ARG
    # tuning values
    assert lib.sim_set_tuning(sim.ctx, s.SIM_TUNE_ROW_PATH, 5) == s.SIM_ERR_ARG
    assert lib.sim_set_tuning(sim.ctx, 99, 0) == s.SIM_ERR_ARG
    # a workspace too small for the radar's windows, then none at all
    small = torch.empty(6 * 64 * 32 * 8 + 256, dtype=torch.uint8, device="cuda")
    base = (small.data_ptr() + 255) & ~255
    assert lib.sim_set_workspace(sim.ctx, base, 6 * 64 * 32 * 8) == s.SIM_OK
    assert lib.sim_update_and_accumulate(sim.ctx, ctypes.byref(g), spec.data_ptr(),
                                         ctypes.byref(r), 0.0, 0, T.data_ptr(), wl.n_spec,
                                         None, None, st) == s.SIM_ERR_WORKSPACE
    assert lib.sim_set_workspace(sim.ctx, None, 0) == s.SIM_OK
    fac = sim.empty_facets()
    assert lib.sim_surface_update(sim.ctx, ctypes.byref(g), spec.data_ptr(), 0.0, 1e-4,
                                  ctypes.byref(sim._facets_struct(fac)), st) == s.SIM_ERR_WORKSPACE
    # back to the full workspace: the context still computes (a zero spectrum
    # is a flat sea)
    s.sim_set_workspace(sim.ctx, sim._ws_ptr, sim.workspace.numel() - 256)
    cnt = sim.counters()
    sim.update_and_accumulate(spec, 0.0, 0, T, counters=cnt)
    torch.cuda.synchronize()
    Tn = T.cpu().numpy()
    assert np.isfinite(Tn.view(np.float32)).all() and np.abs(Tn[0]).max() > 0
    assert not np.any(Tn[1:])
    assert int(cnt.cpu()[:5].sum()) == wl.n_facets
    sim.close()


def test_fp64_context_rejects_columns_longer_than_its_lds():
    from paper_2408_11472_amd import simradar as s
    print_case("errors fp64 ny")
    wl = workloads.tiny(nx=32, ny=16384, spacing=1.0)
    with pytest.raises(s.SimError) as e:
        s.Simulator(wl.grid, wl.radar, s.SIM_PREC_FP64)
    assert e.value.status == s.SIM_ERR_UNSUPPORTED


def test_batch_rejects_empty_runs():
    from paper_2408_11472_amd import simradar as s
    print_case("errors batch")
    wl = workloads.tiny()
    with pytest.raises(s.SimError) as e:
        s.Batch([(wl.grid, wl.radar, 0)])
    assert e.value.status == s.SIM_ERR_SHAPE
