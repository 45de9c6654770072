"""The allocation-free accumulate entry point against the workspace one.

sim_range_doppler_accumulate_noalloc keeps its band windows in the
library's static device scratch instead of the context's workspace.  On the
same facet set it must give the same per-facet codes and counters (bit for
bit) and the same T_fast[j] up to the summation order of the partial spectra
(relative L2 <= 1e-12 in FP64, 1e-5 in FP32: float sums of a few thousand
terms per window cell, in another band partition).  Two calls in a row on
one device, the second on a smaller grid, check that the scratch keeps no
state that the second call would read (headers and counters of the first
call's extra bands).
"""
import numpy as np
import pytest

from paper_2408_11472_amd import inputs, workloads
from tests.gpu_helpers import print_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case(sim, wl, j):
    """The facet set of update j from the GPU surface update."""
    g, r = wl.grid, wl.radar
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed, wl.sea.swell)
    cdt = np.complex128 if sim.precision == 0 else np.complex64
    spec_t = torch.as_tensor(spec.astype(cdt), device="cuda")
    t = wl.update_time(j)
    return sim.surface_update(spec_t, t, 1.0 / r.prf_hz), t


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_accumulate_equals_workspace_accumulate(prec):
    from paper_2408_11472_amd import simradar
    fp64 = prec == "fp64"
    pcode = simradar.SIM_PREC_FP64 if fp64 else simradar.SIM_PREC_FP32_PHASE64
    tol = 1e-12 if fp64 else 1e-5
    # a large grid first (512 bands in the workspace path, 256 in the scratch),
    # then a smaller one with fewer bands and another radar
    cases = [workloads.tiny(nx=1024, ny=1024, spacing=1.0, n_gates=64, n_doppler=128,
                            n_fast=64, n_updates=4, swh=2.0),
             workloads.tiny(nx=256, ny=128, spacing=1.0, n_gates=32, n_doppler=64,
                            n_fast=32, n_updates=3, swh=1.5, seed=5)]
    for wl in cases:
        print_case("noalloc accumulate", prec, wl.grid.nx, wl.grid.ny)
        sim = simradar.Simulator(wl.grid, wl.radar, pcode)
        j = wl.n_updates // 2
        fac, t = _case(sim, wl, j)
        g = wl.grid
        T_ws = sim.empty_spectra(wl.n_spec)
        T_na = sim.empty_spectra(wl.n_spec)
        c_ws, c_na = sim.counters(), sim.counters()
        k_ws = torch.empty((g.ny, g.nx), dtype=torch.int32, device="cuda")
        k_na = torch.full((g.ny, g.nx), 7, dtype=torch.int32, device="cuda")
        sim.range_doppler_accumulate(fac, t, j, T_ws, counters=c_ws, facet_code=k_ws)
        sim.range_doppler_accumulate_noalloc(fac, t, j, T_na, counters=c_na, facet_code=k_na)
        torch.cuda.synchronize()
        assert torch.equal(k_ws, k_na)
        cw, cn = c_ws.cpu().numpy(), c_na.cpu().numpy()
        assert (cw[:5] == cn[:5]).all(), (cw, cn)
        assert int(cn[:5].sum()) == g.nx * g.ny
        assert int(cn[0]) > 0
        # only spectrum j is touched
        others = [i for i in range(wl.n_spec) if i != j]
        assert not torch.any(T_na[others] != 0)
        err = rel_l2(T_na[j].cpu().numpy(), T_ws[j].cpu().numpy())
        print(f"noalloc vs workspace {prec} {g.nx}x{g.ny}: rel L2 {err:.2e}, "
              f"illuminated {int(cn[0])}", flush=True)
        assert err <= tol, err
        sim.close()


def test_noalloc_accumulate_needs_no_workspace():
    """The scratch entry point runs on a context with no workspace attached,
    where the workspace entry point reports SIM_ERR_WORKSPACE."""
    from paper_2408_11472_amd import simradar
    print_case("noalloc without workspace")
    wl = workloads.tiny(nx=64, ny=64, spacing=2.0, n_gates=32, n_doppler=16, n_fast=16,
                        n_updates=2)
    sim = simradar.Simulator(wl.grid, wl.radar, simradar.SIM_PREC_FP32_PHASE64)
    fac, t = _case(sim, wl, 1)
    T_ref = sim.empty_spectra(wl.n_spec)
    sim.range_doppler_accumulate(fac, t, 1, T_ref)
    simradar.sim_set_workspace(sim.ctx, None, 0)
    T = sim.empty_spectra(wl.n_spec)
    with pytest.raises(simradar.SimError) as e:
        sim.range_doppler_accumulate(fac, t, 1, T)
    assert e.value.status == simradar.SIM_ERR_WORKSPACE
    sim.range_doppler_accumulate_noalloc(fac, t, 1, T)
    torch.cuda.synchronize()
    assert rel_l2(T.cpu().numpy(), T_ref.cpu().numpy()) <= 1e-5
    sim.close()
