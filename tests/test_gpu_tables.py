"""Tabulated antenna pattern and NRCS on the GPU (sim_set_tables, Sec. II.A
look-up tables) against the oracle with the same tables.

Same facet set for both (the oracle's surface, rounded to the context
precision): indices bit-exact (the tables change amplitudes only),
T_fast <= 1e-12 (FP64) / 1e-5 (FP32) relative L2 - the interpolation is
continuous across cells, so where the float and double cell coordinates
differ the values still agree to rounding.  The tables: a complex two-way
pattern (Gaussian beam times a phase ramp, so that the interpolated phase
matters) on a u-v grid that covers the scene, and an NRCS over the local
incidence (geometric optics times a ripple).  The whole chain from the
spectrum with tables is checked end to end at the FP64 bound."""
import numpy as np
import pytest

import oracle.fastmode as ofm
import oracle.iq as oiq
import oracle.scatter as osc
import oracle.surface as osurf
import oracle.tables as otab
from paper_2408_11472_amd import inputs, workloads
from tests.gpu_helpers import print_case, rel_l2, rounded_facets, to_torch_facets

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _tables(radar, span):
    gamma = (2.0 / np.log(2.0)) * np.sin(0.5 * radar.beamwidth_3db) ** 2
    k = 2.0 / gamma
    n = 65
    h = 2 * span / (n - 1)
    U = -span + h * np.arange(n)
    ant = np.exp(-k * (U[None, :] ** 2 + U[:, None] ** 2)) * \
        np.exp(1j * (3000.0 * U[None, :] - 2000.0 * U[:, None]))
    th = np.linspace(0.0, 0.6, 97)
    t2 = np.tan(th) ** 2
    c2 = 1.0 / (1.0 + t2)
    nrcs = radar.fresnel_sq / (radar.mss * c2 * c2) * np.exp(-t2 / radar.mss) * \
        (1.0 + 0.2 * np.sin(37.0 * th))
    return otab.Tables(antenna=ant, u0=U[0], du=h, v0=U[0], dv=h, nrcs=nrcs,
                       dtheta=th[1] - th[0])


def _set(sim, tab, which, fp64):
    cdt = torch.complex128 if fp64 else torch.complex64
    rdt = torch.float64 if fp64 else torch.float32
    ant = torch.as_tensor(tab.antenna, dtype=cdt, device="cuda") if "ant" in which else None
    nr = torch.as_tensor(tab.nrcs, dtype=rdt, device="cuda") if "nrcs" in which else None
    sim.set_tables(antenna=ant, u0=tab.u0, du=tab.du, v0=tab.v0, dv=tab.dv, nrcs=nr,
                   dtheta=tab.dtheta)
    return otab.Tables(antenna=tab.antenna if ant is not None else None, u0=tab.u0, du=tab.du,
                       v0=tab.v0, dv=tab.dv, nrcs=tab.nrcs if nr is not None else None,
                       dtheta=tab.dtheta)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("which", [("ant", "nrcs"), ("ant",), ("nrcs",)])
@pytest.mark.parametrize("nx,ny", [(128, 64), (512, 256)])
def test_tables_accumulate_matches_oracle(prec, which, nx, ny):
    from paper_2408_11472_amd import simradar
    print_case("tables accumulate", prec, which, nx, ny)
    fp64 = prec == "fp64"
    wl = workloads.tiny(nx=nx, ny=ny, spacing=2.0, n_gates=64, n_doppler=32, n_fast=32,
                        n_updates=2, swh=1.5)
    g, r = wl.grid, wl.radar
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)
    t = wl.update_time(1)
    fac = rounded_facets(osurf.facets(spec, g, t, 1.0 / r.prf_hz),
                         np.float64 if fp64 else np.float32)
    # the grid of the pattern covers the scene seen from the track (|u|, |v| < 1e-3)
    tab = _tables(r, span=2e-3)
    sim = simradar.Simulator(g, r, simradar.SIM_PREC_FP64 if fp64 else
                             simradar.SIM_PREC_FP32_PHASE64)
    otb = _set(sim, tab, which, fp64)
    T_ref, code_ref, cnt_ref = osc.accumulate(fac, g, r, t, tables=otb)
    T = sim.empty_spectra(wl.n_spec)
    code = torch.empty((g.ny, g.nx), dtype=torch.int32, device="cuda")
    sim.range_doppler_accumulate(to_torch_facets(fac, sim.real_dtype, "cuda"), t, 1, T,
                                 facet_code=code)
    torch.cuda.synchronize()
    assert np.array_equal(code.cpu().numpy(), code_ref)
    assert cnt_ref["illuminated"] > 0
    err = rel_l2(T[1].cpu().numpy(), T_ref)
    print(f"tables {which} {prec} {nx}x{ny}: T rel L2 {err:.2e}", flush=True)
    assert err <= (1e-12 if fp64 else 1e-5), err
    # the closed forms again after clearing the tables
    sim.set_tables()
    T2 = sim.empty_spectra(wl.n_spec)
    sim.range_doppler_accumulate(to_torch_facets(fac, sim.real_dtype, "cuda"), t, 1, T2)
    torch.cuda.synchronize()
    T2_ref = osc.accumulate(fac, g, r, t)[0]
    assert rel_l2(T2[1].cpu().numpy(), T2_ref) <= (1e-12 if fp64 else 1e-5)
    sim.close()


def test_tables_end_to_end_fp64_and_adjoint_rejected():
    from paper_2408_11472_amd import simradar
    print_case("tables end to end")
    wl = workloads.tiny(nx=128, ny=128, spacing=2.0, n_gates=64, n_doppler=32, n_fast=32,
                        n_updates=3, swh=1.5)
    g, r = wl.grid, wl.radar
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)
    tab = _tables(r, span=2e-3)
    sim = simradar.Simulator(g, r, simradar.SIM_PREC_FP64)
    otb = _set(sim, tab, ("ant", "nrcs"), True)
    T, Y = sim.run(torch.as_tensor(spec, device="cuda"), wl.n_updates)
    torch.cuda.synchronize()
    T_ref = np.stack([osc.accumulate(osurf.facets(spec, g, wl.update_time(j), 1.0 / r.prf_hz),
                                     g, r, wl.update_time(j), tables=otb)[0]
                      for j in range(wl.n_spec)])
    Y_ref = oiq.segments_to_iq(T_ref, r.n_fast, r.window)
    assert rel_l2(T.cpu().numpy(), T_ref) <= 1e-9
    assert rel_l2(Y.cpu().numpy(), Y_ref) <= 1e-9
    # the closed-form run differs (the tables are really used)
    T0, _ = ofm.simulate(spec, g, r, wl.n_updates)
    assert rel_l2(T_ref, T0) > 1e-3
    fac = sim.surface_update(torch.as_tensor(spec, device="cuda"), 0.0, 1.0 / r.prf_hz)
    with pytest.raises(simradar.SimError) as e:
        sim.range_doppler_accumulate_adjoint(fac, 0.0, 0, T)
    assert e.value.status == simradar.SIM_ERR_UNSUPPORTED
    sim.close()
