"""Out-of-core runs (sim_streamer_*, Sec. III.B memory management): T_fast
and Y in pinned host memory, device caches of K update intervals, against
the in-HBM run of the same kernels on the same prepared spectrum.

The two runs execute the same kernels on the same inputs, so the spectra and
the IQ agree up to the order of the LDS float atomics within the window
cells: <= 1e-13 (FP64) and 1e-6 (FP32) relative L2.  Chunk sizes cover a
chunk of one interval, ragged last chunks, one chunk for the whole run and
more than the run.  The oracle pins the in-HBM path elsewhere; the streamed
IQ is also checked against the oracle's post-processing of the streamed
spectra (1e-12 / 1e-5)."""
import numpy as np
import pytest

import oracle.iq as oiq
from paper_2408_11472_amd import inputs, workloads
from tests.gpu_helpers import print_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("chunk", [1, 3, 4, 10, 64])
def test_streamed_run_equals_in_memory_run(prec, chunk):
    from paper_2408_11472_amd import simradar
    print_case("streamed run", prec, chunk)
    fp64 = prec == "fp64"
    wl = workloads.tiny(nx=256, ny=128, spacing=2.0, n_gates=64, n_doppler=64, n_fast=48,
                        n_updates=10, swh=1.5)
    g, r = wl.grid, wl.radar
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)
    sim = simradar.Simulator(g, r, simradar.SIM_PREC_FP64 if fp64 else
                             simradar.SIM_PREC_FP32_PHASE64)
    spec_t = torch.as_tensor(spec.astype(np.complex128 if fp64 else np.complex64),
                             device="cuda")
    prep = sim.prepare_spectrum(spec_t)
    T, Y = sim.run(None, wl.n_updates, prepared=prep)
    torch.cuda.synchronize()
    Th, Yh = sim.run_streamed(prep, wl.n_updates, chunk)
    assert not Th.is_cuda and not Yh.is_cuda
    tol = 1e-13 if fp64 else 1e-6
    eT = rel_l2(Th.numpy(), T.cpu().numpy())
    eY = rel_l2(Yh.numpy(), Y.cpu().numpy())
    print(f"streamed {prec} chunk {chunk}: T {eT:.2e} Y {eY:.2e}", flush=True)
    assert eT <= tol and eY <= tol, (eT, eY)
    Y_ref = oiq.segments_to_iq(Th.numpy().astype(np.complex128), r.n_fast, r.window)
    assert rel_l2(Yh.numpy(), Y_ref) <= (1e-12 if fp64 else 1e-5)
    # without the spectra
    _, Yh2 = sim.run_streamed(prep, wl.n_updates, chunk, keep_spectra=False)
    assert rel_l2(Yh2.numpy(), Y.cpu().numpy()) <= tol
    sim.close()


def test_streamer_rejects_bad_arguments():
    from paper_2408_11472_amd import simradar
    print_case("streamer errors")
    wl = workloads.tiny(nx=64, ny=64, spacing=2.0, n_gates=16, n_doppler=16, n_fast=16,
                        n_updates=2)
    sim = simradar.Simulator(wl.grid, wl.radar, simradar.SIM_PREC_FP32_PHASE64)
    with pytest.raises(simradar.SimError) as e:
        simradar.sim_streamer_create(sim.ctx, sim.radar, 0)
    assert e.value.status == simradar.SIM_ERR_SHAPE
    st = simradar.sim_streamer_create(sim.ctx, sim.radar, 2)
    n = simradar.sim_streamer_cache_size(st)
    cache = torch.empty(n, dtype=torch.uint8, device="cuda")
    y = torch.empty((32, 16), dtype=torch.complex64, pin_memory=True)
    spec = torch.zeros((64, 64), dtype=torch.complex64, device="cuda")
    prep = sim.prepare_spectrum(spec)
    stream = torch.cuda.current_stream().cuda_stream
    with pytest.raises(simradar.SimError) as e:     # cache too small
        simradar.sim_streamer_run(st, sim.grid, prep.data_ptr(), 2, None, y.data_ptr(),
                                  cache.data_ptr(), n - 1, stream)
    assert e.value.status == simradar.SIM_ERR_WORKSPACE
    with pytest.raises(simradar.SimError) as e:     # no update interval
        simradar.sim_streamer_run(st, sim.grid, prep.data_ptr(), 0, None, y.data_ptr(),
                                  cache.data_ptr(), n, stream)
    assert e.value.status == simradar.SIM_ERR_SHAPE
    simradar.sim_streamer_destroy(st)
    sim.close()
