"""Parity of the HIP adjoint chain (waveform loss, IQ adjoint, per-facet
gradients, autograd wrapper) with the FP64 oracle adjoint.

Tolerances: FP64 context <= 1e-10 relative L2; FP32 context <= 2e-4
(float spectra, IQ and adjoint transforms; the range and phase derivative in
double)."""
import numpy as np
import pytest

import oracle.adjoint as oad
import oracle.iq as oiq
import oracle.surface as osurf
from paper_2408_11472_amd import inputs, workloads
from tests.gpu_helpers import print_case, rel_l2, rounded_facets, to_torch_facets

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PRECS = [("fp64", 0, np.float64, 1e-10), ("fp32", 1, np.float32, 2e-4)]


def _sim(wl, pcode):
    from paper_2408_11472_amd import simradar
    return simradar.Simulator(wl.grid, wl.radar, pcode)


@pytest.mark.parametrize("prec,pcode,npdt,tol", PRECS)
@pytest.mark.parametrize("G,N,n_fast,n_spec,window", [(5, 8, 8, 3, 0), (64, 64, 64, 9, 1),
                                                      (3, 16, 24, 4, 0), (130, 256, 128, 3, 0)])
def test_iq_adjoint_matches_oracle(prec, pcode, npdt, tol, G, N, n_fast, n_spec, window):
    print_case("iq adjoint", prec, G, N, n_fast, n_spec, window)
    wl = workloads.tiny(n_gates=G, n_doppler=N, n_fast=n_fast, window=window)
    sim = _sim(wl, pcode)
    rng = np.random.default_rng(G + N)
    Yb = rng.standard_normal(((n_spec - 1) * n_fast, G)) + 1j * rng.standard_normal(((n_spec - 1) * n_fast, G))
    cdt = np.complex64 if npdt == np.float32 else np.complex128
    got = sim.segments_to_iq_adjoint(torch.as_tensor(Yb.astype(cdt), device="cuda"), n_spec)
    ref = oad.segments_to_iq_adjoint(Yb.astype(cdt).astype(complex), n_spec, N, n_fast, window)
    assert rel_l2(got.cpu().numpy(), ref) <= tol


def _case(nx=32, ny=32, U=3, seed=41):
    wl = workloads.tiny(nx=nx, ny=ny, spacing=2.0, n_gates=32, n_doppler=16, n_fast=16,
                        n_updates=U, seed=seed)
    g, r = wl.grid, wl.radar
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)
    times = [wl.update_time(j) for j in range(wl.n_spec)]
    facs = [osurf.facets(spec, g, t, 1.0 / r.prf_hz) for t in times]
    target = np.random.default_rng(seed).random(r.n_gates) * 50.0
    return wl, facs, times, target


@pytest.mark.parametrize("prec,pcode,npdt,tol", PRECS)
def test_autograd_waveform_loss_matches_oracle_gradient(prec, pcode, npdt, tol):
    from paper_2408_11472_amd.autograd import FIXED_FIELDS, waveform_loss
    print_case("autograd", prec)
    wl, facs, times, target = _case()
    facs_r = [rounded_facets(f, npdt) for f in facs]
    L_ref, g_ref = oad.gradients(facs_r, times, wl.grid, wl.radar, target)
    sim = _sim(wl, pcode)
    dt = sim.real_dtype
    stack = lambda k: torch.as_tensor(np.stack([f[k] for f in facs_r]), dtype=dt, device="cuda")
    h = stack("h").requires_grad_(True)
    sx = stack("sx").requires_grad_(True)
    sy = stack("sy").requires_grad_(True)
    fixed = {k: stack(k) for k in FIXED_FIELDS}
    tgt = torch.as_tensor(target, dtype=dt, device="cuda")
    L = waveform_loss(h, sx, sy, sim, fixed, times, tgt)
    (2.5 * L).backward()
    torch.cuda.synchronize()
    assert abs(float(L) - L_ref) <= (1e-10 if prec == "fp64" else 1e-4) * abs(L_ref)
    for name, t in (("h", h), ("sx", sx), ("sy", sy)):
        ref = 2.5 * np.stack([g[name] for g in g_ref])
        err = rel_l2(t.grad.cpu().numpy(), ref)
        assert err <= tol, (name, err)


@pytest.mark.parametrize("prec,pcode,npdt,tol", PRECS)
def test_gradient_workload_shape_one_update(prec, pcode, npdt, tol):
    # the 2048^2-facet gradient workload, one update's facet gradients against
    # the oracle (T_bar from the oracle chain of that single update)
    print_case("gradient 2048 one update", prec)
    wl = workloads.gradient_2048()
    g, r = wl.grid, wl.radar
    spec = inputs.sea_spectrum(g.nx, g.ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)
    j = 5
    t = wl.update_time(j)
    fac = rounded_facets(osurf.facets(spec, g, t, 1.0 / r.prf_hz), npdt)
    rng = np.random.default_rng(3)
    Tbar = (rng.standard_normal((wl.n_spec, r.n_gates, r.n_doppler))
            + 1j * rng.standard_normal((wl.n_spec, r.n_gates, r.n_doppler)))
    cdt = np.complex64 if npdt == np.float32 else np.complex128
    Tbar = Tbar.astype(cdt)
    ref = oad.facet_gradients(fac, g, r, t, Tbar[j].astype(complex))
    sim = _sim(wl, pcode)
    got = sim.range_doppler_accumulate_adjoint(to_torch_facets(fac, sim.real_dtype, "cuda"), t, j,
                                               torch.as_tensor(Tbar, device="cuda"))
    torch.cuda.synchronize()
    for name in ("h", "sx", "sy"):
        err = rel_l2(got[name].cpu().numpy(), ref[name])
        assert err <= tol, (name, err)
