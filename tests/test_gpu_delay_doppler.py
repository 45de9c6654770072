"""Delay-Doppler processing on the GPU (sim_delay_doppler, Sec. IV.C)
against the oracle on the same IQ.

Bounds (relative L2 unless stated): the focused beams, beam powers and
multi-looked waveform <= 1e-12 in FP64 and 1e-5 in FP32 (float transforms of
<= 256 points and double sums); the centroid used per burst within 1e-12
(FP64) / 1e-6 (FP32) cycles per pulse.  The oracle returns powers only, so
the complex beams are compared through a second oracle evaluation of the
same steps (centroid ramp, along-track DFT, delay coefficients)."""
import numpy as np
import pytest

import oracle.delay_doppler as odd
from paper_2408_11472_amd import workloads
from tests.gpu_helpers import print_case, rel_l2

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _oracle_beams(Y, radar, M, centroid, migration):
    """Complex beams of every burst (the oracle's steps 1-3 without |.|^2)."""
    nb = Y.shape[0] // M
    out, cents = [], []
    x = np.arange(M)
    E = np.exp(-2j * np.pi * np.outer(x, x) / M)
    G = Y.shape[1]
    q = np.arange(G)
    qs = np.where(q < G // 2, q, q - G)
    for b in range(nb):
        blk = Y[b * M:(b + 1) * M]
        uc = odd.centroid_cycles(blk) if centroid is None else centroid
        cents.append(uc)
        Z = E @ (blk * np.exp(-2j * np.pi * uc * x)[:, None])
        if migration:
            for f in range(M):
                d = odd.migration_gates(odd.beam_cycles(M)[f], radar)
                Z[f] = np.fft.ifft(np.fft.fft(Z[f]) * np.exp(2j * np.pi * qs * d / G))
        out.append(Z)
    return np.stack(out), np.array(cents)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("M,G,n_pulses,centroid,migration", [
    (64, 128, 640, None, True), (16, 32, 200, 0.0, True), (64, 64, 256, 0.0137, False),
    (256, 16, 512, None, True), (2, 2, 9, None, False), (8, 2048, 16, None, True)])
def test_delay_doppler_matches_oracle(prec, M, G, n_pulses, centroid, migration):
    from paper_2408_11472_amd import simradar
    print_case("delay doppler", prec, M, G, n_pulses, centroid, migration)
    fp64 = prec == "fp64"
    wl = workloads.tiny(n_gates=G, n_doppler=16, n_fast=16)
    sim = simradar.Simulator(wl.grid, wl.radar, simradar.SIM_PREC_FP64 if fp64 else
                             simradar.SIM_PREC_FP32_PHASE64)
    rng = np.random.default_rng(M * 1000 + G)
    # random IQ with a drifting tone so that the centroid is not trivial
    x = np.arange(n_pulses)
    Y = (rng.standard_normal((n_pulses, G)) + 1j * rng.standard_normal((n_pulses, G))) * 0.3
    Y += np.exp(2j * np.pi * 0.021 * x)[:, None]
    Yc = Y.astype(np.complex128 if fp64 else np.complex64)
    out = sim.delay_doppler(torch.as_tensor(Yc, device="cuda"), burst=M, centroid=centroid,
                            migration=migration)
    torch.cuda.synchronize()
    Yr = Yc.astype(np.complex128)
    Zr, cr = _oracle_beams(Yr, wl.radar, M, centroid, migration)
    P, w = odd.delay_doppler(Yr, wl.radar, burst=M, centroid=centroid, migration=migration)
    tol = 1e-12 if fp64 else 1e-5
    c = out["centroid"].cpu().numpy().astype(np.float64)
    assert np.max(np.abs(c - cr)) <= (1e-12 if fp64 else 1e-6), (c, cr)
    if not fp64 and centroid is None:
        # the float kernel removes its own (float-rounded) centroid: compare
        # with the oracle's beams for that centroid
        Zr = np.stack([_oracle_beams(Yr[b * M:(b + 1) * M], wl.radar, M, float(c[b]),
                                     migration)[0][0] for b in range(len(c))])
        P = np.abs(Zr) ** 2
        w = P.mean(axis=(0, 1))
    errs = {"beams": rel_l2(out["beams"].cpu().numpy(), Zr),
            "beam_power": rel_l2(out["beam_power"].cpu().numpy(), P.mean(axis=0)),
            "waveform": rel_l2(out["waveform"].cpu().numpy(), w)}
    assert np.allclose(P, np.abs(Zr) ** 2, rtol=1e-10, atol=0)
    print(f"delay doppler {prec} M={M} G={G}: {errs}", flush=True)
    for k, v in errs.items():
        assert v <= tol, (k, v)
    sim.close()


def test_delay_doppler_rejects_bad_sizes():
    from paper_2408_11472_amd import simradar
    print_case("delay doppler errors")
    wl = workloads.tiny(n_gates=24, n_doppler=16, n_fast=16)
    sim = simradar.Simulator(wl.grid, wl.radar, simradar.SIM_PREC_FP32_PHASE64)
    Y = torch.zeros((128, 24), dtype=torch.complex64, device="cuda")
    with pytest.raises(simradar.SimError) as e:
        sim.delay_doppler(Y, burst=64)      # 24 gates: not a power of two
    assert e.value.status == simradar.SIM_ERR_UNSUPPORTED
    sim.close()
    wl = workloads.tiny(n_gates=32, n_doppler=16, n_fast=16)
    sim = simradar.Simulator(wl.grid, wl.radar, simradar.SIM_PREC_FP32_PHASE64)
    Y = torch.zeros((32, 32), dtype=torch.complex64, device="cuda")
    with pytest.raises(simradar.SimError) as e:
        sim.delay_doppler(Y, burst=64)      # fewer pulses than one burst
    assert e.value.status == simradar.SIM_ERR_SHAPE
    with pytest.raises(simradar.SimError) as e:
        sim.delay_doppler(Y, burst=24)
    assert e.value.status == simradar.SIM_ERR_UNSUPPORTED
    sim.close()
