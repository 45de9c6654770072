"""The decomposition of the surface transform that the GPU column and row
passes use (Sec. II.A surface synthesis), restated with NumPy and checked
against the oracle's fields: the 11 real fields (8 at t, 3 increments over
the pulse pair) come from eight column transforms taken over the columns
kx >= 0 only, one per y-dependence, each row rebuilt with a factor of kx
(1, i kx or -kx^2), the conjugate of the mirror column for kx < 0, the real
part of column 0 and a zero Nyquist column, two real fields per complex row
transform.  A wrong multiplier, factor, pairing or mirror rule fails here
without a GPU."""
import numpy as np
import pytest

import oracle.surface as osurf
from paper_2408_11472_amd import inputs, workloads

# (half plane, kx factor) of the real and imaginary field of each row transform
FAC1, FACIK, FACK2 = 0, 1, 2
PAIRS = [((0, FAC1), (1, FACIK)),    # h + i Dx
         ((2, FAC1), (0, FACIK)),    # Dy + i h_x
         ((3, FAC1), (1, FACK2)),    # h_y + i Dx_x
         ((2, FACIK), (4, FAC1)),    # Dx_y + i Dy_y
         ((5, FAC1), (6, FACIK)),    # dh + i dDx
         ((7, FAC1), None)]          # dDy
NAMES = [("h", "disp_x"), ("disp_y", "h_x"), ("h_y", "dx_x"), ("dx_y", "dy_y"),
         ("dh", "ddisp_x"), ("ddisp_y", None)]


def _half_plane_fields(spec, g, t, dt):
    nx, ny = g.nx, g.ny
    KX, KY = osurf.wavenumbers(g)
    K = np.hypot(KX, KY)
    ik = np.zeros_like(K)
    np.divide(1.0, K, out=ik, where=K > 0)
    w = np.sqrt(g.gravity * K)
    c = np.array(spec, dtype=complex)
    c[0, 0] = 0.0
    c[ny // 2, :] = 0.0
    c[:, nx // 2] = 0.0
    cm = c[(-np.arange(ny)) % ny][:, (-np.arange(nx)) % nx]          # c(-k)
    e0, e1 = np.exp(-1j * w * t), np.exp(-1j * w * (t + dt))
    zeta = 0.5 * (c * e0 + np.conj(cm) * np.conj(e0))
    dzeta = 0.5 * (c * (e1 - e0) + np.conj(cm) * (np.conj(e1) - np.conj(e0)))
    d = 1.0 if g.cwm else 0.0
    spectra = [zeta, d * ik * zeta, 1j * d * KY * ik * zeta, 1j * KY * zeta,
               -d * KY * KY * ik * zeta, dzeta, d * ik * dzeta, 1j * d * KY * ik * dzeta]
    # column transforms (unnormalised inverse along y), columns kx >= 0 only
    half = [np.fft.ifft(s, axis=0)[:, : nx // 2] * ny for s in spectra]
    kx = KX[0, : nx // 2]

    def field_row(src):
        q, fac = src
        H = half[q].copy()
        H[:, 0] = H[:, 0].real                                        # column 0 is real
        if fac == FACIK:
            H = H * (1j * kx)
        elif fac == FACK2:
            H = H * (-kx * kx)
        full = np.zeros((ny, nx), dtype=complex)
        full[:, : nx // 2] = H
        full[:, nx // 2 + 1:] = np.conj(H[:, 1:][:, ::-1])            # column nx - j <- conj(j)
        return full

    out = {}
    for (a, b), (na, nb) in zip(PAIRS, NAMES):
        Z = field_row(a) + (1j * field_row(b) if b is not None else 0.0)
        z = np.fft.ifft(Z, axis=1) * nx
        out[na] = z.real
        if nb is not None:
            out[nb] = z.imag
    return out


@pytest.mark.parametrize("nx,ny", [(16, 16), (16, 8), (32, 16), (8, 32)])
@pytest.mark.parametrize("cwm", [0, 1])
@pytest.mark.parametrize("dt", [1.0 / 18.0e3, 0.2])
def test_half_planes_give_the_oracle_fields(nx, ny, cwm, dt):
    wl = workloads.tiny(nx=nx, ny=ny, spacing=2.0, cwm=cwm, seed=nx * 7 + ny)
    g = wl.grid
    spec = inputs.sea_spectrum(nx, ny, g.dx, g.dy, wl.sea.swh, wl.sea.peak_wavelength,
                               wl.sea.seed)
    t = 0.83
    got = _half_plane_fields(spec, g, t, dt)
    f0 = osurf.fields(spec, g, t)
    f1 = osurf.fields(spec, g, t + dt, names=("h", "disp_x", "disp_y"))
    want = dict(f0)
    want["dh"] = f1["h"] - f0["h"]
    want["ddisp_x"] = f1["disp_x"] - f0["disp_x"]
    want["ddisp_y"] = f1["disp_y"] - f0["disp_y"]
    scale = max(np.max(np.abs(f0["h"])), 1e-300)
    for name, ref in want.items():
        # the oracle's increments difference two evaluations: rounding of h
        np.testing.assert_allclose(got[name], ref, rtol=0,
                                   atol=1e-12 * max(scale, np.max(np.abs(ref))),
                                   err_msg=name)
