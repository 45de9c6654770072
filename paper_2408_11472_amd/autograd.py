"""torch.autograd wrapper of the differentiable chain of the HIP library.

WaveformLoss(h, sx, sy) runs, for every update j, the scatterers and their
rasterisation from the facet set (h[j], sx[j], sy[j] plus fixed fields), the
post-processing into IQ and the multi-look waveform loss; its backward runs
the hand-written adjoint kernels (loss -> IQ -> Doppler spectra -> facets),
recomputing every scatterer instead of storing them.  Every step runs in the
HIP library; this module only marshals tensors.
"""
from __future__ import annotations

import torch

from . import simradar

FIXED_FIELDS = ("disp_x", "disp_y", "jac", "ddisp_x", "ddisp_y", "dh")


def _facets(fixed, h, sx, sy, j):
    f = {k: fixed[k][j] for k in FIXED_FIELDS}
    f["h"], f["sx"], f["sy"] = h[j], sx[j], sy[j]
    return f


class WaveformLoss(torch.autograd.Function):
    """L = sum_g (P[g] - target[g])^2 with P the multi-look waveform of the
    run whose update j has facet heights h[j] and slopes sx[j], sy[j]
    (tensors [n_spec, ny, nx]); `fixed` holds the other facet fields with the
    same shape, `times` the first-pulse time of every update."""

    @staticmethod
    def forward(ctx, h, sx, sy, sim, fixed, times, target):
        n_spec = h.shape[0]
        T = sim.empty_spectra(n_spec)
        for j in range(n_spec):
            sim.range_doppler_accumulate(_facets(fixed, h, sx, sy, j), times[j], j, T)
        Y = sim.segments_to_iq(T)
        P, L = sim.waveform_loss(Y, target)
        ctx.save_for_backward(h, sx, sy, Y, P, target)
        ctx.sim, ctx.fixed, ctx.times = sim, fixed, times
        return L

    @staticmethod
    def backward(ctx, gL):
        h, sx, sy, Y, P, target = ctx.saved_tensors
        sim = ctx.sim
        n_spec = h.shape[0]
        scale = gL.detach().reshape(1).to(sim.real_dtype).contiguous()
        Yb = sim.waveform_loss_adjoint(Y, P, target, scale)
        Tb = sim.segments_to_iq_adjoint(Yb, n_spec)
        gh = torch.empty_like(h)
        gsx = torch.empty_like(sx)
        gsy = torch.empty_like(sy)
        for j in range(n_spec):
            sim.range_doppler_accumulate_adjoint(_facets(ctx.fixed, h, sx, sy, j), ctx.times[j],
                                                 j, Tb, out=(gh[j], gsx[j], gsy[j]))
        return gh, gsx, gsy, None, None, None, None


def waveform_loss(h, sx, sy, sim: "simradar.Simulator", fixed, times, target):
    return WaveformLoss.apply(h, sx, sy, sim, fixed, times, target)
