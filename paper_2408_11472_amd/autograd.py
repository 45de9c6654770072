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


def _stacked(fixed, h, sx, sy):
    """The run's facet sets, every field [n_spec][ny][nx]."""
    f = dict(fixed)
    f["h"], f["sx"], f["sy"] = h, sx, sy
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
        sim.range_doppler_accumulate_run(_stacked(fixed, h, sx, sy), times[:n_spec], 0, T)
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
        sim.range_doppler_accumulate_adjoint_run(_stacked(ctx.fixed, h, sx, sy),
                                                 ctx.times[:n_spec], 0, Tb, (gh, gsx, gsy))
        return gh, gsx, gsy, None, None, None, None


def waveform_loss(h, sx, sy, sim: "simradar.Simulator", fixed, times, target):
    return WaveformLoss.apply(h, sx, sy, sim, fixed, times, target)
