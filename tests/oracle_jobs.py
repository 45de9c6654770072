"""Oracle evaluations run in worker processes, so that the tests at the full
workload sizes finish in test time (each spectrum of the oracle is
independent of the others: Algorithm 1 regenerates the surface at every
update).  Every function here only calls the oracle."""
from __future__ import annotations

import multiprocessing
import os
from concurrent.futures import ProcessPoolExecutor

import oracle.adjoint as oad
import oracle.scatter as osc
import oracle.surface as osurf


def workers(n_jobs: int) -> int:
    """Worker count: one per job, at most the CPU share of one GPU (16) and
    the host's cores."""
    return max(1, min(n_jobs, 16, os.cpu_count() or 1))


def pool(n_jobs: int) -> ProcessPoolExecutor:
    """A pool of fresh interpreters (spawned, so that no GPU state of the
    parent is inherited)."""
    return ProcessPoolExecutor(max_workers=workers(n_jobs),
                               mp_context=multiprocessing.get_context("spawn"))


def spectrum_update(spec0, grid, radar, t, keep_facets=False, keep_codes=False):
    """Surface at the pulse pair (t, t + 1/PRF), scatterers and rasterize:
    (T_fast[j], facets or None, codes or None)."""
    fac = osurf.facets(spec0, grid, t, 1.0 / radar.prf_hz)
    code, c = osc.scatterers(fac, grid, radar, t)
    T = osc.rasterize(code, c, radar)
    return T, (fac if keep_facets else None), (code if keep_codes else None)


def accumulate(fac, grid, radar, t):
    """T_fast[j] of a given facet set."""
    return osc.accumulate(fac, grid, radar, t)[0]


def facet_gradients(fac, grid, radar, t, tbar_j):
    return oad.facet_gradients(fac, grid, radar, t, tbar_j)
