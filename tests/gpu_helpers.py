"""Shared helpers of the GPU parity tests."""
from __future__ import annotations

import numpy as np

import oracle.scatter as osc
import oracle.surface as osurf


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (den if den > 0 else 1.0))


def to_torch_facets(fac, dtype, device):
    import torch
    return {k: torch.as_tensor(np.ascontiguousarray(fac[k]), dtype=dtype, device=device)
            for k in osurf.FACET_FIELDS}


def rounded_facets(fac, np_dtype):
    """The facet set as the GPU sees it (rounded to its precision), in float64."""
    return {k: np.asarray(v, dtype=np_dtype).astype(np.float64) for k, v in fac.items()}


def print_case(*parts):
    print("CASE", *parts, flush=True)


def print_precision(config, context, output, value, note=""):
    """One line of the per-output precision table (collected from the test log)."""
    print(f"PRECISION {config} {context} {output} {value:.3e} {note}".rstrip(), flush=True)


def continuous_coordinates(fac, grid, radar, t):
    """The oracle's continuous gate and bin coordinates of every facet, its
    Jacobian and its facing product q (scaled by 1/R): the quantities whose
    integer or sign decisions make the per-facet code."""
    with np.errstate(all="ignore"):
        dx, dy, dz, r, r2 = osc.pulse_pair_ranges(fac, grid, radar, t)
        xi = osc.gate_coordinate(r, radar)
        ub = osc.doppler_cycles(r, r2, radar) * radar.n_doppler
        q = (-fac["sx"] * dx - fac["sy"] * dy + dz) / r
    return xi, ub, np.asarray(fac["jac"], dtype=np.float64), q


def explain_mismatches(code, code_ref, coords, edge_tol, jac_tol, q_tol):
    """Every per-facet code that differs from the oracle's must be explained
    by a decision the oracle takes within a stated distance of its threshold:
    a gate or Doppler-bin edge (edge_tol in gate or bin units, which also
    covers the two ends of the range window), the fold test J > 0 (|J| <
    jac_tol) or the facing test q > 0 (|q| / R < q_tol).  Returns the number
    of mismatches; raises AssertionError naming the first unexplained one."""
    bad = np.argwhere(code != code_ref)
    if bad.size == 0:
        return 0
    xi, ub, jac, q = coords
    idx = tuple(bad.T)
    dg = np.abs(xi[idx] - np.round(xi[idx]))
    db = np.abs((ub[idx] + 0.5) - np.round(ub[idx] + 0.5))
    c, cr = code[idx], code_ref[idx]
    fold = (c == osc.CODE_FOLDED) | (cr == osc.CODE_FOLDED)
    back = (c == osc.CODE_BACKFACING) | (cr == osc.CODE_BACKFACING)
    ok = np.where(fold, np.abs(jac[idx]) < jac_tol,
                  np.where(back, np.abs(q[idx]) < q_tol, np.minimum(dg, db) < edge_tol))
    if not ok.all():
        i = int(np.argmin(ok))
        raise AssertionError(
            f"unexplained index mismatch at {tuple(bad[i])}: code {c[i]} vs oracle {cr[i]}, "
            f"gate edge distance {dg[i]:.3e}, bin edge distance {db[i]:.3e}, "
            f"J {jac[idx][i]:.3e}, q/R {q[idx][i]:.3e}")
    return int(bad.shape[0])


def expected_flips(coords_gpu, coords_ref, illuminated):
    """Expected number of gate or bin flips per update from the measured
    position error: a facet flips when its coordinate error crosses an edge,
    which for coordinates spread uniformly over the edges happens with
    probability |delta| (edges one unit apart)."""
    xi, ub = coords_gpu[0], coords_gpu[1]
    xr, ur = coords_ref[0], coords_ref[1]
    m = illuminated
    d = np.abs(xi[m] - xr[m]) + np.abs(ub[m] - ur[m])
    d = d[np.isfinite(d)]
    return float(np.sum(np.minimum(d, 1.0)))
