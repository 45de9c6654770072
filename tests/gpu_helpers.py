"""Shared helpers of the GPU parity tests."""
from __future__ import annotations

import numpy as np

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
