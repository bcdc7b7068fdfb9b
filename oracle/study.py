"""Reference-solution comparison of Sec. 6: error norms of a coarse numerical
solution against a reference computed on a grid refined by r in space and
time (r = 16 in the paper).

TEST INFRASTRUCTURE ONLY (part of the oracle).

Sampling (our reading of "mesh resolutions 16 times smaller"): the fine grid
has spacing h/r and step dt/r over the same domain, so coarse node i is fine
node r i and the coarse time t^n = n dt is fine step r n.  A trace row n
holds u^{n+1}, hence coarse trace row n matches fine trace row r (n+1) - 1,
and a coarse snapshot u^n matches the fine u^{r n}.  The point source keeps
its physical scaling (q = dt^2 s / h^d on either grid) and the damping band
its physical width (r nb fine cells, same eta_max).

Norms (Sec. 6.1.1, eqs. snapnorm1, snapnorm2, snapnormmax and their trace
analogues with tau for h):
  snapshot: L1 = sum |e| / h^2, L2 = sqrt(sum e^2) / h, Linf = max |e|
  trace:    L1 = sum |e| / dt,  L2 = sqrt(sum e^2) / dt, Linf = max |e|
(the printed 1/h^2 and 1/h are used as printed, for either dimension count).
"""
from __future__ import annotations

from typing import Dict

import numpy as np


def error_norms(num: np.ndarray, ref: np.ndarray, scale: float) -> Dict[str, float]:
    """L1 = sum|e| / scale^2, L2 = sqrt(sum e^2) / scale, Linf = max|e|."""
    e = np.asarray(num, dtype=np.float64) - np.asarray(ref, dtype=np.float64)
    if e.size == 0:
        return {"l1": 0.0, "l2": 0.0, "linf": 0.0}
    return {"l1": float(np.sum(np.abs(e)) / scale ** 2), "l2": float(np.sqrt(np.sum(e * e)) / scale),
            "linf": float(np.max(np.abs(e)))}


def sample_snapshot(fine: np.ndarray, r: int) -> np.ndarray:
    """Fine field on the coarse nodes (every r-th node along every axis)."""
    sl = tuple(slice(None, None, r) for _ in range(fine.ndim))
    return np.ascontiguousarray(fine[sl])


def sample_traces(fine: np.ndarray, r: int) -> np.ndarray:
    """Fine traces [r nt, nrec] at the coarse trace times: rows r (n+1) - 1."""
    return np.ascontiguousarray(fine[r - 1::r])
