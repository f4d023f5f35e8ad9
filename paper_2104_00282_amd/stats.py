"""Outcome statistics of an allocation (host-side analysis, not the hot path).

The paper reports, for its medium-size example (§6.2), the share of jobs that
use two resources, the share with slack (1^T x_i < 1), and for the
target-priority utility the share of jobs reaching the target throughput,
overall and by priority.  These are computed here from a dense allocation as
returned by Problem.allocation (a device tensor) or any array.
"""
from __future__ import annotations

import numpy as np


def allocation_statistics(T, w, c, kind, X, used_tol=1e-9, slack_tol=1e-6, target_rtol=1e-5):
    """T, X: (n, m); w, c, kind: (n,) (kind 1 = capped linear with cap c)."""
    X = np.asarray(X, dtype=np.float64)
    used = X > used_tol
    out = {"two_resources": float(np.mean(used.sum(1) == 2)),
           "slack": float(np.mean(X.sum(1) < 1.0 - slack_tol))}
    kind = np.asarray(kind)
    cap = kind == 1
    if cap.any():
        t = np.einsum("ij,ij->i", np.asarray(T, dtype=np.float64), X)
        reach = t >= np.asarray(c, dtype=np.float64) * (1.0 - target_rtol)
        w = np.asarray(w)
        out["reach_target"] = float(np.mean(reach[cap]))
        if (cap & (w == 2)).any():
            out["reach_target_w2"] = float(np.mean(reach[cap & (w == 2)]))
        if (cap & (w == 1)).any():
            out["miss_target_w1"] = float(1.0 - np.mean(reach[cap & (w == 1)]))
    return out


def dense_from_support(n, m, j_pair, x_pair):
    """Dense X (n, m) from the per-job support of ra_dual_eval (j_pair: (n, 2)
    resource indices, -1 = unused; x_pair: (n, 2) amounts), on the host."""
    jp = np.asarray(j_pair).astype(np.int64)
    xp = np.asarray(x_pair, dtype=np.float64)
    X = np.zeros((n, m))
    rows = np.arange(n)
    for k in (0, 1):
        sel = jp[:, k] >= 0
        X[rows[sel], jp[sel, k]] = xp[sel, k]
    return X
