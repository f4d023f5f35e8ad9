"""Helpers shared by the GPU tests: device upload and parity checks against
the oracle (the oracle is only called here, on the test side)."""
import numpy as np

import oracle


def to_device(I, torch, device="cuda"):
    T = torch.from_numpy(np.ascontiguousarray(I.T)).to(device)
    w = torch.from_numpy(np.ascontiguousarray(I.w)).to(device)
    c = torch.from_numpy(np.ascontiguousarray(I.c)).to(device)
    kind = torch.from_numpy(np.ascontiguousarray(I.kind)).to(device)
    return T, w, c, kind


def round_prices(p, dtype):
    """Prices exactly representable in the problem's element type."""
    return np.asarray(p, dtype=dtype).astype(np.float64)


def dense_x(n, m, jlo, jhi, xlo, xhi):
    X = np.zeros((n, m))
    idx = np.arange(n)
    k = jlo >= 0
    np.add.at(X, (idx[k], jlo[k]), xlo[k])
    k = jhi >= 0
    np.add.at(X, (idx[k], jhi[k]), xhi[k])
    return X


def job_values(T, p, kind, w, c, eps, X):
    """Net utility u_i(a_i^T x_i) - p^T x_i of given allocations, in FP64."""
    T = T.astype(np.float64)
    t = np.einsum("ij,ij->i", T, X)
    u = np.where(kind == 0, w * np.log(np.maximum(t + eps, 1e-300)), w * np.minimum(t, c))
    af = kind == 2
    if af.any():
        # alpha-fair with exponent c (c = 1: log)
        e = 1.0 - c[af]
        te = np.maximum(t[af] + eps, 1e-300)
        with np.errstate(divide="ignore", invalid="ignore"):
            ua = np.where(e == 0, w[af] * np.log(te), w[af] * te ** e / np.where(e == 0, 1, e))
        u = u.copy()
        u[af] = ua
    return u - X @ p, t


def keys64(T, p):
    """Efficiency per price a_ij / p_j in FP64 (p_j = 0: +inf for a_ij > 0;
    a_ij = 0: key 0, never chosen)."""
    T = np.asarray(T, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        k = np.where(p[None, :] > 0, T / np.where(p > 0, p, 1.0)[None, :], np.inf)
    return np.where(T > 0, k, 0.0)


def check_first_vertex(T, p, j1, ref_j1, margin, min_clear=0.99, tie_tol=1e-6):
    """First envelope vertex (§4.1: the largest efficiency per price) against
    the exact FP64 argmax: equal wherever the oracle's margin exceeds
    tie_tol; on near-ties the GPU's resource must have an FP64 key within
    tie_tol (relative) of the best.  At least min_clear of the rows must be
    clear, so that the exact comparison is not vacuous.  Returns the number
    of near-tie rows."""
    j1 = np.asarray(j1, dtype=np.int64)
    clear = margin > tie_tol
    assert clear.mean() >= min_clear, "only %.4f of rows are clear of ties" % clear.mean()
    bad = np.nonzero(j1[clear] != ref_j1[clear])[0]
    assert bad.size == 0, "j1 differs from the FP64 argmax on %d clear rows" % bad.size
    nt = np.nonzero(~clear)[0]
    if nt.size:
        K = keys64(T[nt], p)
        kb = K.max(axis=1)
        none = ref_j1[nt] < 0
        assert np.all(j1[nt][none] == -1), "a row with nothing to buy got a first vertex"
        sel = ~none
        jg = j1[nt][sel]
        assert np.all(jg >= 0)
        kg = K[np.nonzero(sel)[0], jg]
        kbs = kb[sel]
        ok = np.where(np.isinf(kbs), np.isinf(kg), kg >= kbs * (1.0 - tie_tol))
        assert np.all(ok), "a near-tie choice is not within %g of the best key" % tie_tol
    return int(nt.size)


# Sums of per-job FP32 terms (each within a few 1e-7 of its magnitude) carry
# an error near 1e-7 times the summed magnitude; relative to the sum itself
# that stays below tol while the terms cancel by less than CANCEL_MAX.
CANCEL_MAX = 50.0


def check_relative(got, want, magnitude, tol, what):
    """|got - want| <= tol |want| (relative to the value itself), or, where
    the summed terms cancel by more than CANCEL_MAX, tol times their
    magnitude."""
    if magnitude <= CANCEL_MAX * abs(want):
        assert abs(got - want) <= tol * abs(want), (what, got, want)
    else:
        assert abs(got - want) <= tol * magnitude, (what, got, want, magnitude)


def _utility64(kind, w, c, eps, t):
    """u_i(t) in FP64 (log, capped linear, alpha-fair with exponent c)."""
    u = np.where(kind == 0, w * np.log(np.maximum(t + eps, 1e-300)), w * np.minimum(t, c))
    af = kind == 2
    if af.any():
        e = 1.0 - c[af]
        te = np.maximum(t[af] + eps, 1e-300)
        with np.errstate(divide="ignore", invalid="ignore"):
            u[af] = np.where(e == 0, w[af] * np.log(te), w[af] * te ** e / np.where(e == 0, 1, e))
    return u


class Pairs:
    """A per-job allocation with at most two nonzero shares (§4.1), kept as
    index / share pairs (index -1: unused) instead of a dense n x m matrix."""

    def __init__(self, jlo, jhi, xlo, xhi):
        self.j = np.stack([np.asarray(jlo, np.int64), np.asarray(jhi, np.int64)], 1)
        self.x = np.stack([np.asarray(xlo, np.float64), np.asarray(xhi, np.float64)], 1)
        self.x = np.where(self.j >= 0, self.x, 0.0)
        self.j = np.where(self.x != 0, self.j, -1)

    def share(self, rows, idx):
        """x_{i, idx_i} for each row i in rows (0 where idx_i = -1)."""
        jj, xx = self.j[rows], self.x[rows]
        return np.where((jj == idx[:, None]) & (idx[:, None] >= 0), xx, 0.0).sum(1)

    def colsum(self, m, scale=None):
        r = np.zeros(m)
        for k in range(2):
            ok = self.j[:, k] >= 0
            r += np.bincount(self.j[ok, k], weights=self.x[ok, k], minlength=m)
        return r

    def throughput(self, T, s=None):
        """t_i = a_i^T x_i, or a_i^T diag(s) x_i."""
        rows = np.arange(len(self.j))
        t = np.zeros(len(self.j))
        for k in range(2):
            jj = np.maximum(self.j[:, k], 0)
            a = T[rows, jj].astype(np.float64)
            f = s[jj] if s is not None else 1.0
            t += np.where(self.j[:, k] >= 0, a * f * self.x[:, k], 0.0)
        return t

    def dense(self, rows, m):
        X = np.zeros((len(rows), m))
        for k in range(2):
            ok = self.j[rows, k] >= 0
            np.add.at(X, (np.nonzero(ok)[0], self.j[rows, k][ok]), self.x[rows, k][ok])
        return X


def clear_of_ties(J, margin=1e-6):
    """Jobs whose optimum is clear of ties (R14): the oracle's first-vertex
    margin and its allocation margin (how far the best allocation's value is
    from that of any different candidate) both above `margin`."""
    return (J["margin1"] > margin) & (J["marginx"] > margin)


def check_clear_allocations(J, jp, xp, tol):
    """Every job clear of ties has the oracle's allocation: each share of
    either support within tol (abs), whatever the order of the two ends.
    jp, xp: the GPU's (n, 2) support and shares.  Returns the clear share."""
    clear = clear_of_ties(J)
    rows = np.nonzero(clear)[0]
    G = Pairs(jp[rows, 0], jp[rows, 1], xp[rows, 0], xp[rows, 1])
    O = Pairs(J["jlo"][rows], J["jhi"][rows], J["xlo"][rows], J["xhi"][rows])
    loc = np.arange(rows.size)
    dx = np.zeros(rows.size)
    for src in (G, O):
        for k in range(2):
            idx = src.j[:, k]
            dx = np.maximum(dx, np.abs(G.share(loc, idx) - O.share(loc, idx)))
    bad = np.nonzero(dx > tol)[0]
    assert bad.size == 0, ("%d jobs clear of ties have another allocation than the oracle's "
                           "(first: job %d)" % (bad.size, rows[bad[0]]))
    return float(clear.mean())


def compare_dual(I, p, out, tol, max_mismatch_frac=1e-3, min_clear=0.99, ref=None):
    """Element-by-element parity of one GPU dual evaluation with the oracle.

    - j1 equal to the exact (FP64) argmax of a_ij / p_j wherever the oracle's
      efficiency-per-price margin exceeds 1e-6 (at least min_clear of the
      jobs), and within 1e-6 of the best key on the near-ties;
    - per-job allocation equal (abs tol) on every job clear of ties (the
      oracle's first-vertex margin and allocation margin both above 1e-6);
      elsewhere it may differ, but must be feasible and optimal to within
      tol, on at most max_mismatch_frac of the jobs;
    - r equal to the oracle's r with the GPU's near-tie choices substituted;
    - g and U(X~) equal to relative tol (check_relative).
    ref: the oracle's per-job evaluation at p, if already computed.
    Returns a dict of diagnostics, among them how many j1 differ from the
    argmax decided in the data's own precision (a diagnostic only)."""
    n, m = I.T.shape
    if ref is None:
        ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
    J = ref.jobs
    j1 = out["j1"].cpu().numpy().astype(np.int64)
    near = check_first_vertex(I.T, p, j1, J["j1"], J["margin1"], min_clear=min_clear)
    mirror = None
    if n <= 2_000_000:
        mirror = int(np.count_nonzero(j1 != oracle.first_vertex(I.T, p)))

    jp = out["j_pair"].cpu().numpy().astype(np.int64)
    xp = out["x_pair"].cpu().numpy().astype(np.float64)
    G = Pairs(jp[:, 0], jp[:, 1], xp[:, 0], xp[:, 1])
    O = Pairs(J["jlo"], J["jhi"], J["xlo"], J["xhi"])
    assert np.all(G.x >= 0) and np.all(G.x.sum(1) <= 1 + 1e-5)
    assert not np.any((G.j[:, 0] >= 0) & (G.j[:, 0] == G.j[:, 1]))
    rows = np.arange(n)
    dx = np.zeros(n)
    for src in (G, O):
        for k in range(2):
            idx = src.j[:, k]
            dx = np.maximum(dx, np.abs(G.share(rows, idx) - O.share(rows, idx)))
    mism = np.nonzero(dx > tol)[0]
    clear_x = clear_of_ties(J)
    bad = mism[clear_x[mism]]
    assert bad.size == 0, ("%d jobs clear of ties have another allocation than the oracle's "
                           "(first: job %d)" % (bad.size, bad[0]))
    if mism.size:
        Xg = G.dense(mism, m)
        vg, _ = job_values(I.T[mism], p, I.kind[mism], I.w[mism].astype(np.float64),
                           I.c[mism].astype(np.float64), I.eps, Xg)
        vo = J["v"][mism]
        slack = tol * np.maximum(1.0, np.abs(vo))
        assert np.all(vg >= vo - slack), "GPU allocation suboptimal on mismatched jobs"
    assert mism.size <= max(2, max_mismatch_frac * n), "%d of %d jobs differ" % (mism.size, n)

    rg = G.colsum(m)
    r_sub = O.colsum(m)
    if mism.size:
        r_sub = r_sub + G.dense(mism, m).sum(0) - O.dense(mism, m).sum(0)
    r_gpu = out["r"]
    scale_r = np.maximum(np.maximum(I.R, np.abs(r_sub)), 1.0)
    assert np.all(np.abs(r_gpu - r_sub) <= tol * scale_r), (r_gpu, r_sub)
    # the reported r is the sum of the reported per-job allocations
    assert np.all(np.abs(r_gpu - rg) <= 1e-6 * scale_r)

    scale_g = abs(float(p @ I.R)) + np.abs(J["v"]).sum()
    check_relative(out["g"], ref.g, scale_g, tol, "g")
    if "lower_bound" in out:
        # rounding of the bound scales with the summed terms: the utilities at
        # the scaled allocation (steep for alpha-fair exponents > 1 when the
        # scales cut throughput) as well as at the unscaled one
        s = np.where(rg > I.R, I.R / np.maximum(rg, 1e-300), 1.0)
        w64, c64 = I.w.astype(np.float64), I.c.astype(np.float64)
        uabs = (np.abs(_utility64(I.kind, w64, c64, I.eps, J["t"])).sum()
                + np.abs(_utility64(I.kind, w64, c64, I.eps, G.throughput(I.T, s))).sum())
        # recovery of the GPU's own allocation, recomputed by the oracle
        Gd = {"jlo": jp[:, 0].astype(np.int32), "jhi": jp[:, 1].astype(np.int32),
              "xlo": xp[:, 0].copy(), "xhi": xp[:, 1].copy()}
        Ug, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, rg, Gd)
        check_relative(out["lower_bound"], Ug, uabs, tol, "U(X~)")
        if mism.size == 0:
            U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, ref.r, J)
            check_relative(out["lower_bound"], U, uabs, tol, "U(X~)")
    return {"mismatched": int(mism.size), "clear_of_ties": float(clear_x.mean()),
            "g": out["g"], "g_ref": ref.g,
            "j1_near_ties": near, "j1_vs_element_type_argmax": mirror}
