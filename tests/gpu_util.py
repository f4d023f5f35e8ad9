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


def compare_dual(I, p, out, tol, max_mismatch_frac=1e-3):
    """Element-by-element parity of one GPU dual evaluation with the oracle.

    - j1 equal wherever the oracle's efficiency-per-price margin exceeds 1e-6;
    - per-job allocation equal (abs tol) except for near-ties, where the
      GPU's allocation must be feasible and optimal to within tol;
    - r equal to the oracle's r with the GPU's near-tie choices substituted;
    - g and U(X~) equal to relative tol (scaled by the magnitude of the sums).
    Returns a dict of diagnostics."""
    n, m = I.T.shape
    ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
    J = ref.jobs
    j1 = out["j1"].cpu().numpy().astype(np.int64)
    # an index decided by floating point: bit-exact against the oracle's
    # decision in the data's own precision ...
    j1k = oracle.first_vertex(I.T, p)
    bad_j1 = np.nonzero(j1 != j1k)[0]
    assert bad_j1.size == 0, "j1 differs on %d jobs, e.g. %s" % (bad_j1.size, bad_j1[:5])
    # ... which is the exact (FP64) argmax wherever that is not a near-tie
    clear = J["margin1"] > 1e-6
    assert np.array_equal(j1k[clear], J["j1"][clear])

    jp = out["j_pair"].cpu().numpy().astype(np.int64)
    xp = out["x_pair"].cpu().numpy().astype(np.float64)
    Xg = dense_x(n, m, jp[:, 0], jp[:, 1], xp[:, 0], xp[:, 1])
    Xo = dense_x(n, m, J["jlo"], J["jhi"], J["xlo"], J["xhi"])
    assert np.all(Xg >= 0) and np.all(Xg.sum(1) <= 1 + 1e-5)
    assert np.all((Xg > 0).sum(1) <= 2)
    dx = np.abs(Xg - Xo).max(1)
    mism = np.nonzero(dx > tol)[0]
    if mism.size:
        vg, _ = job_values(I.T[mism], p, I.kind[mism], I.w[mism].astype(np.float64),
                           I.c[mism].astype(np.float64), I.eps, Xg[mism])
        vo = J["v"][mism]
        slack = tol * np.maximum(1.0, np.abs(vo))
        assert np.all(vg >= vo - slack), "GPU allocation suboptimal on mismatched jobs"
    assert mism.size <= max(2, max_mismatch_frac * n), "%d of %d jobs differ" % (mism.size, n)

    r_sub = Xo.sum(0) + (Xg[mism] - Xo[mism]).sum(0)
    r_gpu = out["r"]
    scale_r = np.maximum(np.maximum(I.R, np.abs(r_sub)), 1.0)
    assert np.all(np.abs(r_gpu - r_sub) <= tol * scale_r), (r_gpu, r_sub)
    # the reported r is the sum of the reported per-job allocations
    assert np.all(np.abs(r_gpu - Xg.sum(0)) <= 1e-6 * scale_r)

    scale_g = abs(float(p @ I.R)) + np.abs(J["v"]).sum()
    assert abs(out["g"] - ref.g) <= tol * scale_g, (out["g"], ref.g)
    if "lower_bound" in out:
        # rounding of the bound scales with the summed terms: the utilities at
        # the scaled allocation (steep for alpha-fair exponents > 1 when the
        # scales cut throughput) as well as at the unscaled one
        rg = Xg.sum(0)
        s = np.where(rg > I.R, I.R / np.maximum(rg, 1e-300), 1.0)
        uabs = sum(np.abs(job_values(I.T, np.zeros(m), I.kind, I.w.astype(np.float64),
                                     I.c.astype(np.float64), I.eps, X)[0]).sum()
                   for X in (Xo, Xg * s[None, :]))
        # recovery of the GPU's own allocation, recomputed by the oracle
        G = {"jlo": jp[:, 0].astype(np.int32), "jhi": jp[:, 1].astype(np.int32),
             "xlo": xp[:, 0].copy(), "xhi": xp[:, 1].copy()}
        Ug, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, Xg.sum(0), G)
        assert abs(out["lower_bound"] - Ug) <= tol * (uabs + scale_g), (out["lower_bound"], Ug)
        if mism.size == 0:
            U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, ref.r, J)
            assert abs(out["lower_bound"] - U) <= tol * (uabs + scale_g), (out["lower_bound"], U)
    return {"mismatched": int(mism.size), "g": out["g"], "g_ref": ref.g}
