"""FP64 reference of the warm-start network and its features (test
infrastructure only; never imported by the product path).

Network: in_dim -> hidden (ReLU) -> hidden (ReLU) -> out_dim; inputs
standardised with (x_mean, x_std), outputs y = y_s * y_std + y_mean; loss
mean((y_s - t_s)^2) over the batch and outputs with t_s the standardised
targets; flat parameter order W1, b1, W2, b2, W3, b3 (row-major weights of
shape out x in).

Features of a problem: rows floor(k n / S), k < S = min(n, 8192); per
resource j: the 10/50/90 % nearest-rank quantiles (index floor(q (N - 1) +
0.5) of the sorted values) of column j over the log jobs and over the
capped-linear jobs (0 when a kind has no job), R_j / n, log of the column
mean; then 8-bin histograms of w on [0.5, 2] (width 0.1875, clamped) per
kind, as fractions of S.  This is a definition of inputs for a learned
model (not from the paper), so its pins are brute-force sorting and
counting in the tests.
"""
import math

import numpy as np

LOG = 0


def unpack(params, D, H, O):
    p = np.asarray(params, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * D].reshape(H, D); o += H * D
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + O * H].reshape(O, H); o += O * H
    b3 = p[o:o + O]; o += O
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def num_params(D, H, O):
    return H * D + H + H * H + H + O * H + O


def forward(params, D, H, O, norm, X):
    """Returns (Y de-standardised, cache)."""
    xm, xs, ym, ys = [np.asarray(v, dtype=np.float64) for v in norm]
    W1, b1, W2, b2, W3, b3 = unpack(params, D, H, O)
    Xs = (np.asarray(X, dtype=np.float64) - xm) / xs
    Z1 = Xs @ W1.T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2.T + b2
    H2 = np.maximum(Z2, 0.0)
    Ys = H2 @ W3.T + b3
    return Ys * ys + ym, (Xs, Z1, H1, Z2, H2, Ys)


def loss_and_grad(params, D, H, O, norm, X, Ty):
    """MSE of standardised outputs and the flat gradient (FP64 backprop)."""
    xm, xs, ym, ys = [np.asarray(v, dtype=np.float64) for v in norm]
    W1, b1, W2, b2, W3, b3 = unpack(params, D, H, O)
    _, (Xs, Z1, H1, Z2, H2, Ys) = forward(params, D, H, O, norm, X)
    Ts = (np.asarray(Ty, dtype=np.float64) - ym) / ys
    B = Xs.shape[0]
    d = Ys - Ts
    L = float(np.mean(d * d))
    dYs = 2.0 * d / (B * O)
    gW3 = dYs.T @ H2
    gb3 = dYs.sum(0)
    dH2 = dYs @ W3
    dZ2 = dH2 * (Z2 > 0)
    gW2 = dZ2.T @ H1
    gb2 = dZ2.sum(0)
    dH1 = dZ2 @ W2
    dZ1 = dH1 * (Z1 > 0)
    gW1 = dZ1.T @ Xs
    gb1 = dZ1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return L, g


SAMPLE = 8192


def features(T, w, c, kind, R):
    """Feature vector (FP64) of one problem."""
    T = np.asarray(T)
    n, m = T.shape
    S = min(n, SAMPLE)
    rows = (np.arange(S, dtype=np.int64) * n) // S
    Ts = np.asarray(T[rows], dtype=np.float64)
    ks = np.asarray(kind)[rows]
    ws = np.asarray(w, dtype=np.float64)[rows]
    out = np.zeros(8 * m + 16)
    for j in range(m):
        for kk in (0, 1):
            vals = np.sort(Ts[ks == kk, j])
            N = vals.size
            for q, qv in enumerate((0.1, 0.5, 0.9)):
                if N > 0:
                    out[8 * j + 3 * kk + q] = vals[int(math.floor(qv * (N - 1) + 0.5))]
        out[8 * j + 6] = R[j] / n
        out[8 * j + 7] = math.log(max(Ts[:, j].mean(), 1e-30))
    # bins use FP32 arithmetic on the FP32 weights, as stored in the problem
    w32 = np.asarray(w, dtype=np.float32)[rows]
    bins = np.floor((w32 - np.float32(0.5)) / np.float32(0.1875)).astype(np.int64)
    bins = np.clip(bins, 0, 7)
    for kk in (0, 1):
        for b in range(8):
            out[8 * m + 8 * kk + b] = np.count_nonzero((ks == kk) & (bins == b)) / S
    return out
