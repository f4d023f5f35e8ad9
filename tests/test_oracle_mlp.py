"""Pins of the FP64 warm-start network and feature reference (oracle/mlp.py)."""
import math

import numpy as np

from oracle import mlp as om


def _net(seed, D=7, H=5, O=3):
    rng = np.random.default_rng(seed)
    params = rng.standard_normal(om.num_params(D, H, O)) * 0.5
    norm = (rng.standard_normal(D), 0.5 + rng.random(D), rng.standard_normal(O), 0.5 + rng.random(O))
    return params, norm, rng


def test_gradient_matches_finite_differences():
    D, H, O, B = 7, 5, 3, 4
    params, norm, rng = _net(1, D, H, O)
    X = rng.standard_normal((B, D)) * 2
    Ty = rng.standard_normal((B, O))
    L, g = om.loss_and_grad(params, D, H, O, norm, X, Ty)
    h = 1e-6
    for k in range(params.size):
        e = np.zeros_like(params)
        e[k] = h
        Lp, _ = om.loss_and_grad(params + e, D, H, O, norm, X, Ty)
        Lm, _ = om.loss_and_grad(params - e, D, H, O, norm, X, Ty)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_zero_weights_output_is_bias():
    D, H, O = 4, 6, 2
    params = np.zeros(om.num_params(D, H, O))
    params[-O:] = [0.5, -1.0]
    norm = (np.zeros(D), np.ones(D), np.array([2.0, 3.0]), np.array([4.0, 0.5]))
    Y, _ = om.forward(params, D, H, O, norm, np.ones((3, D)))
    assert np.allclose(Y, [[2.0 + 0.5 * 4.0, 3.0 - 1.0 * 0.5]] * 3)


def test_loss_is_mean_squared_standardised_error():
    D, H, O = 3, 4, 2
    params, norm, rng = _net(2, D, H, O)
    X = rng.standard_normal((5, D))
    Y, _ = om.forward(params, D, H, O, norm, X)
    Ty = Y + rng.standard_normal(Y.shape) * norm[3]
    L, _ = om.loss_and_grad(params, D, H, O, norm, X, Ty)
    assert L == np.mean(((Y - Ty) / norm[3]) ** 2).item() or math.isclose(
        L, np.mean(((Y - Ty) / norm[3]) ** 2), rel_tol=1e-12)


def _brute_features(T, w, kind, R):
    n, m = len(T), len(T[0])
    S = min(n, 8192)
    rows = [k * n // S for k in range(S)]
    out = []
    for j in range(m):
        for kk in (0, 1):
            vals = sorted(float(T[i][j]) for i in rows if kind[i] == kk)
            for q in (0.1, 0.5, 0.9):
                out.append(vals[int(math.floor(q * (len(vals) - 1) + 0.5))] if vals else 0.0)
        out.append(R[j] / n)
        out.append(math.log(sum(float(T[i][j]) for i in rows) / S))
    for kk in (0, 1):
        counts = [0] * 8
        for i in rows:
            if kind[i] == kk:
                b = int(math.floor((np.float32(w[i]) - np.float32(0.5)) / np.float32(0.1875)))
                counts[min(7, max(0, b))] += 1
        out += [cnt / S for cnt in counts]
    return np.array(out)


def test_features_brute_force():
    rng = np.random.default_rng(3)
    for n, m in ((50, 3), (9000, 2), (20000, 4)):
        T = rng.random((n, m)).astype(np.float32) * 3
        kind = (rng.random(n) < 0.4).astype(np.uint8)
        w = (0.3 + 2.0 * rng.random(n)).astype(np.float32)  # some weights outside [0.5, 2]
        R = rng.random(m) * n
        f = om.features(T, w, np.zeros(n, np.float32), kind, R)
        b = _brute_features(T.tolist(), w.tolist(), kind.tolist(), R)
        assert np.allclose(f, b, rtol=0, atol=1e-12)


def test_features_one_kind_only_and_quantile_definition():
    T = np.arange(1, 12, dtype=np.float32).reshape(11, 1)
    kind = np.zeros(11, np.uint8)
    f = om.features(T, np.ones(11, np.float32), np.zeros(11, np.float32), kind, np.array([5.5]))
    # sorted 1..11, N = 11: indices floor(0.1*10+.5)=1, 5, floor(9.5)=9
    assert list(f[:3]) == [2.0, 6.0, 10.0]
    assert list(f[3:6]) == [0.0, 0.0, 0.0]  # no capped-linear job
    assert f[6] == 0.5 and math.isclose(f[7], math.log(6.0))
    assert f[8 + 2] == 1.0  # every w = 1 falls in bin floor(0.5/0.1875) = 2
