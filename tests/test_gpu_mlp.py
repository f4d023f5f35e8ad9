"""GPU tests of the learned warm start: features, network forward/backward
against the FP64 reference, training, save/load and ra_solve_learned."""
import os
import tempfile

import numpy as np
import pytest

import oracle
import synth
from gpu_util import to_device
from oracle import mlp as om

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2104_00282_amd as ra
    c = ra.Context(0)
    yield c
    c.close()


def _problem(ctx, torch, I):
    import paper_2104_00282_amd as ra
    T, w, c, kind = to_device(I, torch)
    return ra.Problem(ctx, T, w, c, kind, I.R, I.eps)


@pytest.mark.parametrize("n,m", [(100, 4), (8192, 16), (50000, 16), (30001, 5)])
def test_features_match_reference(ctx, torch, n, m):
    I = synth.warmstart_instance(n, m=m, seed=4000 + n)
    pr = _problem(ctx, torch, I)
    f = pr.features().cpu().numpy().astype(np.float64)
    ref = om.features(I.T, I.w, I.c, I.kind, I.R)
    idx = np.arange(8 * m + 16)
    per = idx < 8 * m
    exact = ~per | (idx % 8 < 6)  # quantiles and histograms: selections and counts
    assert np.array_equal(f[exact], ref[exact].astype(np.float32).astype(np.float64))
    assert np.allclose(f[per & (idx % 8 == 6)], ref[per & (idx % 8 == 6)], rtol=1e-6)
    assert np.allclose(f[per & (idx % 8 == 7)], ref[per & (idx % 8 == 7)], atol=1e-5)
    pr.close()


def _random_net(ctx, D, H, O, seed):
    import paper_2104_00282_amd as ra
    rng = np.random.default_rng(seed)
    params = (rng.standard_normal(om.num_params(D, H, O)) * np.sqrt(1.0 / H)).astype(np.float32)
    norm = [rng.standard_normal(D).astype(np.float32), (0.5 + rng.random(D)).astype(np.float32),
            rng.standard_normal(O).astype(np.float32), (0.5 + rng.random(O)).astype(np.float32)]
    net = ra.MLP(ctx, D, H, O, seed=1)
    net.set_params(params)
    net.set_normalization(*norm)
    return net, params, norm, rng


@pytest.mark.parametrize("D,H,O,B", [(144, 256, 16, 256), (37, 70, 5, 3), (20, 33, 9, 129)])
def test_forward_and_gradients_match_fp64(ctx, torch, D, H, O, B):
    net, params, norm, rng = _random_net(ctx, D, H, O, seed=D + H + O)
    assert net.num_params() == om.num_params(D, H, O)
    X = rng.standard_normal((B, D)).astype(np.float32) * 2
    Ty = rng.standard_normal((B, O)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Tyd = torch.from_numpy(Ty).cuda()
    Y = net.forward(Xd).cpu().numpy().astype(np.float64)
    Yref, _ = om.forward(params.astype(np.float64), D, H, O, norm, X)
    assert np.linalg.norm(Y - Yref) <= 1e-5 * np.linalg.norm(Yref)
    g, loss = net.gradients(Xd, Tyd)
    Lref, gref = om.loss_and_grad(params.astype(np.float64), D, H, O, norm, X, Ty)
    assert loss == pytest.approx(Lref, rel=1e-5)
    # per tensor relative l2 error
    offs = np.cumsum([0, H * D, H, H * H, H, O * H, O])
    for a, b in zip(offs[:-1], offs[1:]):
        num = np.linalg.norm(g[a:b] - gref[a:b])
        den = np.linalg.norm(gref[a:b])
        assert num <= 1e-4 * max(den, 1e-12), (a, b, num, den)
    net.close()


@pytest.mark.parametrize("H", [256, 33, 6200])
def test_predicted_prices_match_fp64(ctx, torch, H):
    """ra_predict_prices (features, then the single-row forward kernel, or for a
    network whose activations do not fit its LDS budget, H = 6200, the batched
    forward and a copy to the host) against the FP64 network on the same
    feature row."""
    m = 16
    D = 8 * m + 16
    I = synth.warmstart_instance(50000, m=m, seed=777)
    pr = _problem(ctx, torch, I)
    net, params, norm, _ = _random_net(ctx, D, H, m, seed=H)
    f = pr.features().cpu().numpy()
    p = pr.predict_prices(net)
    yref, _ = om.forward(params.astype(np.float64), D, H, m, norm, f[None, :])
    assert np.all(p > 0)
    # FP32 dot products of length H: the rounding of a sum grows like sqrt(H)
    tol = 1e-5 * max(1.0, np.sqrt(H / 256.0))
    assert np.allclose(np.log(p), yref[0], rtol=tol, atol=tol * np.abs(yref).max())
    # the batched forward path gives the same outputs
    yb = net.forward(torch.from_numpy(f[None, :]).cuda()).cpu().numpy()[0]
    assert np.allclose(yb, np.log(p), rtol=1e-5, atol=1e-5 * np.abs(yref).max())
    net.close()
    pr.close()


def test_training_reduces_loss_and_save_load(ctx, torch):
    import paper_2104_00282_amd as ra
    D, H, O, B = 24, 64, 4, 128
    rng = np.random.default_rng(11)
    A = rng.standard_normal((D, O)) / np.sqrt(D)
    X = rng.standard_normal((2048, D)).astype(np.float32)
    Ty = (np.tanh(X @ A) * 2).astype(np.float32)
    net = ra.MLP(ctx, D, H, O, seed=5)
    net.set_normalization(X.mean(0), X.std(0), Ty.mean(0), Ty.std(0))
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(Ty).cuda()
    first = net.gradients(Xd[:B], Td[:B])[1]
    for step in range(400):
        k = (step * B) % 2048
        net.train_step(Xd[k:k + B], Td[k:k + B], 3e-3)
    last = net.gradients(Xd[:B], Td[:B])[1]
    assert last < 0.1 * first
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "net.bin")
        net.save(path)
        net2 = ra.MLP.load(ctx, path)
        assert torch.equal(net.forward(Xd[:50]), net2.forward(Xd[:50]))
        assert np.array_equal(net.get_params(), net2.get_params())
        net2.close()
    net.close()


def test_learned_solve_warm_and_fallback(ctx, torch):
    """A network whose output is exactly log p* (zero weights, bias = log p*)
    reaches the target in fewer passes than a cold start; a wildly wrong one
    is abandoned for a cold restart and still converges."""
    import paper_2104_00282_amd as ra
    m = 8
    I = synth.warmstart_instance(200000, m=m, seed=4242)
    pr = _problem(ctx, torch, I)
    p_star, info, _ = pr.solve(tol_rel=1e-7, max_iter=300, stall_evals=60)
    target = max(1e-6, 1.5 * info["rel_gap"])
    _, cold, _ = pr.solve(tol_rel=target, max_iter=300, stall_evals=60)
    D, H = 8 * m + 16, 32
    net = ra.MLP(ctx, D, H, m, seed=0)
    params = np.zeros(net.num_params(), np.float32)
    params[-m:] = np.log(p_star).astype(np.float32)
    net.set_params(params)
    _, warm, _ = pr.solve_learned(net, tol_rel=target, max_iter=300, stall_evals=60)
    assert warm["restarted"] == 0 and warm["converged"] == 1
    assert warm["dual_evals"] < cold["dual_evals"]
    params[-m:] = 20.0  # prices e^20: nothing is bought
    net.set_params(params)
    _, bad, _ = pr.solve_learned(net, tol_rel=target, max_iter=300, stall_evals=60)
    assert bad["restarted"] == 1 and bad["warm_evals"] >= 3
    assert bad["rel_gap"] <= max(target, 1.5 * cold["rel_gap"])
    wrong = ra.MLP(ctx, 10, 4, m)
    with pytest.raises(ra.RAError):
        pr.solve_learned(wrong)
    net.close()
    wrong.close()
    pr.close()


def test_learned_solve_stall_fallback(ctx, torch):
    """With warm_stall_restarts set, a warm run that stalls short of the
    tolerance (with its own stall window, warm_stall_evals) is followed by
    the cold solve ra_solve would run; the result is the better certified
    point of the two runs, and both runs' passes are counted (and bounded
    together by max_evals)."""
    import paper_2104_00282_amd as ra
    m = 8
    I = synth.warmstart_instance(200000, m=m, seed=4243)
    pr = _problem(ctx, torch, I)
    p_star, _, _ = pr.solve(tol_rel=1e-7, max_iter=300, stall_evals=60)
    net = ra.MLP(ctx, 8 * m + 16, 32, m, seed=0)
    params = np.zeros(net.num_params(), np.float32)
    z = np.random.default_rng(5).standard_normal(m)
    params[-m:] = (np.log(p_star) + 0.1 * z).astype(np.float32)
    net.set_params(params)
    kw = dict(tol_rel=0.0, max_iter=300, stall_evals=10, stall_restarts=1)
    p_w, w, _ = pr.solve_learned(net, **dict(kw, stall_evals=6))  # the warm run alone
    assert w["restarted"] == 0 and w["converged"] == 0
    p_c, c, _ = pr.solve(**kw)
    fb = dict(warm_stall_restarts=1, warm_stall_evals=6)
    p, info, st = pr.solve_learned(net, **fb, **kw)
    assert st == ra.RA_ENOTCONV and info["restarted"] == 2 and info["converged"] == 0
    assert info["warm_evals"] == w["dual_evals"]
    assert info["dual_evals"] == w["dual_evals"] + c["dual_evals"]
    assert info["iters"] == w["iters"] + c["iters"]
    best_p, best = (p_w, w) if w["rel_gap"] <= c["rel_gap"] else (p_c, c)
    assert info["rel_gap"] == best["rel_gap"] and np.array_equal(p, best_p)
    # a warm run that meets the tolerance is not followed by anything
    _, ok, _ = pr.solve_learned(net, **fb, **dict(kw, tol_rel=max(1e-4, 2 * w["rel_gap"])))
    assert ok["restarted"] == 0 and ok["converged"] == 1
    # the pass budget covers both runs
    budget = w["dual_evals"] + 5
    _, capped, _ = pr.solve_learned(net, max_evals=budget, **fb, **kw)
    assert capped["restarted"] == 2 and capped["dual_evals"] <= budget
    with pytest.raises(ra.RAError):
        pr.solve_learned(net, warm_stall_restarts=-2)
    with pytest.raises(ra.RAError):
        pr.solve_learned(net, warm_stall_evals=-1)
    net.close()
    pr.close()
