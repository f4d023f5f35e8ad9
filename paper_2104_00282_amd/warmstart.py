"""Training and evaluating the learned warm start (thin driver over the C ABI).

Every numerical step runs in libresalloc.so: instances are solved by the
batched price-discovery loop (ra_batch_solve), features come from
ra_features, the network is trained with ra_mlp_train_step and used through
ra_solve_learned.  This module only moves arrays between those calls.
"""
from __future__ import annotations

import time

import numpy as np

from . import MLP, Problem, batch_solve


def solved_set(ctx, count, n, m, seed0, group=500, tol_rel=1e-6, max_iter=300, stall_evals=60,
               log=None):
    """Generate `count` instances (synth.warmstart_device, seeds seed0 + k),
    solve them with the batched solver and return (features (count, 8m+16),
    log-prices (count, m), relative gaps (count,))."""
    import torch

    import synth

    feats, targets, gaps = [], [], []
    for g0 in range(0, count, group):
        gn = min(group, count - g0)
        probs = []
        for k in range(gn):
            T, w, c, kind, R = synth.warmstart_device(n, m, seed=seed0 + g0 + k)
            probs.append(Problem(ctx, T, w, c, kind, R, 1e-3, validate=False))
        ps, infos, _ = batch_solve(probs, tol_rel=tol_rel, max_iter=max_iter,
                                   stall_evals=stall_evals)
        feats.append(torch.stack([pr.features() for pr in probs]).cpu().numpy())
        targets.append(np.log(np.maximum(np.stack(ps), 1e-8)).astype(np.float32))
        gaps.append(np.array([i["rel_gap"] for i in infos]))
        for pr in probs:
            pr.close()
        del probs
        if log:
            log("solved %d / %d" % (g0 + gn, count))
    return np.concatenate(feats), np.concatenate(targets), np.concatenate(gaps)


def train(ctx, X, Y, hidden=256, epochs=40, batch=256, lr=1e-3, seed=7, val_frac=0.05,
          log=None):
    """Train a network on features X and log-prices Y (numpy, float32).
    Standardisation comes from the training split. Returns (network, dict)."""
    import torch

    N, D = X.shape
    O = Y.shape[1]
    nval = max(1, int(round(val_frac * N))) if N > 20 else 0
    Xt, Yt = X[: N - nval], Y[: N - nval]
    xm, xs = Xt.mean(0), Xt.std(0)
    xs = np.where(xs > 1e-6, xs, 1.0)
    ym, ys = Yt.mean(0), Yt.std(0)
    ys = np.where(ys > 1e-6, ys, 1.0)
    net = MLP(ctx, D, hidden, O, seed=seed)
    net.set_normalization(xm, xs, ym, ys)
    dev = torch.device("cuda")
    Xd = torch.from_numpy(np.ascontiguousarray(Xt)).to(dev)
    Yd = torch.from_numpy(np.ascontiguousarray(Yt)).to(dev)
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    ntr = Xt.shape[0]
    steps = 0
    loss = float("nan")
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(ntr)).to(dev)
        lr_ep = lr * (0.1 ** (ep / max(1, epochs - 1)))
        tot, cnt = 0.0, 0
        for b0 in range(0, ntr - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            tot += net.train_step(Xd[idx], Yd[idx], lr_ep)
            cnt += 1
            steps += 1
        loss = tot / max(cnt, 1)
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log("epoch %d loss %.4f" % (ep, loss))
    out = {"train_loss": loss, "steps": steps, "seconds": time.perf_counter() - t0,
           "n_train": int(ntr), "n_val": int(nval)}
    if nval:
        Xv = torch.from_numpy(np.ascontiguousarray(X[N - nval:])).to(dev)
        Yv = torch.from_numpy(np.ascontiguousarray(Y[N - nval:])).to(dev)
        out["val_loss"] = net.gradients(Xv, Yv)[1]
        out["const_val_loss"] = float(np.mean(((Y[N - nval:] - ym) / ys) ** 2))
    return net, out


def constant_network(ctx, net_like, Y_train):
    """Ablation: a network that always predicts the training mean log-prices."""
    O = Y_train.shape[1]
    D = net_like.in_dim
    const = MLP(ctx, D, 1, O, seed=0)
    const.set_params(np.zeros(const.num_params(), np.float32))
    const.set_normalization(np.zeros(D), np.ones(D), Y_train.mean(0), np.ones(O))
    return const


LEVELS = (1e-3, 1e-4, "floor", "floor_any")


def evaluate(ctx, net, count, n, m, seed0, const_net=None, group=50, floor_iters=300,
             ref_stall_evals=100, stall_evals=30, stall_restarts=5, warm_stall_restarts=2,
             warm_stall_evals=20, max_iter=500, fallback_window=5, levels=LEVELS, near_sigma=0.0,
             log=None):
    """Cold start (p = 1), the paper's data-dependent start and the learned
    warm start (and optionally a constant predictor) on fresh instances, to each
    relative-gap level of `levels` separately ("floor" = max(1e-6, 1.5 x the
    smallest gap a long reference run from p = 1 certifies, the tightest
    target the column-scaling recovery allows on that path; "floor_any" the
    same with the smallest gap of three long reference runs, from p = 1, from
    the paper's start and from the network's prediction, so that no start's
    own path defines the target). Returns a list of per-instance dicts
    {"floor_gap": g, "floor_any_gap": g, level: {arm: info, "target": tol}}.
    The reference runs stop when their best gap has not improved within
    ref_stall_evals passes; the timed arms, all alike, when it has not
    improved within stall_evals passes for the (stall_restarts + 1)-th time,
    the earlier stalls restarting the update from the best certified point;
    the learned solves (warm and const) stall after warm_stall_evals passes
    without improvement, restart warm_stall_restarts times and then, if still
    short of the target, continue with the cold solve (warm_stall_restarts =
    -1: no such fallback).
    near_sigma > 0 adds the arm "near": a start at the p = 1 reference run's
    prices times exp(near_sigma z), z standard normal (seeded per instance),
    closer to p* than any prediction, which shows how much a target tied to
    one start's own path favours that start."""
    import synth

    rows = []
    for g0 in range(0, count, group):
        gn = min(group, count - g0)
        probs = []
        for k in range(gn):
            T, w, c, kind, R = synth.warmstart_device(n, m, seed=seed0 + g0 + k)
            probs.append(Problem(ctx, T, w, c, kind, R, 1e-3, validate=False))
        pref, ref, _ = batch_solve(probs, tol_rel=0.0, max_iter=floor_iters,
                                   stall_evals=ref_stall_evals)
        refs = [ref]
        if "floor_any" in levels:
            _, rp, _ = batch_solve(probs, tol_rel=0.0, max_iter=floor_iters,
                                   stall_evals=ref_stall_evals, paper_init=True)
            # the learned solve's empty-memory step is 0.5 % of max p
            preds = [pr.predict_prices(net) for pr in probs]
            _, rw, _ = batch_solve(probs, p0=preds, tol_rel=0.0, max_iter=floor_iters,
                                   stall_evals=ref_stall_evals, init_step=0.005)
            refs += [rp, rw]
        for k, (pr, rf) in enumerate(zip(probs, ref)):
            pr.solve(max_iter=0)  # capture the evaluation graph outside the timings
            any_gap = min(r[k]["rel_gap"] for r in refs)
            row = {"floor_gap": rf["rel_gap"], "floor_any_gap": any_gap}
            for lv in levels:
                if lv == "floor":
                    tol = max(1e-6, 1.5 * rf["rel_gap"])
                elif lv == "floor_any":
                    tol = max(1e-6, 1.5 * any_gap)
                else:
                    tol = float(lv)
                arms = {}
                kw = dict(tol_rel=tol, max_iter=max_iter, stall_evals=stall_evals,
                          stall_restarts=stall_restarts)
                arms["cold"] = pr.solve(**kw)[1]
                lw = dict(fallback_window=fallback_window, warm_stall_restarts=warm_stall_restarts,
                          warm_stall_evals=warm_stall_evals)
                arms["warm"] = pr.solve_learned(net, **lw, **kw)[1]
                arms["paper"] = pr.solve(paper_init=True, **kw)[1]
                if near_sigma > 0:
                    z = np.random.default_rng(seed0 + g0 + k).standard_normal(m)
                    arms["near"] = pr.solve(p0=np.asarray(pref[k]) * np.exp(near_sigma * z),
                                            init_step=0.005, **kw)[1]
                if const_net is not None:
                    arms["const"] = pr.solve_learned(const_net, **lw, **kw)[1]
                arms["target"] = tol
                row[str(lv)] = arms
            rows.append(row)
        for pr in probs:
            pr.close()
        if log:
            log("evaluated %d / %d" % (g0 + gn, count))
    return rows


def summarize(rows, levels=LEVELS):
    out = {"instances": len(rows),
           "floor_median": float(np.median([r["floor_gap"] for r in rows]))}
    if "floor_any_gap" in rows[0]:
        out["floor_any_median"] = float(np.median([r["floor_any_gap"] for r in rows]))
    for lv in levels:
        key = str(lv)

        def col(arm, k):
            return np.array([r[key][arm][k] for r in rows], dtype=np.float64)

        lvl = {}
        for arm in ("cold", "warm", "paper", "const", "near"):
            if arm not in rows[0][key]:
                continue
            lvl[arm] = {
                "seconds_total": float(col(arm, "seconds").sum()),
                "seconds_median": float(np.median(col(arm, "seconds"))),
                "evals_median": float(np.median(col(arm, "dual_evals"))),
                "evals_mean": float(np.mean(col(arm, "dual_evals"))),
                "reached": int(col(arm, "converged").sum()),
                "restarted": int((col(arm, "restarted") > 0).sum()),
                "stall_fallbacks": int((col(arm, "restarted") == 2).sum()),
            }
        lvl["speedup_total"] = lvl["cold"]["seconds_total"] / lvl["warm"]["seconds_total"]
        lvl["speedup_median"] = float(np.median(col("cold", "seconds") / col("warm", "seconds")))
        lvl["fallback_rate"] = lvl["warm"]["restarted"] / len(rows)
        lvl["stall_fallback_rate"] = lvl["warm"]["stall_fallbacks"] / len(rows)
        lvl["paper_speedup_total"] = lvl["cold"]["seconds_total"] / lvl["paper"]["seconds_total"]
        lvl["warm_vs_paper_total"] = lvl["paper"]["seconds_total"] / lvl["warm"]["seconds_total"]
        if "const" in lvl:
            lvl["const_speedup_total"] = (lvl["cold"]["seconds_total"] /
                                          lvl["const"]["seconds_total"])
        if "near" in lvl:
            lvl["near_speedup_total"] = (lvl["cold"]["seconds_total"] /
                                         lvl["near"]["seconds_total"])
        if lv in ("floor", "floor_any"):
            lvl["targets_at_1e-6"] = int(sum(r[key]["target"] <= 1e-6 for r in rows))
        out[key] = lvl
    return out
