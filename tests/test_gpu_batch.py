"""GPU tests of the batched solver (C ABI ra_batch_solve)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import round_prices, to_device

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


def _batch_instances():
    """Uneven sizes (including n < 64 and ragged tiles) and every m class."""
    out = []
    rng = np.random.default_rng(77)
    for k, (n, m) in enumerate([(37, 4), (64, 8), (1000, 16), (5003, 32), (130, 4), (20000, 8),
                                (777, 32), (4096, 16), (65, 32), (12345, 4), (3000, 8),
                                (50000, 16)]):
        I = synth.random_small(n, m, seed=1000 + k, dtype=np.float32)
        I.T *= (0.2 + 4.8 * rng.random(m)).astype(np.float32)[None, :]
        out.append(I)
    return out


def _problems(ctx, torch, insts):
    import paper_2104_00282_amd as ra
    probs = []
    for I in insts:
        T, w, c, kind = to_device(I, torch)
        probs.append(ra.Problem(ctx, T, w, c, kind, I.R, I.eps))
    return probs


def _with_alpha_fair(insts, seed):
    rng = np.random.default_rng(seed)
    for I in insts:
        sel = rng.random(I.n) < 0.5
        I.kind = np.where(sel, 2, I.kind).astype(np.uint8)
        I.c = np.where(sel, rng.choice([0.0, 0.5, 2.0], I.n), I.c).astype(np.float32)
    return insts


@pytest.mark.parametrize("alpha_fair", [False, True])
def test_batched_pass_matches_oracle(ctx, torch, alpha_fair):
    """Two passes: the first evaluates p0, the second certifies it; the
    returned g(p0) and U(X~(p0)) match the oracle for every problem (also
    with half of the jobs alpha-fair)."""
    import paper_2104_00282_amd as ra
    insts = _batch_instances()
    if alpha_fair:
        insts = _with_alpha_fair(insts, 78)
    probs = _problems(ctx, torch, insts)
    rng = np.random.default_rng(5)
    p0 = [round_prices(0.2 + rng.random(I.m) * 2, np.float32) for I in insts]
    ps, infos, st = ra.batch_solve(probs, p0=p0, tol_rel=0.0, max_evals=2)
    for I, p, pi, inf in zip(insts, p0, ps, infos):
        assert np.array_equal(pi, p)
        d = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
        U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, d.r, d.jobs)
        scale = abs(float(p @ I.R)) + np.abs(d.jobs["v"]).sum()
        assert abs(inf["g"] - d.g) <= 1e-5 * scale, (I.n, I.m, inf["g"], d.g)
        assert abs(inf["U_lb"] - U) <= 1e-5 * (scale + abs(U)), (I.n, I.m, inf["U_lb"], U)
        assert inf["dual_evals"] == 2
    for pr in probs:
        pr.close()


def test_batched_solve_matches_single(ctx, torch):
    """Each problem's batched solve reaches the same quality as its own solve,
    and the certificate holds under the oracle."""
    import paper_2104_00282_amd as ra
    insts = _batch_instances()
    probs = _problems(ctx, torch, insts)
    ps, infos, st = ra.batch_solve(probs, tol_rel=1e-5, max_iter=150)
    for I, pr, p, inf in zip(insts, probs, ps, infos):
        ps1, i1, _ = pr.solve(tol_rel=1e-5, max_iter=150)
        # summation order differs between the batched and the single kernel,
        # so the two trajectories are close but not identical
        assert inf["rel_gap"] <= max(3 * i1["rel_gap"], 1e-5) + 1e-6
        d = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
        U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, d.r, d.jobs)
        scale = abs(d.g) + abs(U)
        assert abs(inf["g"] - d.g) <= 1e-5 * scale
        assert abs(inf["U_lb"] - U) <= 1e-5 * scale
    for pr in probs:
        pr.close()


def test_batched_full_config_sampled(ctx, torch):
    """The 512-instance batch at full size (n log-uniform in [1e3, 1e6], m in
    {4, 8, 16, 32}), solved in the launch configuration the benchmark times;
    the certificates of a sample of instances (the largest among them) are
    re-evaluated by the oracle one by one."""
    import paper_2104_00282_amd as ra
    print("batched full config: generating", flush=True)
    insts = synth.batch_instances()
    probs = _problems(ctx, torch, insts)
    print("batched full config: solving", flush=True)
    ps, infos, st = ra.batch_solve(probs, tol_rel=1e-4, max_iter=80, stall_evals=40)
    # many of these instances have a gap floor above 1e-4 (small n: a job
    # moving between resources shifts a column by a large share), so the
    # check is that every instance ends with a certificate, most of them tight
    gaps = np.array([inf["rel_gap"] for inf in infos])
    assert np.all(np.isfinite(gaps))
    assert np.median(gaps) < 1e-3
    rng = np.random.default_rng(11)
    pick = set(rng.choice(len(insts), 8, replace=False).tolist())
    pick.add(int(np.argmax([I.n for I in insts])))
    for b in sorted(pick):
        I, p, inf = insts[b], ps[b], infos[b]
        print("batched full config: oracle on instance %d (n=%d, m=%d)" % (b, I.n, I.m), flush=True)
        d = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
        U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, d.r, d.jobs)
        scale = abs(d.g) + abs(U)
        assert abs(inf["g"] - d.g) <= 1e-5 * scale
        assert abs(inf["U_lb"] - U) <= 1e-5 * scale
        assert U <= d.g
    for pr in probs:
        pr.close()


def _two_group_instances():
    """24 problems (two interleaved groups of rounds): the uneven set and
    twelve more, among them a single job."""
    more = [(513, 4), (2049, 8), (7001, 16), (300, 32), (1, 4), (15000, 8), (901, 32),
            (4000, 16), (64, 4), (9999, 4), (2500, 8), (30000, 16)]
    return _batch_instances() + [synth.random_small(n, m, seed=3000 + k, dtype=np.float32)
                                 for k, (n, m) in enumerate(more)]


@pytest.mark.parametrize("alpha_fair", [False, True])
def test_batched_two_groups_pass_matches_oracle(ctx, torch, alpha_fair):
    """A batch of 24 runs as two groups whose rounds alternate on the stream:
    g(p0) and U(X~(p0)) of every problem against the oracle."""
    insts = _two_group_instances()
    if alpha_fair:
        insts = _with_alpha_fair(insts, 79)
    probs = _problems(ctx, torch, insts)
    _two_pass_check(probs, insts, 6)
    for pr in probs:
        pr.close()


def test_batched_two_groups_solve(ctx, torch):
    """Two groups solved to 1e-5: every certificate holds under the oracle
    and matches the quality of the problem's own solve; then all problems
    but one stop at once, so that one group runs out of problems while the
    other goes on."""
    import paper_2104_00282_amd as ra
    insts = _two_group_instances()
    probs = _problems(ctx, torch, insts)
    ps, infos, st = ra.batch_solve(probs, tol_rel=1e-5, max_iter=150)
    single = []
    for I, pr, p, inf in zip(insts, probs, ps, infos):
        _, i1, _ = pr.solve(tol_rel=1e-5, max_iter=150)
        single.append(i1)
        assert inf["rel_gap"] <= max(3 * i1["rel_gap"], 1e-5) + 1e-6
        d = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
        assert abs(inf["g"] - d.g) <= 1e-5 * (abs(float(p @ I.R)) + np.abs(d.jobs["v"]).sum())
        # near p* many jobs sit at ties, where the GPU (FP32) and the oracle
        # (FP64) may pick different, equally optimal supports; with a few
        # hundred jobs one such choice moves the column scaling visibly, so
        # the certificate is checked as the utility of the GPU's own scaled
        # allocation (same per-job arithmetic in every kernel), recomputed
        # by the oracle
        out = pr.dual_eval(p, support=True)
        jp = out["j_pair"].cpu().numpy().astype(np.int32)
        xp = out["x_pair"].cpu().numpy().astype(np.float64)
        Gd = {"jlo": jp[:, 0].copy(), "jhi": jp[:, 1].copy(), "xlo": xp[:, 0].copy(),
              "xhi": xp[:, 1].copy()}
        rg = np.zeros(I.m)
        for k in range(2):
            ok = jp[:, k] >= 0
            rg += np.bincount(jp[ok, k], weights=xp[ok, k], minlength=I.m)
        Ug, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, rg, Gd)
        assert abs(inf["U_lb"] - Ug) <= 1e-5 * (abs(d.g) + abs(Ug)), (I.n, I.m, inf["U_lb"], Ug)
    # every problem but the largest stops at its first certificate
    last = int(np.argmax([I.n for I in insts]))
    tol = np.full(len(insts), 1e30)
    tol[last] = 1e-5
    _, inf2, _ = ra.batch_solve(probs, tol_each=tol, max_iter=150)
    for k, inf in enumerate(inf2):
        if k != last:
            assert inf["converged"] == 1 and inf["dual_evals"] <= 2
    assert inf2[last]["dual_evals"] > 5
    assert inf2[last]["rel_gap"] <= max(3 * single[last]["rel_gap"], 1e-5) + 1e-6
    for pr in probs:
        pr.close()


def test_batched_graph_equals_direct(ctx, torch):
    import paper_2104_00282_amd as ra
    insts = _batch_instances()[:6]
    probs = _problems(ctx, torch, insts)
    pa, ia, _ = ra.batch_solve(probs, tol_rel=1e-6, max_iter=30, use_graph=True)
    pb, ib, _ = ra.batch_solve(probs, tol_rel=1e-6, max_iter=30, use_graph=False)
    for x, y, u, v in zip(pa, pb, ia, ib):
        assert np.array_equal(x, y) and u["g"] == v["g"]
    for pr in probs:
        pr.close()


def test_batched_rejects_unsupported(ctx, torch):
    import paper_2104_00282_amd as ra
    probs = _problems(ctx, torch, [synth.random_small(100, 64, seed=1, dtype=np.float32),
                                   synth.random_small(100, 4, seed=2, dtype=np.float32)])
    with pytest.raises(ra.RAError) as e:
        ra.batch_solve(probs)
    assert e.value.status == ra.RA_EUNSUPPORTED
    p64 = _problems(ctx, torch, [synth.random_small(100, 4, seed=3, dtype=np.float64)])
    with pytest.raises(ra.RAError):
        ra.batch_solve(p64)
    for pr in probs + p64:
        pr.close()


def _larger_instances():
    return [synth.random_small(n, m, seed=2000 + k, dtype=np.float32)
            for k, (n, m) in enumerate([(200003, 4), (90001, 16), (60001, 32)])]


def _two_pass_check(probs, insts, seed):
    """Evaluate random prices p0 and certify them (two passes); g(p0) and
    U(X~(p0)) of every problem against the oracle."""
    import paper_2104_00282_amd as ra
    rng = np.random.default_rng(seed)
    p0 = [round_prices(0.2 + rng.random(I.m) * 2, np.float32) for I in insts]
    ps, infos, st = ra.batch_solve(probs, p0=p0, tol_rel=0.0, max_evals=2)
    for I, p, pi, inf in zip(insts, p0, ps, infos):
        assert np.array_equal(pi, p)
        d = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
        U, _ = oracle.lower_bound(I.T, I.w, I.c, I.kind, I.eps, I.R, d.r, d.jobs)
        scale = abs(float(p @ I.R)) + np.abs(d.jobs["v"]).sum()
        assert abs(inf["g"] - d.g) <= 1e-5 * scale, (I.n, I.m, inf["g"], d.g)
        assert abs(inf["U_lb"] - U) <= 1e-5 * (scale + abs(U)), (I.n, I.m, inf["U_lb"], U)


# launch shapes: (tile floats, rows per tile for m = 4, 8, 16, 32, blocks per CU);
# one block per CU with 64-row tiles gives every wave several tiles
SHAPES = [
    (1024, (256, 128, 64, 0), 0),
    (1024, (64, 64, 64, 0), 1),
    (2048, (512, 256, 128, 64), 0),
    (2048, (64, 64, 64, 64), 1),
    (2048, (128, 128, 64, 64), 2),
    (4096, (512, 512, 256, 128), 0),
    (4096, (64, 128, 256, 64), 1),
]


@pytest.mark.parametrize("shape", SHAPES, ids=["tf%d_r%s_b%d" % (s[0], "-".join(map(str, s[1])),
                                                s[2]) for s in SHAPES])
def test_batched_shapes_match_oracle(torch, shape):
    """Every tile budget, tile heights from one to eight jobs per lane, and
    grids of one block per CU: the evaluated and certified values match the
    oracle (also with alpha-fair jobs)."""
    import paper_2104_00282_amd as ra
    tf, rows, bpc = shape
    ctx = ra.Context(0)
    try:
        ctx.set_batch_shape(tf, rows, bpc)
        # with three larger problems every wave gets several tiles
        insts = [I for I in _batch_instances() + _larger_instances()
                 if tf >= 2048 or I.m != 32]
        print("shape %s: %d problems" % (shape, len(insts)), flush=True)
        probs = _problems(ctx, torch, insts)
        _two_pass_check(probs, insts, seed=6)
        for pr in probs:
            pr.close()
        af = _with_alpha_fair([I for I in _batch_instances() if tf >= 2048 or I.m != 32][:5], 79)
        probs = _problems(ctx, torch, af)
        _two_pass_check(probs, af, seed=7)
        for pr in probs:
            pr.close()
        assert ctx.batch_tuning() == {}  # a fixed shape is never tuned
    finally:
        ctx.close()


def test_batched_shape_validation(torch):
    import paper_2104_00282_amd as ra
    ctx = ra.Context(0)
    try:
        for tf, rows in [(3000, (64, 64, 64, 64)), (2048, (100, 64, 64, 64)),
                         (1024, (64, 64, 64, 64)), (2048, (512, 512, 64, 64)),
                         (4096, (1024, 64, 64, 64))]:
            with pytest.raises(ra.RAError) as e:
                ctx.set_batch_shape(tf, rows)
            assert e.value.status == ra.RA_EINVAL
        with pytest.raises(ra.RAError):
            ctx.set_batch_shape(2048, (64, 64, 64, 64), 9)
        # a shape without a tile for m = 32 refuses batches that have such problems
        ctx.set_batch_shape(1024, (256, 128, 64, 0))
        probs = _problems(ctx, torch, [synth.random_small(100, 32, seed=4, dtype=np.float32)])
        with pytest.raises(ra.RAError) as e:
            ra.batch_solve(probs)
        assert e.value.status == ra.RA_EINVAL
        ctx.set_batch_shape(0)
        ra.batch_solve(probs, max_iter=2)
        for pr in probs:
            pr.close()
    finally:
        ctx.close()


def test_batched_tuner_record_and_cache(torch, tmp_path, monkeypatch):
    """The autotuner times tile heights per m class and blocks per CU, records
    its candidates, keeps the fastest whole round, and stores its choice in
    the cache file, from which a new context takes it without tuning."""
    import paper_2104_00282_amd as ra
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("RESALLOC_TUNE_CACHE", str(cache))
    insts = _batch_instances()
    ctx = ra.Context(0)
    try:
        probs = _problems(ctx, torch, insts)
        ra.batch_solve(probs, max_iter=3)
        rec = ctx.batch_tuning()
        cands = rec["candidates"]
        chosen = rec["chosen"]
        for c in cands:
            assert c["ms"] > 0
        per_class = [c for c in cands if c["m"] != 0]
        whole = [c for c in cands if c["m"] == 0]
        # every budget (1024 excluded: the batch has m = 32 problems), every
        # valid height of every class, every block count up to what fits
        assert {c["tile_floats"] for c in cands} == {2048, 4096}
        for tf in (2048, 4096):
            for m in (4, 8, 16, 32):
                hs = sorted(c["rows"] for c in per_class
                            if c["tile_floats"] == tf and c["m"] == m)
                assert hs == [r for r in (64, 128, 256, 512) if r * m <= tf], (tf, m, hs)
        best = min(whole, key=lambda c: c["ms"])
        assert chosen["tile_floats"] == best["tile_floats"]
        assert chosen["rows"] == best["rows"] and chosen["bpc"] == best["bpc"]
        # these classes are too small for a trusted time per job: the split
        # weighs bytes (all costs zero)
        assert chosen["cost_ns_per_job"] == [0, 0, 0, 0]
        line = cache.read_text().split()
        assert len(line) == 11 and int(line[1]) == chosen["tile_floats"]
        assert [int(x) for x in line[2:6]] == chosen["rows"] and int(line[6]) == chosen["bpc"]
        for pr in probs:
            pr.close()
    finally:
        ctx.close()
    ctx2 = ra.Context(0)
    try:
        probs = _problems(ctx2, torch, insts)
        _two_pass_check(probs, insts, seed=8)
        assert ctx2.batch_tuning() == {}  # taken from the cache file
        for pr in probs:
            pr.close()
    finally:
        ctx2.close()


def test_batched_workspace_reuse_across_variants(torch):
    """One context runs batches of different sizes and kernel variants (with
    and without alpha-fair jobs, a larger batch after a smaller one): its
    reused workspace and captured graph give every batch its own variant's
    results, checked against the oracle."""
    import paper_2104_00282_amd as ra
    ctx = ra.Context(0)
    try:
        base = _batch_instances()
        for k, (sel, af) in enumerate([(slice(0, 4), False), (slice(0, 4), True),
                                       (slice(0, 12), False), (slice(2, 7), True),
                                       (slice(0, 12), True)]):
            insts = base[sel]
            if af:
                insts = _with_alpha_fair([synth.random_small(I.n, I.m, seed=3000 + j,
                                                             dtype=np.float32)
                                          for j, I in enumerate(insts)], 80 + k)
            print("workspace reuse: batch %d (%d problems, alpha-fair %s)" % (k, len(insts), af),
                  flush=True)
            probs = _problems(ctx, torch, insts)
            _two_pass_check(probs, insts, seed=20 + k)
            for pr in probs:
                pr.close()
    finally:
        ctx.close()
