"""GPU parity of the dual evaluation (C ABI ra_dual_eval) with the FP64 oracle.

Tolerance: relative 1e-5 for FP32 problems (the kernel computes per job in
FP32 and sums in FP64), 1e-9 for FP64 problems.  Argmax (first envelope
vertex) exact wherever the oracle's efficiency-per-price margin exceeds 1e-6.
"""
import numpy as np
import pytest

import synth
from gpu_util import compare_dual, round_prices, to_device

pytestmark = pytest.mark.gpu

TOL32 = 1e-5
TOL64 = 1e-9


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a HIP device"
    return t


@pytest.fixture(scope="module")
def ctx(torch):
    import paper_2104_00282_amd as ra
    c = ra.Context(0)
    yield c
    c.close()


def _problem(ctx, torch, I, **kw):
    import paper_2104_00282_amd as ra
    T, w, c, kind = to_device(I, torch)
    return ra.Problem(ctx, T, w, c, kind, I.R, I.eps, **kw)


def _run(ctx, torch, I, p, tol):
    prob = _problem(ctx, torch, I)
    p = round_prices(p, I.T.dtype)
    out = prob.dual_eval(p, lower_bound=True, support=True, j1=True)
    info = compare_dual(I, p, out, tol)
    prob.close()
    return info


# several blocks and a ragged last tile; every wave gets at most one tile at
# this size (the grid asks for one wave per tile up to its occupancy cap), so
# the carry of prefetched tiles and deferred stores from one tile to the next
# is covered by test_vectorised_several_tiles_per_wave
N_SMALL = 64 * 4 * 5 + 37

# The vectorised kernels launch at most 8 blocks of 4 waves per CU (2048
# threads per CU): with n above 2 x 64 x 32 x CUs every wave takes at least
# two 64-job tiles, whatever the kernel's occupancy.
def _n_two_tiles_per_wave(torch):
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    return 2 * 64 * 32 * cus


@pytest.mark.parametrize("m", [4, 8, 16, 32, 64])
def test_vectorised_classes(ctx, torch, m):
    print("vectorised m=%d" % m, flush=True)
    I = synth.random_small(N_SMALL, m, seed=100 + m, dtype=np.float32)
    rng = np.random.default_rng(m)
    for p in (np.ones(m), 0.2 + rng.random(m) * 3):
        _run(ctx, torch, I, p, TOL32)


@pytest.mark.parametrize("m", [4, 8, 16, 32])
def test_vectorised_several_tiles_per_wave(ctx, torch, m):
    """Every job compared with the oracle at a size where each wave of the
    vectorised kernel solves two or more tiles (prefetch of the next tile,
    per-job outputs stored one tile late) and the last tile is ragged."""
    n = _n_two_tiles_per_wave(torch) + 37
    print("vectorised m=%d n=%d" % (m, n), flush=True)
    I = synth.random_small(n, m, seed=150 + m, dtype=np.float32)
    p = 0.2 + np.random.default_rng(150 + m).random(m) * 3
    _run(ctx, torch, I, p, TOL32)


@pytest.mark.parametrize("m", [1, 3, 5, 17, 100, 256])
def test_generic_m(ctx, torch, m):
    print("generic m=%d" % m, flush=True)
    I = synth.random_small(777, m, seed=200 + m, dtype=np.float32)
    p = 0.2 + np.random.default_rng(m).random(m) * 3
    _run(ctx, torch, I, p, TOL32)


@pytest.mark.parametrize("m", [4, 7])
def test_fp64(ctx, torch, m):
    print("fp64 m=%d" % m, flush=True)
    I = synth.random_small(N_SMALL, m, seed=300 + m, dtype=np.float64)
    p = 0.2 + np.random.default_rng(m).random(m) * 3
    _run(ctx, torch, I, p, TOL64)


def test_small_log_config_fp64(ctx, torch):
    I = synth.small_log()
    rng = np.random.default_rng(5)
    for p in (np.ones(4), 5 + 10 * rng.random(4)):
        _run(ctx, torch, I, p, TOL64)


def test_zero_entries_and_zero_prices(ctx, torch):
    print("zeros", flush=True)
    for m in (4, 16, 64, 5):
        I = synth.random_small(N_SMALL, m, seed=400 + m, dtype=np.float32, zero_frac=0.3)
        I.T[::17] = 0.0  # some all-zero rows
        p = 0.2 + np.random.default_rng(m).random(m) * 3
        p[::3] = 0.0
        # free resources make the allocation non-unique: every differing job
        # is checked for optimality instead
        prob = _problem(ctx, torch, I)
        p = round_prices(p, np.float32)
        out = prob.dual_eval(p, lower_bound=True, support=True, j1=True)
        compare_dual(I, p, out, TOL32, max_mismatch_frac=1.0, min_clear=0.0)
        prob.close()


def test_single_job_single_resource(ctx, torch):
    for m in (1, 4):
        I = synth.random_small(1, m, seed=500 + m, dtype=np.float32)
        _run(ctx, torch, I, np.full(m, 0.7), TOL32)


def test_misaligned_T_uses_generic_path(ctx, torch):
    import paper_2104_00282_amd as ra
    I = synth.random_small(N_SMALL, 16, seed=600, dtype=np.float32)
    T, w, c, kind = to_device(I, torch)
    big = torch.empty(T.numel() + 1, dtype=T.dtype, device=T.device)
    big[1:] = T.reshape(-1)
    Tm = big[1:].view(T.shape)  # 4-byte offset: not 16-byte aligned
    assert Tm.data_ptr() % 16 != 0
    prob = ra.Problem(ctx, Tm, w, c, kind, I.R, I.eps)
    p = round_prices(0.3 + np.arange(16) / 10, np.float32)
    out = prob.dual_eval(p, lower_bound=True, support=True, j1=True)
    compare_dual(I, p, out, TOL32)
    prob.close()


def test_exact_ties(ctx, torch):
    """Identical rows and repeated prices: many exact ties; the GPU's choices
    must be optimal and r must add up."""
    m = 8
    n = 2000
    rng = np.random.default_rng(7)
    base = rng.random((5, m)).astype(np.float32)
    I = synth.random_small(n, m, seed=700, dtype=np.float32)
    I.T[:] = base[rng.integers(0, 5, n)]
    I.T[:, 3] = I.T[:, 1]  # duplicate columns
    p = np.array([1, 2, 1, 2, 0.5, 0.5, 3, 3], dtype=np.float64)
    _run_ties = _problem(ctx, torch, I)
    out = _run_ties.dual_eval(p, lower_bound=True, support=True, j1=True)
    compare_dual(I, p, out, TOL32, max_mismatch_frac=1.0, min_clear=0.0)
    _run_ties.close()


def test_mixed16_full_size(ctx, torch):
    """The mixed-16 workload at full size (n = 1e6, m = 16) at two price
    vectors, every job compared with the oracle."""
    print("mixed-16 full size", flush=True)
    I = synth.mixed_16()
    for p in (np.ones(16), np.linspace(0.05, 0.4, 16)):
        _run(ctx, torch, I, p, TOL32)


def test_roofline64_full_size(ctx, torch):
    """The roofline workload (n = 1e7, m = 64) in the launch configuration
    the benchmark times, every job compared with the oracle: j1, the support
    and shares of all 1e7 jobs, r, g and U(X~) (relative 1e-5)."""
    print("roofline-64 full size: generating", flush=True)
    I = synth.roofline_64()
    prob = _problem(ctx, torch, I, validate=False)
    p = round_prices(np.full(64, 0.12), np.float32)
    print("roofline-64: evaluating", flush=True)
    out = prob.dual_eval(p, lower_bound=True, support=True, j1=True)
    prob.close()
    print("roofline-64: oracle over all rows", flush=True)
    info = compare_dual(I, p, out, TOL32)
    print("roofline-64:", info, flush=True)


def test_deterministic(ctx, torch):
    I = synth.random_small(50000, 16, seed=800, dtype=np.float32)
    prob = _problem(ctx, torch, I)
    p = round_prices(0.3 + np.arange(16) / 20, np.float32)
    a = prob.dual_eval(p, lower_bound=True, support=True)
    b = prob.dual_eval(p, lower_bound=True, support=True)
    assert a["g"] == b["g"] and np.array_equal(a["grad"], b["grad"])
    assert a["lower_bound"] == b["lower_bound"]
    assert torch.equal(a["x_pair"], b["x_pair"]) and torch.equal(a["j_pair"], b["j_pair"])


def test_invalid_inputs_rejected(ctx, torch):
    import paper_2104_00282_amd as ra
    I = synth.random_small(100, 4, seed=900, dtype=np.float32)
    T, w, c, kind = to_device(I, torch)
    Tb = T.clone()
    Tb[3, 2] = -1.0
    with pytest.raises(ra.RAError) as e:
        ra.Problem(ctx, Tb, w, c, kind, I.R, I.eps)
    assert e.value.status == ra.RA_EINVAL
    with pytest.raises(ra.RAError):
        ra.Problem(ctx, T, w, c, kind, -I.R, I.eps)
    prob = ra.Problem(ctx, T, w, c, kind, I.R, I.eps)
    with pytest.raises(ra.RAError) as e:
        prob.dual_eval(np.array([1.0, -1.0, 1.0, 1.0]))
    assert e.value.status == ra.RA_EINVAL
    with pytest.raises(ra.RAError):
        prob.dual_eval(np.array([1.0, np.nan, 1.0, 1.0]))


def _with_alpha_fair(I, seed, frac=0.5):
    """Half of the jobs become alpha-fair with exponents in {0, 0.5, 2, 3}
    (linear, power, and the two negative-power cases)."""
    rng = np.random.default_rng(seed)
    sel = rng.random(I.n) < frac
    I.kind = np.where(sel, 2, I.kind).astype(np.uint8)
    I.c = np.where(sel, rng.choice([0.0, 0.5, 2.0, 3.0], I.n), I.c).astype(I.c.dtype)
    return I


@pytest.mark.parametrize("m,dtype", [(4, np.float32), (16, np.float32), (64, np.float32),
                                     (5, np.float32), (7, np.float64)])
def test_alpha_fair_utilities(ctx, torch, m, dtype):
    """Log, capped-linear and alpha-fair jobs mixed in one problem:
    vectorised and generic FP32 kernels and FP64, against the oracle."""
    print("alpha-fair m=%d %s" % (m, np.dtype(dtype).name), flush=True)
    I = _with_alpha_fair(synth.random_small(N_SMALL, m, seed=300 + m, dtype=dtype), 400 + m)
    rng = np.random.default_rng(500 + m)
    for p in (np.ones(m), 0.2 + rng.random(m) * 3):
        _run(ctx, torch, I, p, TOL32 if dtype == np.float32 else TOL64)


def test_alpha_fair_exponent_one_is_log(ctx, torch):
    """Exponent 1 is packed as the log utility: identical results."""
    I = synth.random_small(N_SMALL, 8, seed=600, dtype=np.float32, log_frac=1.0)
    p = round_prices(0.3 + np.arange(8) * 0.2, np.float32)
    a = _problem(ctx, torch, I).dual_eval(p, lower_bound=True)
    I.kind = np.full(I.n, 2, np.uint8)
    I.c = np.ones(I.n, np.float32)
    b = _problem(ctx, torch, I).dual_eval(p, lower_bound=True)
    assert a["g"] == b["g"] and a["lower_bound"] == b["lower_bound"]
    assert np.array_equal(a["grad"], b["grad"])


def test_alpha_fair_exponents_near_one_and_zero(ctx, torch):
    """Exponents one float step either side of 1, within 2^-20 of 1, exactly
    1 (the log utility) and exactly 0 (linear, packed with the sign bit as
    -0): finite results and parity with the oracle."""
    I = synth.random_small(N_SMALL, 8, seed=470, dtype=np.float32)
    one = np.float32(1.0)
    exps = np.array([np.nextafter(one, np.float32(0)), np.nextafter(one, np.float32(2)),
                     one - np.float32(2.0 ** -20), one + np.float32(2.0 ** -20), one,
                     np.float32(0.0)], dtype=np.float32)
    sel = np.arange(I.n) % 3 != 0
    I.kind = np.where(sel, 2, I.kind).astype(np.uint8)
    I.c = np.where(sel, exps[np.arange(I.n) % len(exps)], I.c).astype(np.float32)
    pr = _problem(ctx, torch, I)
    for p in (np.ones(8), 0.3 + np.random.default_rng(471).random(8) * 2):
        p = round_prices(p, np.float32)
        out = pr.dual_eval(p, lower_bound=True, support=True, j1=True)
        assert np.isfinite(out["g"]) and np.isfinite(out["lower_bound"])
        compare_dual(I, p, out, 1e-5)
    pr.close()


def test_first_vertex_probe_mappings_agree_with_oracle(ctx, torch):
    """The first-vertex scan probe (one lane per job, or 2-16 lanes per job
    joined by a shuffle argmax) gives every job the oracle's first vertex
    wherever it is clear of a near-tie, and all mappings agree exactly;
    several tiles per wave (n = 64 x 4 x 2 x CUs x 2 + 64 x 3)."""
    import oracle
    import paper_2104_00282_amd as ra
    from gpu_util import check_first_vertex
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    n = 64 * (4 * 2 * cus * 2 + 3)
    I = synth.random_small(n, 64, seed=4100, dtype=np.float32)
    T = torch.from_numpy(np.ascontiguousarray(I.T)).cuda()
    p = round_prices(0.2 + np.random.default_rng(4101).random(64) * 2, np.float32)
    ref = oracle.dual_eval(I.T, I.w, I.c, I.kind, I.eps, I.R, p, per_job=True)
    first = None
    for G in (1, 2, 4, 8, 16):
        j1 = torch.full((n,), -7, dtype=torch.int16, device="cuda")
        ms = ra.ra_probe_first_vertex_ms(ctx.handle, T.data_ptr(), n, p, G, 1, j1.data_ptr())
        assert ms > 0.0
        got = j1.cpu().numpy().astype(np.int64)
        check_first_vertex(I.T, p, got, ref.jobs["j1"], ref.jobs["margin1"])
        if first is None:
            first = got
        assert np.array_equal(got, first), G
    with pytest.raises(ra.RAError):
        ra.ra_probe_first_vertex_ms(ctx.handle, T.data_ptr(), n - 1, p, 1, 1, j1.data_ptr())
    with pytest.raises(ra.RAError):
        ra.ra_probe_first_vertex_ms(ctx.handle, T.data_ptr(), n, p, 3, 1, j1.data_ptr())
