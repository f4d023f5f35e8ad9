"""Full-size parity for the benchmark's extension workloads (n = 1e7, m = 64,
FP32, the vectorised kernel): per-job demands and alpha-fair utilities.
Sampled jobs' supports are compared with the oracle solved on those rows
alone, and r with the sum of the kernel's own per-job outputs (FP64 on the
device).  The demand-vector workload has the same test beside its other
tests."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import round_prices

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


@pytest.mark.parametrize("variant", ["demands", "alpha-fair"])
def test_full_size_sampled_parity(ctx, torch, variant):
    import paper_2104_00282_amd as ra
    print("full-size %s" % variant, flush=True)
    I = synth.extension_device(variant)
    n, m = I["n"], I["m"]
    pr = ra.Problem(ctx, I["T"], I["w"], I["c"], I["kind"], I["R"], I["eps"], validate=False)
    if variant == "demands":
        pr.set_demands(I["d"])
    p = round_prices(I["p"], np.float32)
    out = pr.dual_eval(p, support=True)
    jp = out["j_pair"].long()
    xp = out["x_pair"].double()
    dd = I["d"].double() if variant == "demands" else torch.ones(n, dtype=torch.float64,
                                                                 device="cuda")
    r = torch.zeros(m, dtype=torch.float64, device="cuda")
    for k in (0, 1):
        ok = jp[:, k] >= 0
        r.index_add_(0, jp[ok, k], dd[ok] * xp[ok, k])
    assert np.allclose(out["r"], r.cpu().numpy(), rtol=1e-5)
    idx = np.sort(np.random.default_rng(860).choice(n, 3000, replace=False))
    ti = torch.from_numpy(idx).cuda()
    T = I["T"][ti].cpu().numpy()
    w = I["w"][ti].cpu().numpy()
    c = I["c"][ti].cpu().numpy()
    kind = I["kind"][ti].cpu().numpy()
    d = I["d"][ti].cpu().numpy().astype(np.float64) if variant == "demands" else None
    ref = oracle.dual_eval(T, w, c, kind, I["eps"], I["R"], p, per_job=True, d=d)
    jps = jp[ti].cpu().numpy()
    xps = xp[ti].cpu().numpy()
    same = (jps[:, 1] == ref.jobs["jhi"]) & np.isclose(xps[:, 1], ref.jobs["xhi"], atol=1e-4)
    assert same.mean() >= 0.998
    if variant == "alpha-fair":
        assert (kind == 2).sum() > 800  # the sample holds alpha-fair jobs
    pr.close()
