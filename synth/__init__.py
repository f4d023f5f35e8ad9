"""Seeded synthetic instances of the fungible resource allocation problem.

This module only draws random data; it contains none of the allocation
method's arithmetic.  Both the FP64 oracle (``oracle/``) and the HIP path
(``paper_2104_00282_amd``) consume what it produces, so it imports neither.

An instance is the data of the resource allocation problem (paper §2.4,
eq. e-res-alloc): the efficiency matrix T (row i is the job's efficiency
vector a_i, §2.1), one utility per job (log or capped-linear, §2.2), the
resource limits R and the log offset ``eps``.

Determinism: rows are generated in chunks of ``CHUNK`` jobs; chunk k draws
from ``numpy.random.default_rng(SeedSequence([seed, k]))`` in the fixed
order T (C order), kind, w, c.  Instance-wide draws (column scales, limit
ratios) come from ``SeedSequence([seed, GLOBAL_KEY])``.  Any row range can
therefore be regenerated without generating the whole matrix, and the bytes
do not depend on the number of threads used.

Utility kinds: ``LOG`` (u(t) = w*log(t + eps)) and ``CAPLIN``
(u(t) = w*min(t, c)); capped-linear is the target-priority utility of §2.2
shifted by the constant w*c.
"""
from __future__ import annotations

import dataclasses
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

LOG = 0
CAPLIN = 1

CHUNK = 1 << 16
GLOBAL_KEY = 0xFFFFFFFF
BASE_SEED = 210400282


@dataclasses.dataclass
class Instance:
    """Problem data. T is (n, m) C-contiguous; w, c are (n,) of T's dtype;
    kind is (n,) uint8; R is (m,) float64."""

    name: str
    T: np.ndarray
    w: np.ndarray
    c: np.ndarray
    kind: np.ndarray
    R: np.ndarray
    eps: float
    seed: int

    @property
    def n(self) -> int:
        return self.T.shape[0]

    @property
    def m(self) -> int:
        return self.T.shape[1]

    @property
    def dtype(self):
        return self.T.dtype


# ---------------------------------------------------------------- recipes --
# Each recipe fills rows [lo, hi) of one chunk from its own generator.

def _rows_uniform(rng, rows, m, dt, glob):
    # T_ij ~ U[0.1, 1]
    return (0.1 + 0.9 * rng.random((rows, m), dtype=np.float64)).astype(dt)


def _rows_lognormal_clipped(rng, rows, m, dt, glob):
    # T_ij = clip(exp(0.5 Z), 0.01, 10), Z ~ N(0, 1)
    z = rng.standard_normal((rows, m), dtype=np.float32)
    t = np.exp(np.float32(0.5) * z)
    np.clip(t, np.float32(0.01), np.float32(10.0), out=t)
    return t.astype(dt, copy=False)


def _rows_scaled_lognormal(rng, rows, m, dt, glob):
    # T_ij = s_j * exp(Z_ij), Z ~ N(0, 1), per-column scale s_j (instance-wide)
    z = rng.standard_normal((rows, m), dtype=np.float32)
    t = np.exp(z)
    t *= glob["colscale"].astype(np.float32)[None, :]
    return t.astype(dt, copy=False)


def _rows_scaled_lognormal_clipped(rng, rows, m, dt, glob):
    # learned-warm-start generator: s_j * clip(exp(0.5 Z), 0.01, 10)
    t = _rows_lognormal_clipped(rng, rows, m, np.float32, glob)
    t *= glob["colscale"].astype(np.float32)[None, :]
    return t.astype(dt, copy=False)


def _utils_all_log(rng, rows, dt):
    kind = np.zeros(rows, dtype=np.uint8)
    w = (0.5 + 1.5 * rng.random(rows)).astype(dt)
    c = np.zeros(rows, dtype=dt)
    return kind, w, c


def _utils_mixed(rng, rows, dt):
    # kind ~ Bernoulli(1/2), interleaved; w ~ U[0.5, 2]; c ~ U[0.5, 2]
    kind = (rng.random(rows) < 0.5).astype(np.uint8)
    w = (0.5 + 1.5 * rng.random(rows)).astype(dt)
    c = (0.5 + 1.5 * rng.random(rows)).astype(dt)
    c[kind == LOG] = 0
    return kind, w, c


def _gen_rows(seed, n, m, dt, row_fn, util_fn, glob, threads=None):
    T = np.empty((n, m), dtype=dt)
    kind = np.empty(n, dtype=np.uint8)
    w = np.empty(n, dtype=dt)
    c = np.empty(n, dtype=dt)
    nchunks = (n + CHUNK - 1) // CHUNK

    def work(k):
        lo = k * CHUNK
        hi = min(n, lo + CHUNK)
        rng = np.random.default_rng(np.random.SeedSequence([seed, k]))
        T[lo:hi] = row_fn(rng, hi - lo, m, dt, glob)
        kind[lo:hi], w[lo:hi], c[lo:hi] = util_fn(rng, hi - lo, dt)

    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    if nchunks == 1 or threads == 1:
        for k in range(nchunks):
            work(k)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, range(nchunks)))
    return T, kind, w, c


def _global_rng(seed):
    return np.random.default_rng(np.random.SeedSequence([seed, GLOBAL_KEY]))


# --------------------------------------------------------------- configs --

def small_log(n=1000, m=4, seed=BASE_SEED + 1, dtype=np.float64):
    """n=1e3, m=4, FP64: T ~ U[0.1,1]; all log, w ~ U[0.5,2], eps=1e-3;
    R_j = 0.25 (n/m) mean(T)."""
    T, kind, w, c = _gen_rows(seed, n, m, dtype, _rows_uniform, _utils_all_log, {})
    R = np.full(m, 0.25 * (n / m) * float(T.mean(dtype=np.float64)))
    return Instance("small-log", T, w, c, kind, R, 1e-3, seed)


def mixed_16(n=1_000_000, m=16, seed=BASE_SEED + 2, dtype=np.float32):
    """n=1e6, m=16, FP32: T = clip(lognormal(0, 0.5), 0.01, 10); half log
    (w log(s + 1e-3)), half capped-linear (w min(s, c)), interleaved;
    w, c ~ U[0.5, 2]; R_j = 0.3 n/m."""
    T, kind, w, c = _gen_rows(seed, n, m, dtype, _rows_lognormal_clipped, _utils_mixed, {})
    R = np.full(m, 0.3 * n / m)
    return Instance("mixed-16", T, w, c, kind, R, 1e-3, seed)


def roofline_64(n=10_000_000, m=64, seed=BASE_SEED + 3, dtype=np.float32, threads=None):
    """n=1e7, m=64, FP32: T_ij = s_j exp(Z_ij), s_j ~ U[0.2, 5], Z ~ N(0,1);
    mixed utilities as mixed_16; R_j = 0.1 n/m."""
    g = _global_rng(seed)
    glob = {"colscale": 0.2 + 4.8 * g.random(m)}
    T, kind, w, c = _gen_rows(seed, n, m, dtype, _rows_scaled_lognormal, _utils_mixed, glob,
                              threads=threads)
    R = np.full(m, 0.1 * n / m)
    return Instance("roofline-64", T, w, c, kind, R, 1e-3, seed)


def roofline_rows(lo, hi, n=10_000_000, m=64, seed=BASE_SEED + 3, dtype=np.float32):
    """Rows [lo, hi) of roofline_64 (chunk-aligned regeneration), returned as
    (T, kind, w, c) without generating the rest of the matrix."""
    g = _global_rng(seed)
    glob = {"colscale": 0.2 + 4.8 * g.random(m)}
    k0, k1 = lo // CHUNK, (hi + CHUNK - 1) // CHUNK
    parts = []
    for k in range(k0, k1):
        a = k * CHUNK
        b = min(n, a + CHUNK)
        rng = np.random.default_rng(np.random.SeedSequence([seed, k]))
        T = _rows_scaled_lognormal(rng, b - a, m, dtype, glob)
        kind, w, c = _utils_mixed(rng, b - a, dtype)
        parts.append((a, T, kind, w, c))
    T = np.concatenate([p[1] for p in parts])
    kind = np.concatenate([p[2] for p in parts])
    w = np.concatenate([p[3] for p in parts])
    c = np.concatenate([p[4] for p in parts])
    off = lo - k0 * CHUNK
    s = slice(off, off + (hi - lo))
    return T[s], kind[s], w[s], c[s]


def warmstart_instance(n, m=16, seed=BASE_SEED + 100000, dtype=np.float32):
    """Generator for the learned warm start: mixed utilities and clipped
    lognormal(0, 0.5) entries as mixed_16, times a per-instance column scale
    s_j ~ U[0.2, 5]; per-instance limits R_j = rho_j n/m, rho_j ~ U[0.1, 0.5]."""
    g = _global_rng(seed)
    colscale = 0.2 + 4.8 * g.random(m)
    rho = 0.1 + 0.4 * g.random(m)
    T, kind, w, c = _gen_rows(seed, n, m, dtype, _rows_scaled_lognormal_clipped, _utils_mixed,
                              {"colscale": colscale})
    R = rho * n / m
    return Instance("warmstart", T, w, c, kind, R, 1e-3, seed)


def batch_instances(count=512, seed0=BASE_SEED + 1000, dtype=np.float32, nmin=1e3, nmax=1e6,
                    ms=(4, 8, 16, 32)):
    """Batched workload: instance b has n_b = round(10^U[log10 nmin, log10 nmax]),
    m_b uniform on ``ms``, and the mixed_16 recipe (seed seed0 + b)."""
    out = []
    for b in range(count):
        g = _global_rng(seed0 + b)
        n = int(round(10 ** (math.log10(nmin) + (math.log10(nmax) - math.log10(nmin)) * g.random())))
        m = int(ms[int(g.integers(len(ms)))])
        out.append(mixed_16(n=n, m=m, seed=seed0 + b, dtype=dtype))
    return out


def random_small(n, m, seed, dtype=np.float64, log_frac=0.5, zero_frac=0.0, eps=1e-3,
                 r_scale=0.3):
    """Small random instance for tests: T ~ U[0, 1] with an optional fraction
    of exact zeros, mixed utilities, R_j = r_scale n/m."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7]))
    T = rng.random((n, m))
    if zero_frac > 0:
        T[rng.random((n, m)) < zero_frac] = 0.0
    kind = (rng.random(n) >= log_frac).astype(np.uint8)
    w = 0.5 + 1.5 * rng.random(n)
    c = 0.5 + 1.5 * rng.random(n)
    c[kind == LOG] = 0
    R = np.full(m, r_scale * n / m)
    return Instance("random-small", T.astype(dtype), w.astype(dtype), c.astype(dtype), kind, R,
                    eps, seed)


def e1_instance(kind, n=1_000_000, seed=BASE_SEED + 5, dtype=np.float32):
    """The paper's medium-size example (§6.2): m = 4 with a_i1 ~ U(0.1, 0.3),
    a_i2 ~ U(0.1, 0.5), a_i3 ~ U(0.3, 0.8), a_i4 ~ U(0.6, 1.0) and limits
    R = (8e5, 1e5, 1e4, 1e3) (scaled by n / 1e6 for other n).
    kind "log": u_i = log t (w = 1, eps = 0).  kind "target": target-priority
    utility with target throughput 0.2 and priority w_i = 1 or 2 with
    probability 1/2 each, in the capped form w min(t, 0.2) (same maximisers).
    The paper's draws are not published; these are seeded."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 11]))
    lo = np.array([0.1, 0.1, 0.3, 0.6])
    hi = np.array([0.3, 0.5, 0.8, 1.0])
    T = (lo + (hi - lo) * rng.random((n, 4))).astype(dtype)
    R = np.array([8e5, 1e5, 1e4, 1e3]) * (n / 1e6)
    if kind == "log":
        w = np.ones(n)
        c = np.zeros(n)
        k = np.full(n, LOG, np.uint8)
    elif kind == "target":
        w = np.where(rng.random(n) < 0.5, 1.0, 2.0)
        c = np.full(n, 0.2)
        k = np.full(n, CAPLIN, np.uint8)
    else:
        raise ValueError(kind)
    return Instance("e1-" + kind, T, w.astype(dtype), c.astype(dtype), k, R, 0.0, seed)


CONFIGS = {
    "small-log": small_log,
    "mixed-16": mixed_16,
    "roofline-64": roofline_64,
}


def warmstart_device(n, m=16, seed=BASE_SEED + 100000, device="cuda"):
    """The warm-start generator drawn on the GPU with torch's seeded generator
    (fast enough for tens of thousands of instances): per-instance column
    scale s_j ~ U[0.2, 5] and limit ratio rho_j ~ U[0.1, 0.5];
    T_ij = s_j clip(exp(0.5 Z_ij), 0.01, 10); kind ~ Bernoulli(1/2);
    w, c ~ U[0.5, 2]; R_j = rho_j n / m.  Returns (T, w, c, kind) device
    tensors and R (numpy).  The streams differ from the numpy generator's, so
    these instances are checked through properties and per-instance oracle
    runs on copies, not regenerated on the host."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
    colscale = 0.2 + 4.8 * torch.rand(m, generator=g, device=device, dtype=torch.float64)
    rho = 0.1 + 0.4 * torch.rand(m, generator=g, device=device, dtype=torch.float64)
    T = torch.randn((n, m), generator=g, device=device, dtype=torch.float32)
    T.mul_(0.5).exp_().clamp_(0.01, 10.0)
    T.mul_(colscale.to(torch.float32)[None, :])
    kind = (torch.rand(n, generator=g, device=device) < 0.5).to(torch.uint8)
    w = 0.5 + 1.5 * torch.rand(n, generator=g, device=device)
    c = 0.5 + 1.5 * torch.rand(n, generator=g, device=device)
    R = (rho * n / m).cpu().numpy()
    return T.contiguous(), w, c, kind, R


def extension_device(variant, n=10_000_000, m=64, device="cuda"):
    """Instances of the roofline-64 shape for the §7 extensions and the
    alpha-fair family, drawn on the GPU with torch's seeded generator:
    T_ij = s_j exp(Z_ij), s_j ~ U[0.2, 5]; w ~ U[0.5, 2]; eps = 1e-3; and a
    seeded price vector p ~ U[0.5, 1.5]^m for evaluations at fixed prices.
    - "demand-vectors" (seed offset 6): kind ~ Bernoulli(1/2) (log / capped
      linear, c ~ U[0.5, 2]); demands D_ij ~ U[0.5, 2] (units of resource j a
      job uses while running on it); R_j = 0.125 n/m (the roofline-64 limits
      times the mean demand).
    - "demands" (offset 7): the same utilities; one demand per job,
      d_i ~ U[0.5, 2]; R_j = 0.125 n/m.
    - "alpha-fair" (offset 8): a third each of log, capped-linear
      (c ~ U[0.5, 2]) and alpha-fair jobs with exponent a ~ U[0, 3] in c;
      R_j = 0.1 n/m.
    Returns a dict of device tensors (T, w, c, kind, and D or d) and host
    values (R, p, eps, n, m)."""
    import torch

    offset = {"demand-vectors": 6, "demands": 7, "alpha-fair": 8}[variant]
    g = torch.Generator(device=device)
    g.manual_seed(int(BASE_SEED + offset) & 0x7FFFFFFFFFFFFFFF)
    colscale = 0.2 + 4.8 * torch.rand(m, generator=g, device=device, dtype=torch.float64)
    T = torch.randn((n, m), generator=g, device=device, dtype=torch.float32)
    T.exp_().mul_(colscale.to(torch.float32)[None, :])
    if variant == "alpha-fair":
        kind = torch.randint(0, 3, (n,), generator=g, device=device).to(torch.uint8)
    else:
        kind = (torch.rand(n, generator=g, device=device) < 0.5).to(torch.uint8)
    w = 0.5 + 1.5 * torch.rand(n, generator=g, device=device)
    c = 0.5 + 1.5 * torch.rand(n, generator=g, device=device)
    out = {"T": T.contiguous(), "w": w, "kind": kind, "eps": 1e-3, "n": n, "m": m}
    if variant == "demand-vectors":
        out["D"] = (0.5 + 1.5 * torch.rand((n, m), generator=g, device=device)).contiguous()
    elif variant == "demands":
        out["d"] = 0.5 + 1.5 * torch.rand(n, generator=g, device=device)
    else:
        a = 3.0 * torch.rand(n, generator=g, device=device)
        c = torch.where(kind == 2, a, c)
    out["c"] = c
    out["p"] = (0.5 + torch.rand(m, generator=g, device=device, dtype=torch.float64)).cpu().numpy()
    out["R"] = np.full(m, (0.1 if variant == "alpha-fair" else 0.125) * n / m)
    return out


def demand_vectors_device(n=10_000_000, m=64, device="cuda"):
    """extension_device("demand-vectors")."""
    return extension_device("demand-vectors", n=n, m=m, device=device)
