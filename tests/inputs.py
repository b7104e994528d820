"""Seeded synthetic inputs shared by the oracle side and the HIP side of the
parity tests.  Only random arrays and workload shapes live here: none of the
method's arithmetic."""
import numpy as np

# Workloads (sizes of the paper's method as configured for this build).
CFG_SMALL = dict(lam=1.0, beta=2.0, eps=0.1, n=10_000, dt=1e-3, T=1.0, K=10, iters=2, cells=200, nq=100)
CFG_LARGE = dict(lam=1.0, beta=2.0, eps=0.01, n=2 ** 20, dt=1e-4, T=10.0, K=64, iters=6, cells=1024, nq=100)


def slow_values(seed, k, n, ties=True):
    """k x n FP64 values shaped like the slow variable (bimodal around +-1),
    with exact ties, signed zeros and a few far outliers when ties=True."""
    rng = np.random.default_rng(seed)
    x = np.where(rng.random((k, n)) < 0.5, -1.0, 1.0) + 0.45 * rng.standard_normal((k, n))
    if ties and n >= 16:
        m = max(1, n // 50)
        for s in range(k):
            idx = rng.choice(n, size=m, replace=False)
            x[s, idx] = np.round(x[s, idx], 1)        # exact ties
            x[s, idx[: max(1, m // 4)]] = -0.0          # signed zeros
            x[s, idx[max(1, m // 4): max(2, m // 2)]] = 0.0
            x[s, idx[-1]] = 7.5 if s % 2 else -9.25     # outlier
    return np.ascontiguousarray(x)


def monotone_knots(seed, k, nq, lo=-2.5, hi=2.5):
    rng = np.random.default_rng(seed)
    q = np.sort(rng.uniform(lo, hi, (k, nq + 1)), axis=1)
    return np.ascontiguousarray(q)


def ranks(seed, k, n):
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(np.stack([rng.permutation(n) for _ in range(k)]).astype(np.uint32))
