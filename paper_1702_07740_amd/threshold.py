"""BP thresholds of protograph (base-matrix) ensembles on the BIAWGN channel.

Monte-Carlo density evolution on the base graph: every base edge carries a
population of message samples, the all-zero word is sent (by symmetry the
threshold is the same for every word and syndrome), and the check and
variable rules are those of the sum-product algorithm (Sec. III-D), applied
to populations whose members are shuffled between uses so that the inputs of
a node are independent, as on the tree.  The threshold is the smallest SNR
s = 1/sigma^2 at which the bit error probability of every column reaches
zero (below 1e-6).  This is the notion behind the paper's ensemble threshold
(Sec. III-B); here it picks the SNRs of the mixed-code workload.

Also: the BIAWGN Shannon limit (capacity C(s) = R, computed by quadrature)
for context.
"""
from __future__ import annotations

import math

import numpy as np


def _groups(index_lists):
    """Group node edge-lists by degree: {d: int array (nodes, d)}."""
    by = {}
    for es in index_lists:
        if len(es):
            by.setdefault(len(es), []).append(es)
    return {d: np.array(v, dtype=np.int64) for d, v in by.items()}


def de_converges(base, snr_db: float, n_samples: int = 20000, max_iters: int = 500,
                 seed: int = 0, tol: float = 1e-6) -> bool:
    """Does density evolution reach zero bit error at this SNR?"""
    rng = np.random.default_rng(seed)
    base = np.asarray(base)
    mb, nb = base.shape
    rows, cols = np.nonzero(base >= 0)
    E, N = rows.size, n_samples
    sigma2 = 10.0 ** (-snr_db / 10.0)
    mu = 2.0 / sigma2
    rgroups = _groups([np.nonzero(rows == r)[0] for r in range(mb)])
    cgroups = _groups([np.nonzero(cols == c)[0] for c in range(nb)])
    ar = np.arange(N)

    def shuffled(a):
        # independent random cyclic shift of every edge's population
        off = rng.integers(0, N, size=(a.shape[0], 1))
        return np.take_along_axis(a, (ar[None, :] + off) % N, axis=1)

    L = mu + np.sqrt(2.0 * mu) * rng.standard_normal((E, N))      # VN -> CN
    m = np.empty((E, N))
    for it in range(max_iters):
        t = shuffled(np.tanh(np.clip(L, -40.0, 40.0) / 2.0))
        for d, idx in rgroups.items():                             # check rule
            T = t[idx]                                             # (R, d, N)
            pre = np.cumprod(np.concatenate([np.ones_like(T[:, :1]), T[:, :-1]], axis=1), axis=1)
            suf = np.cumprod(np.concatenate([np.ones_like(T[:, :1]), T[:, :0:-1]], axis=1),
                             axis=1)[:, ::-1]
            P = np.clip(pre * suf, -1.0 + 1e-15, 1.0 - 1e-15)
            m[idx] = 2.0 * np.arctanh(P)
        ms = shuffled(m)
        worst = 0.0
        for d, idx in cgroups.items():                             # variable rule
            M = ms[idx]                                            # (C, d, N)
            tot = mu + np.sqrt(2.0 * mu) * rng.standard_normal((idx.shape[0], N)) + M.sum(axis=1)
            worst = max(worst, float(np.max(np.mean(tot < 0, axis=1))))
            L[idx] = tot[:, None, :] - M
        if worst < tol:
            return True
        if it > 40 and worst > 0.4:
            return False
    return False


def threshold_db(base, lo_db: float, hi_db: float, steps: int = 12, **kw) -> float:
    """Bisection for the BP threshold in dB between lo (fails) and hi (converges)."""
    for _ in range(steps):
        mid = 0.5 * (lo_db + hi_db)
        if de_converges(base, mid, **kw):
            hi_db = mid
        else:
            lo_db = mid
    return hi_db


def biawgn_capacity(snr: float, n_points: int = 4001) -> float:
    """Capacity in bit/use of BPSK over AWGN with SNR s = 1/sigma^2."""
    sigma = 1.0 / math.sqrt(snr)
    y = np.linspace(-1.0 - 12.0 * sigma, 1.0 + 12.0 * sigma, n_points)
    p = np.exp(-(y - 1.0) ** 2 / (2 * sigma ** 2)) / math.sqrt(2 * math.pi * sigma ** 2)
    integrand = p * np.log2(1.0 + np.exp(-2.0 * y / sigma ** 2))
    return 1.0 - float(np.sum(integrand) * (y[1] - y[0]))


def shannon_limit_db(rate: float) -> float:
    """SNR (dB) at which BIAWGN capacity equals the rate."""
    lo, hi = -30.0, 20.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if biawgn_capacity(10.0 ** (mid / 10.0)) >= rate:
            hi = mid
        else:
            lo = mid
    return hi
