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

The same rules run on multi-edge ensembles given by degree distributions
(ensemble_de_converges), which pins the tool to the threshold the paper
quotes for its rate-0.02 ensemble.

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


def _channel(rng, mu: float, shape):
    """Channel LLRs of the all-zero word on the BIAWGN channel with SNR s:
    N(mu, 2 mu) with mu = 2 s (the consistent Gaussian density)."""
    return mu + np.sqrt(2.0 * mu) * rng.standard_normal(shape)


def _tanh_half(L):
    return np.tanh(np.clip(L, -40.0, 40.0) / 2.0)


def _check_out(P):
    """Check rule of the sum-product algorithm from the product P of the
    other inputs' tanh(L/2): 2 atanh(P)."""
    return 2.0 * np.arctanh(np.clip(P, -1.0 + 1e-15, 1.0 - 1e-15))


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

    L = _channel(rng, mu, (E, N))                                 # VN -> CN
    m = np.empty((E, N))
    for it in range(max_iters):
        t = shuffled(_tanh_half(L))
        for d, idx in rgroups.items():                             # check rule
            T = t[idx]                                             # (R, d, N)
            pre = np.cumprod(np.concatenate([np.ones_like(T[:, :1]), T[:, :-1]], axis=1), axis=1)
            suf = np.cumprod(np.concatenate([np.ones_like(T[:, :1]), T[:, :0:-1]], axis=1),
                             axis=1)[:, ::-1]
            m[idx] = _check_out(pre * suf)
        ms = shuffled(m)
        worst = 0.0
        for d, idx in cgroups.items():                             # variable rule
            M = ms[idx]                                            # (C, d, N)
            tot = _channel(rng, mu, (idx.shape[0], N)) + M.sum(axis=1)
            worst = max(worst, float(np.max(np.mean(tot < 0, axis=1))))
            L[idx] = tot[:, None, :] - M
        if worst < tol:
            return True
        if it > 40 and worst > 0.4:
            return False
    return False


# The paper's rate-0.02 multi-edge ensemble (Sec. III-B) as (fraction of n,
# sockets of edge types 1, 2, 3) per variable class and per check class.  The
# two type-1 check terms are read with their exponents swapped (degree 7 for
# 3/320 of the nodes, degree 3 for 17/1600): as printed, the type-1 sockets of
# the checks (0.1025 n) would not match those of the variables (0.0975 n);
# swapped they match exactly, and the rate is 0.02 either way.
PAPER_RATE_002_VARIABLES = ((9 / 400, (2, 57, 0)), (7 / 400, (3, 57, 0)), (24 / 25, (0, 0, 1)))
PAPER_RATE_002_CHECKS = ((3 / 320, (7, 0, 0)), (17 / 1600, (3, 0, 0)), (3 / 5, (0, 2, 1)),
                         (9 / 25, (0, 3, 1)))
PAPER_RATE_002_CHECKS_AS_PRINTED = ((3 / 320, (3, 0, 0)), (17 / 1600, (7, 0, 0)),
                                    (3 / 5, (0, 2, 1)), (9 / 25, (0, 3, 1)))
# the threshold the paper quotes for it: s = 2.863e-2, i.e. -15.43 dB
PAPER_RATE_002_THRESHOLD_DB = 10.0 * math.log10(2.863e-2)


def ensemble_de_converges(variables, checks, snr_db: float, n_samples: int = 20000,
                          max_iters: int = 500, seed: int = 0, tol: float = 1e-6) -> bool:
    """Density evolution of a multi-edge ensemble (node classes given by their
    fraction and their sockets of each edge type; every variable sees the
    channel).  One population of VN -> CN messages per edge type; a check
    (variable) output on a type-e edge comes from a node class drawn with the
    edge-perspective probability fraction * sockets of type e, combining
    fresh random draws from the populations of its other sockets with the
    same check and variable rules as de_converges.  Converged when every
    variable class's posterior error is below tol."""
    rng = np.random.default_rng(seed)
    T = len(variables[0][1])
    N = n_samples
    mu = 2.0 * 10.0 ** (snr_db / 10.0)
    vfrac = np.array([f for f, _ in variables])
    vdeg = np.array([d for _, d in variables], dtype=np.int64)
    cfrac = np.array([f for f, _ in checks])
    cdeg = np.array([d for _, d in checks], dtype=np.int64)

    def classes(frac, deg, e):
        w = frac * deg[:, e]
        counts = np.floor(N * w / w.sum()).astype(np.int64)   # stratified: fixed counts
        counts[np.argmax(w)] += N - counts.sum()
        return counts

    L = [_channel(rng, mu, N) for _ in range(T)]
    M = [np.zeros(N) for _ in range(T)]
    for it in range(max_iters):
        for e in range(T):                                           # check rule
            out, at = np.empty(N), 0
            for c, k in enumerate(classes(cfrac, cdeg, e)):
                if k == 0:
                    continue
                P = np.ones(k)
                for e2 in range(T):
                    for _ in range(cdeg[c, e2] - (1 if e2 == e else 0)):
                        P *= _tanh_half(L[e2][rng.integers(0, N, k)])
                out[at:at + k] = _check_out(P)
                at += k
            M[e] = rng.permutation(out)
        newL = []
        for e in range(T):                                           # variable rule
            out, at = np.empty(N), 0
            for c, k in enumerate(classes(vfrac, vdeg, e)):
                if k == 0:
                    continue
                acc = _channel(rng, mu, k)
                for e2 in range(T):
                    cnt = vdeg[c, e2] - (1 if e2 == e else 0)
                    if cnt:
                        acc = acc + M[e2][rng.integers(0, N, (k, cnt))].sum(axis=1)
                out[at:at + k] = acc
                at += k
            newL.append(rng.permutation(out))
        L = newL
        worst = 0.0
        for c in range(len(variables)):                              # posteriors
            acc = _channel(rng, mu, N)
            for e2 in range(T):
                if vdeg[c, e2]:
                    acc = acc + M[e2][rng.integers(0, N, (N, vdeg[c, e2]))].sum(axis=1)
            worst = max(worst, float(np.mean(acc < 0)))
        if worst < tol:
            return True
        if it > 60 and worst > 0.45:
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
