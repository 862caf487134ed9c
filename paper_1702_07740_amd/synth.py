"""Seeded synthetic inputs: QC multi-edge base matrices and BIAWGN frames.

This module only draws inputs.  It holds none of the decoder's arithmetic:
no parity checks, no syndromes, no message updates.  Both the CPU oracle
(through the tests) and the HIP decoder consume what it returns.

Code template (the rate-0.02 multi-edge structure of Sec. III-B, made
quasi-cyclic as in Sec. III-C): 6 "core" columns and ``n_deg1`` degree-1
columns; 3 type-1 rows joined to all 6 core columns and ``n_deg1`` type-2
rows, each joined to its own degree-1 column through an unshifted identity
block (the long diagonal of Sec. III-C) and to two core columns dealt in
round-robin pairs (row j takes core columns 2j mod 6 and 2j+1 mod 6).
Every core block gets a seeded shift in [0, Z).  Base entries are -1 for a
zero block and the 0-based right shift s otherwise: row a of the block has
its 1 in column (a + s) mod Z (the paper's I_i with s = i - 1).

Channel (Sec. II-C, virtual BIAWGN with SNR s = 1/sigma^2): x ~ Bernoulli(1/2),
y = (1 - 2x) + N(0, sigma^2), channel LLR 2y/sigma^2 computed in float64 and
rounded to float32.
"""
from __future__ import annotations

import math

import numpy as np

N_CORE = 6
N_TYPE1 = 3

# Degree-1 column counts of the three rates used in the workloads.
N_DEG1_FOR_RATE = {0.02: 144, 0.05: 54, 0.1: 24}


def sigma2_from_snr_db(snr_db: float) -> float:
    """Noise variance of the virtual BIAWGN channel at SNR ``snr_db`` (s = 1/sigma^2)."""
    return 10.0 ** (-snr_db / 10.0)


def snr_db_from_beta(rate: float, beta: float) -> float:
    """SNR in dB for efficiency beta at code rate R: s = 2^(2R/beta) - 1 (eq. snr(beta))."""
    s = 2.0 ** (2.0 * rate / beta) - 1.0
    return 10.0 * math.log10(s)


def template_base(n_deg1: int, Z: int, seed: int = 1) -> np.ndarray:
    """Base matrix of the multi-edge QC template, shape (3 + n_deg1, 6 + n_deg1), int32."""
    if n_deg1 < 0 or Z < 1:
        raise ValueError("n_deg1 >= 0 and Z >= 1 required")
    mb, nb = N_TYPE1 + n_deg1, N_CORE + n_deg1
    rng = np.random.default_rng([0x51D0C0DE, seed, n_deg1, Z])
    B = np.full((mb, nb), -1, dtype=np.int32)
    for r in range(N_TYPE1):
        B[r, :N_CORE] = rng.integers(0, Z, size=N_CORE)
    for j in range(n_deg1):
        r = N_TYPE1 + j
        c1, c2 = (2 * j) % N_CORE, (2 * j + 1) % N_CORE
        B[r, c1] = rng.integers(0, Z)
        B[r, c2] = rng.integers(0, Z)
        B[r, N_CORE + j] = 0
    return B


def template_for_rate(rate: float, Z: int, seed: int = 1) -> np.ndarray:
    return template_base(N_DEG1_FOR_RATE[rate], Z, seed)


def random_bits(n: int, F: int, seed: int, first_frame: int = 0) -> np.ndarray:
    """Uniform key bits, uint8 [F][n]; frame f depends only on (seed, first_frame + f)."""
    out = np.empty((F, n), dtype=np.uint8)
    for f in range(F):
        rng = np.random.default_rng([0xB175, seed, first_frame + f])
        out[f] = rng.integers(0, 2, size=n, dtype=np.uint8)
    return out


def biawgn_frames(n: int, F: int, snr_db: float, seed: int, first_frame: int = 0):
    """Key bits x (uint8 [F][n]) and channel LLRs (float32 [F][n]) at ``snr_db``.

    Frame f is a pure function of (seed, first_frame + f), so a frame decoded
    alone or inside any batch sees identical inputs.
    """
    sigma2 = sigma2_from_snr_db(snr_db)
    sigma = math.sqrt(sigma2)
    x = np.empty((F, n), dtype=np.uint8)
    llr = np.empty((F, n), dtype=np.float32)
    for f in range(F):
        rng = np.random.default_rng([0xF4A3E, seed, first_frame + f])
        xf = rng.integers(0, 2, size=n, dtype=np.uint8)
        y = (1.0 - 2.0 * xf.astype(np.float64)) + sigma * rng.standard_normal(n)
        x[f] = xf
        llr[f] = (2.0 * y / sigma2).astype(np.float32)
    return x, llr


def noiseless_llr(x: np.ndarray, magnitude: float = 20.0) -> np.ndarray:
    """LLRs that point exactly at the bits x with a fixed magnitude."""
    return (magnitude * (1.0 - 2.0 * x.astype(np.float64))).astype(np.float32)


def reconciliation_inputs(n: int, d: int, F: int, snr_db: float, seed: int, first_frame: int = 0):
    """Inputs of d-dimensional reverse reconciliation (Sec. II-C.3).

    Returns (c, X, Z): key bits c uint8 [F][n], Alice's Gaussian samples
    X ~ N(0, 1) and channel noise Z ~ N(0, sigma^2), both float64 [F][n_d]
    with n_d = d * ceil(n / d); the last tuple is padded with extra samples
    whose coordinates are dropped after the LLRs are formed.  Bob holds
    Y = X + Z.
    """
    sigma = math.sqrt(sigma2_from_snr_db(snr_db))
    nd = d * ((n + d - 1) // d)
    c = np.empty((F, n), dtype=np.uint8)
    X = np.empty((F, nd), dtype=np.float64)
    Zn = np.empty((F, nd), dtype=np.float64)
    for f in range(F):
        rng = np.random.default_rng([0x0C7A, d, seed, first_frame + f])
        c[f] = rng.integers(0, 2, size=n, dtype=np.uint8)
        X[f] = rng.standard_normal(nd)
        Zn[f] = sigma * rng.standard_normal(nd)
    return c, X, Zn
