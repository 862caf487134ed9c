"""Octonion reference for the 8-dimensional reconciliation front-end (Sec. II-C.3).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain numpy in float64.

Multiplication follows the Cayley-Dickson doubling the paper names: an element
of dimension 2^k is a pair (a, b) of elements of half the dimension, with
    (a, b)(c, d) = (a c - conj(d) b,  d a + b conj(c)),
    conj(a, b)   = (conj(a), -b),
starting from the reals.  At dimension 2 this is complex multiplication, at 4
the quaternions, at 8 the octonions.  The inverse is conj(x) / |x|^2.

Reverse reconciliation in d dimensions (Sec. II-C.3): Bob sends
M = U Y with U = ((-1)^{c_1}, ..., (-1)^{c_d}) and Y = X + Z; Alice forms
R = M X^{-1} = U + N, N = (U Z) X^{-1}.  N is an isotropic Gaussian with
per-coordinate variance d sigma^2 / |X|^2 (the paper's d = 2 form
(a^2 + b^2) sigma^2 = 2 sigma^2 / |X|^2 generalised), so the channel LLR of
coordinate i is 2 R_i |X|^2 / (d sigma^2).
"""
from __future__ import annotations

import numpy as np


def conj(x):
    x = np.asarray(x, dtype=np.float64)
    out = -x.copy()
    out[..., 0] = x[..., 0]
    return out


def mul(x, y):
    """Cayley-Dickson product of arrays of shape (..., 2^k)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    d = x.shape[-1]
    if d == 1:
        return x * y
    h = d // 2
    a, b = x[..., :h], x[..., h:]
    c, e = y[..., :h], y[..., h:]
    left = mul(a, c) - mul(conj(e), b)
    right = mul(e, a) + mul(b, conj(c))
    return np.concatenate([left, right], axis=-1)


def norm2(x):
    return np.sum(np.asarray(x, dtype=np.float64) ** 2, axis=-1)


def inv(x):
    return conj(x) / norm2(x)[..., None]


def tuples(v, d=8):
    """View a length-(d*k) vector as k d-tuples."""
    v = np.asarray(v, dtype=np.float64)
    return v.reshape(v.shape[:-1] + (v.shape[-1] // d, d))


def bob_message(c_bits, Y, d=8):
    """M = U Y per d-tuple; c_bits has n <= len(Y) entries, padding bits are 0."""
    n8 = Y.shape[-1]
    c = np.zeros(Y.shape[:-1] + (n8,), dtype=np.float64)
    c[..., :c_bits.shape[-1]] = c_bits
    U = 1.0 - 2.0 * c
    return mul(tuples(U, d), tuples(Y, d)).reshape(Y.shape)


def alice_llr(M, X, sigma2, n, d=8):
    """Per-coordinate channel LLR 2 R_i |X|^2 / (d sigma^2), R = M X^{-1}; first n kept."""
    Mt, Xt = tuples(M, d), tuples(X, d)
    R = mul(Mt, inv(Xt))
    L = 2.0 * R * norm2(Xt)[..., None] / (d * sigma2)
    return L.reshape(M.shape)[..., :n]
