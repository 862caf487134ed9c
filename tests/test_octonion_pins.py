"""Pins of the octonion reference (8-D reconciliation front-end, Sec. II-C.3).

Checked against the algebra the paper relies on: the composition property
|ab| = |a||b| (Hurwitz), alternativity, right cancellation (ab)b^{-1} = a used
in the paper's derivation, the unit relations e_i^2 = -1, e_i e_j = -e_j e_i,
the d = 2 noise forms printed in the paper, and the noise variance.
"""
import numpy as np

from oracle import octonion as oc


def test_dimension_two_is_complex_multiplication():
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal((2, 50, 2))
    got = oc.mul(a, b)
    ref = (a[:, 0] + 1j * a[:, 1]) * (b[:, 0] + 1j * b[:, 1])
    np.testing.assert_allclose(got[:, 0], ref.real, atol=1e-14)
    np.testing.assert_allclose(got[:, 1], ref.imag, atol=1e-14)


def test_dimension_four_is_quaternion_multiplication():
    # Hamilton: i j = k, j k = i, k i = j, i^2 = j^2 = k^2 = -1
    E = np.eye(4)
    one, i, j, k = E
    np.testing.assert_allclose(oc.mul(i, j), k)
    np.testing.assert_allclose(oc.mul(j, k), i)
    np.testing.assert_allclose(oc.mul(k, i), j)
    for u in (i, j, k):
        np.testing.assert_allclose(oc.mul(u, u), -one)


def test_octonion_units_and_composition():
    E = np.eye(8)
    for p in range(1, 8):
        np.testing.assert_allclose(oc.mul(E[p], E[p]), -E[0])
        for q in range(1, 8):
            if p != q:
                np.testing.assert_allclose(oc.mul(E[p], E[q]), -oc.mul(E[q], E[p]))
    rng = np.random.default_rng(2)
    a, b, c = rng.standard_normal((3, 200, 8))
    np.testing.assert_allclose(oc.norm2(oc.mul(a, b)), oc.norm2(a) * oc.norm2(b), rtol=1e-12)
    # alternative, not associative
    np.testing.assert_allclose(oc.mul(oc.mul(a, a), b), oc.mul(a, oc.mul(a, b)), atol=1e-10)
    np.testing.assert_allclose(oc.mul(oc.mul(a, b), b), oc.mul(a, oc.mul(b, b)), atol=1e-10)
    assert np.max(np.abs(oc.mul(oc.mul(a, b), c) - oc.mul(a, oc.mul(b, c)))) > 1e-3
    # right cancellation, the step the paper's derivation of R uses
    np.testing.assert_allclose(oc.mul(oc.mul(a, b), oc.inv(b)), a, atol=1e-10)


def test_paper_d2_noise_forms():
    """C = 0, d = 2: N = (U Z) X^{-1} has N1 = a Z1 + b Z2, N2 = a Z2 - b Z1 with
    a = (X1 + X2)/|X|^2 and b = (X2 - X1)/|X|^2."""
    rng = np.random.default_rng(3)
    X, Z = rng.standard_normal((2, 100, 2))
    U = np.ones((100, 2))
    N = oc.mul(oc.mul(U, Z), oc.inv(X))
    n2 = oc.norm2(X)
    a = (X[:, 0] + X[:, 1]) / n2
    b = (X[:, 1] - X[:, 0]) / n2
    np.testing.assert_allclose(N[:, 0], a * Z[:, 0] + b * Z[:, 1], atol=1e-12)
    np.testing.assert_allclose(N[:, 1], a * Z[:, 1] - b * Z[:, 0], atol=1e-12)


def test_reconciliation_recovers_signs_and_noise_variance():
    rng = np.random.default_rng(4)
    k, sigma2 = 200000, 0.7
    X = rng.standard_normal((k, 8))
    Z = np.sqrt(sigma2) * rng.standard_normal((k, 8))
    c = rng.integers(0, 2, size=(k, 8)).astype(np.float64)
    U = 1.0 - 2.0 * c
    M = oc.mul(U, X + Z)
    R = oc.mul(M, oc.inv(X))
    # noiseless: R = U exactly
    np.testing.assert_allclose(oc.mul(oc.mul(U, X), oc.inv(X)), U, atol=1e-10)
    # N = R - U scaled by |X| / sqrt(8 sigma^2) is standard normal per coordinate
    Nn = (R - U) * np.sqrt(oc.norm2(X))[:, None] / np.sqrt(8 * sigma2)
    assert abs(np.mean(Nn)) < 0.01
    assert abs(np.var(Nn) - 1.0) < 0.01
    # the LLR helper is 2 R |X|^2 / (8 sigma^2) on the flattened frame
    n = k * 8 - 3
    L = oc.alice_llr(M.reshape(-1), X.reshape(-1), sigma2, n)
    np.testing.assert_allclose(L, (2 * R * oc.norm2(X)[:, None] / (8 * sigma2)).reshape(-1)[:n])
