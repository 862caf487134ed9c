"""Test-side helpers built straight from the paper's definitions (no decoder code).

``dense_H`` builds the parity-check matrix the way Sec. III-C defines it:
each non-zero base entry becomes the Z x Z identity with every row cyclically
shifted right by the (0-based) shift, each -1 entry a zero block.
``map_llr`` enumerates every word to get exact bitwise MAP posteriors.
"""
import numpy as np


def dense_H(base: np.ndarray, Z: int) -> np.ndarray:
    mb, nb = base.shape
    H = np.zeros((mb * Z, nb * Z), dtype=np.uint8)
    I = np.eye(Z, dtype=np.uint8)
    for r in range(mb):
        for c in range(nb):
            s = int(base[r, c])
            if s >= 0:
                H[r * Z:(r + 1) * Z, c * Z:(c + 1) * Z] = np.roll(I, s, axis=1)
    return H


def syndrome_dense(H: np.ndarray, x: np.ndarray) -> np.ndarray:
    return ((x.astype(np.int64) @ H.T.astype(np.int64)) & 1).astype(np.uint8)


def map_llr(H: np.ndarray, s: np.ndarray, Q: np.ndarray) -> np.ndarray:
    """Exact posterior LLRs ln P(x_v=0 | Q, Hx=s) / P(x_v=1 | Q, Hx=s), by enumeration.

    Prior of a word: prod_v exp((1 - 2 x_v) Q_v / 2), i.e. Q_v = ln P(0)/P(1).
    """
    m, n = H.shape
    assert n <= 20
    words = np.arange(1 << n, dtype=np.int64)
    bits = ((words[:, None] >> np.arange(n)) & 1).astype(np.uint8)
    par = (bits.astype(np.int64) @ H.T.astype(np.int64)) & 1
    valid = np.all(par == s[None, :].astype(np.int64), axis=1)
    lw = -(bits[valid].astype(np.float64) @ Q.astype(np.float64))
    vb = bits[valid]
    out = np.empty(n)
    for v in range(n):
        a = lw[vb[:, v] == 0]
        b = lw[vb[:, v] == 1]
        la = np.max(a) + np.log(np.sum(np.exp(a - np.max(a))))
        lb = np.max(b) + np.log(np.sum(np.exp(b - np.max(b))))
        out[v] = la - lb
    return out


def random_tree_base(rng, n_var: int, n_chk: int, Z: int = 1) -> np.ndarray:
    """Base matrix whose Tanner graph is a tree (each check of degree >= 2).

    A Z-lift of a tree is a forest of Z copies, so BP stays exact after lifting.
    """
    assert n_var - 1 >= n_chk >= 1
    # split the n_var - 1 non-root variables over the checks, >= 1 child each
    cuts = np.sort(rng.choice(np.arange(1, n_var - 1), size=n_chk - 1, replace=False)) \
        if n_chk > 1 else np.array([], dtype=int)
    sizes = np.diff(np.concatenate([[0], cuts, [n_var - 1]])).astype(int)
    B = np.full((n_chk, n_var), -1, dtype=np.int32)
    placed = [0]
    nxt = 1
    for j in range(n_chk):
        parent = placed[rng.integers(0, len(placed))]
        B[j, parent] = rng.integers(0, Z)
        for _ in range(sizes[j]):
            B[j, nxt] = rng.integers(0, Z)
            placed.append(nxt)
            nxt += 1
    rp = rng.permutation(n_chk)
    cp = rng.permutation(n_var)
    return np.ascontiguousarray(B[rp][:, cp])
