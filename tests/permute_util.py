"""Test helpers for reordered inputs: the row-profile form of P A P^T built by
brute force from the entries of A (no tiles, no segments), and the element-
level fill of a small pattern by dense boolean elimination."""
import numpy as np


def profile_entries(f, values):
    """(rows, cols, values) of the lower envelope entries of a row profile."""
    f = np.asarray(f, dtype=np.int64)
    N = len(f)
    lens = np.arange(N) - f + 1
    rp = np.concatenate([[0], np.cumsum(lens)])
    rows = np.repeat(np.arange(N), lens)
    cols = f[rows] + (np.arange(rp[-1]) - rp[rows])
    return rows, cols, np.asarray(values)


def permute_profile(f, values, perm):
    """Row profile (f2, values2) of P A P^T, perm[new] = old."""
    perm = np.asarray(perm, dtype=np.int64)
    N = len(perm)
    iperm = np.empty(N, dtype=np.int64)
    iperm[perm] = np.arange(N)
    rows, cols, v = profile_entries(f, values)
    pi, pj = iperm[rows], iperm[cols]
    hi, lo = np.maximum(pi, pj), np.minimum(pi, pj)
    f2 = np.arange(N, dtype=np.int64)
    np.minimum.at(f2, hi, lo)
    rp2 = np.concatenate([[0], np.cumsum(np.arange(N) - f2 + 1)])
    v2 = np.zeros(rp2[-1])
    v2[rp2[hi] + lo - f2[hi]] = v
    return f2, v2


def filled_lower(N, rows, cols):
    """Boolean lower-triangular pattern of L for the given lower entries."""
    M = np.zeros((N, N), dtype=bool)
    M[rows, cols] = True
    M[np.arange(N), np.arange(N)] = True
    for k in range(N):
        r = np.nonzero(M[k + 1:, k])[0] + k + 1
        if len(r) > 1:
            M[np.ix_(r, r)] |= np.tril(np.ones((len(r), len(r)), dtype=bool))
    return np.tril(M)
