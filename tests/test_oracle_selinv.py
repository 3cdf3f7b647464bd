"""Pins for the oracle's selected inversion (entries of A^{-1} inside the
envelope) against facts fixed outside the oracle: the dense inverse on small
inputs, the closed-form inverses of the second-difference matrix and of a
pure arrowhead (diagonal plus one dense row), and exactly planted integer
inverses (unit lower-triangular integer L, so A^{-1} = L^{-T} L^{-1} is an
integer matrix and every step of the recursion is exact)."""
import numpy as np
import pytest

import oracle
from paper_2501_02483_amd import inputs as I


def _env(p, M):
    """Envelope entries (row-profile order) of a dense matrix."""
    rp = p.row_ptr()
    out = np.empty(rp[-1], dtype=M.dtype)
    for i in range(p.N):
        out[rp[i]:rp[i + 1]] = M[i, p.f[i]:i + 1]
    return out


def _selinv(p, vals):
    L, info = oracle.factor(p.f, vals)
    assert info == 0
    return oracle.selinv(p.f, L)


SHAPES = [
    # n, a, widths, seg
    (60, 5, 7, None),
    (200, 10, [3, 20, 9, 14], 50),
    (150, 0, 12, None),          # band only
    (40, 30, 0, None),           # diagonal plus a thick arrow
    (300, 16, 25, None),
    (97, 1, [0, 11, 4], 30),     # rows with no sub-diagonal entries
]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%d_a%d" % (s[0], s[1]))
def test_selinv_matches_dense_inverse(shape):
    n, a, w, seg = shape
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + 7 * a)
    S = _selinv(p, vals)
    ref = _env(p, np.linalg.inv(I.to_dense(p, vals)))
    assert np.linalg.norm(S - ref) / np.linalg.norm(ref) <= 1e-13


def test_selinv_second_difference_closed_form():
    """tridiag(-1, 2, -1) of order n: (A^{-1})_ij = i (n + 1 - j) / (n + 1)
    for 1-based i <= j."""
    n = 80
    p = I.make_pattern(n, 0, 1)
    rp = p.row_ptr()
    vals = np.empty(rp[-1])
    for i in range(n):
        seg = vals[rp[i]:rp[i + 1]]
        seg[-1] = 2.0
        if i > 0:
            seg[0] = -1.0
    S = _selinv(p, vals)
    i1 = np.arange(1, n + 1, dtype=np.float64)
    ref = np.minimum.outer(i1, i1) * (n + 1 - np.maximum.outer(i1, i1)) / (n + 1)
    assert np.max(np.abs(S - _env(p, ref)) / np.abs(_env(p, ref))) <= 1e-12


def test_selinv_pure_arrowhead_closed_form():
    """A = [[D, b], [b^T, c]] with D diagonal: with s = c - sum b_i^2 / d_i,
    (A^{-1})_nn = 1/s, (A^{-1})_ni = -(b_i/d_i)/s and
    (A^{-1})_ii = 1/d_i + (b_i/d_i)^2/s."""
    n = 64
    rng = np.random.default_rng(3)
    d = rng.uniform(1.0, 4.0, n)
    b = rng.standard_normal(n)
    c = float(np.sum(b * b / d)) + rng.uniform(0.5, 2.0)
    p = I.make_pattern(n, 1, 0)
    vals = np.concatenate([d, b, [c]])
    S = _selinv(p, vals)
    s = c - np.sum(b * b / d)
    u = b / d
    ref = np.concatenate([1.0 / d + u * u / s, -u / s, [1.0 / s]])
    assert np.max(np.abs(S - ref) / np.abs(ref)) <= 1e-13


def _planted_unit(n, a, w, seed, density):
    """Unit lower-triangular integer L inside the envelope (sparse entries in
    {-1, 1}); A = L L^T and A^{-1} = L^{-T} L^{-1}, both exact integers."""
    p = I.make_pattern(n, a, w)
    rng = np.random.default_rng(seed)
    N = p.N
    L = np.zeros((N, N), dtype=object)
    for i in range(N):
        L[i, i] = 1
        for j in range(p.f[i], i):
            if rng.random() < density:
                L[i, j] = int(rng.choice([-1, 1]))
    A = L.dot(L.T)
    # exact inverse of the unit lower-triangular L by forward substitution
    Li = np.zeros((N, N), dtype=object)
    for j in range(N):
        Li[j, j] = 1
        for i in range(j + 1, N):
            Li[i, j] = -sum(L[i, k] * Li[k, j] for k in range(j, i) if L[i, k] != 0)
    Sig = Li.T.dot(Li)
    return p, A, L, Sig


@pytest.mark.parametrize("n,a,w,seed,density", [(30, 3, 3, 1, 0.35), (45, 2, 5, 2, 0.2), (25, 6, 0, 3, 0.5)])
def test_selinv_planted_integer_inverse_is_exact(n, a, w, seed, density):
    p, A, L, Sig = _planted_unit(n, a, w, seed, density)
    big = max(abs(int(x)) for x in Sig.ravel())
    assert big < 2 ** 50, "planted inverse too large for exact FP64"
    vals = _env(p, A).astype(np.float64)
    Lf, info = oracle.factor(p.f, vals)
    assert info == 0
    assert np.array_equal(Lf, _env(p, L).astype(np.float64))
    S = oracle.selinv(p.f, Lf)
    assert np.array_equal(S, _env(p, Sig).astype(np.float64))   # bit-exact


def test_selinv_threads_do_not_change_the_result():
    p = I.make_pattern(400, 12, [5, 30, 17], seg=100)
    vals = I.make_values(p, seed=5)
    L, info = oracle.factor(p.f, vals)
    assert info == 0
    assert np.array_equal(oracle.selinv(p.f, L, nthreads=1), oracle.selinv(p.f, L, nthreads=4))
