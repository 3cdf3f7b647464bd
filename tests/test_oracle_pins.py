"""Pins for the FP64 oracle against facts fixed by mathematics, independent of
the oracle's own code: LAPACK dense Cholesky, exactly planted integer factors,
closed-form determinants of arrowhead and Toeplitz-band matrices, solve
backward error, permutation invariance and the non-SPD failure index."""
import math

import numpy as np
import pytest

import oracle
from paper_2501_02483_amd import inputs as I


def _dense_L(pattern, L):
    N = pattern.N
    D = np.zeros((N, N))
    rp = pattern.row_ptr()
    for i in range(N):
        D[i, pattern.f[i]:i + 1] = L[rp[i]:rp[i + 1]]
    return D


SMALL = [
    (50, 3, 0),      # pure arrowhead (diagonal + arrow)
    (60, 0, 5),      # pure band, no arrow
    (80, 1, 7),      # single arrow row
    (200, 10, 13),
    (333, 17, 40),
    (129, 64, 64),
]


@pytest.mark.parametrize("n,a,w", SMALL)
def test_oracle_matches_lapack(n, a, w):
    p = I.make_pattern(n, a, w)
    v = I.make_values(p, seed=n + a + w)
    A = I.to_dense(p, v)
    Lref = np.linalg.cholesky(A)
    L, info = oracle.factor(p.f, v)
    assert info == 0
    Ld = _dense_L(p, L)
    err = np.linalg.norm(Ld - Lref) / np.linalg.norm(Lref)
    assert err <= 1e-13, err
    # LAPACK's factor is zero outside the envelope (envelope preservation)
    mask = np.zeros_like(A, dtype=bool)
    for i in range(p.N):
        mask[i, :p.f[i]] = True
    assert np.max(np.abs(Lref[mask]), initial=0.0) <= 1e-13 * np.max(np.abs(Lref))


def test_oracle_variable_profile_matches_lapack():
    p = I.make_pattern(400, 12, [3, 40, 9, 25], seg=100)
    v = I.make_values(p, seed=9)
    A = I.to_dense(p, v)
    L, info = oracle.factor(p.f, v)
    assert info == 0
    err = np.linalg.norm(_dense_L(p, L) - np.linalg.cholesky(A)) / np.linalg.norm(A)
    assert err <= 1e-13


def test_oracle_single_small_workload_full_lapack():
    """The full n=2,000 / w=50 / a=10 workload against dense LAPACK."""
    p = I.single_small()
    v = I.make_values(p, seed=1)
    A = I.to_dense(p, v)
    Lref = np.linalg.cholesky(A)
    L, info = oracle.factor(p.f, v, nthreads=4)
    assert info == 0
    err = np.linalg.norm(_dense_L(p, L) - Lref) / np.linalg.norm(Lref)
    assert err <= 1e-13, err
    ld = oracle.logdet(p.f, L)
    s, ld_ref = np.linalg.slogdet(A)
    assert s > 0 and abs(ld - ld_ref) <= 1e-12 * abs(ld_ref)


def _planted(n, a, w, seed):
    """Integer L inside the envelope, entries in {-1,0,1}, diagonal in 1..5;
    A = L L^T is formed exactly in integer arithmetic."""
    p = I.make_pattern(n, a, w)
    rng = np.random.default_rng(seed)
    N = p.N
    Lint = np.zeros((N, N), dtype=np.int64)
    for i in range(N):
        Lint[i, p.f[i]:i] = rng.integers(-1, 2, size=i - p.f[i])
        Lint[i, i] = rng.integers(1, 6)
    Aint = Lint @ Lint.T                     # exact (small integers)
    # Fill of L L^T stays inside the envelope (envelope preservation).
    rp = p.row_ptr()
    vals = np.empty(rp[-1])
    Lv = np.empty(rp[-1])
    for i in range(N):
        vals[rp[i]:rp[i + 1]] = Aint[i, p.f[i]:i + 1]
        Lv[rp[i]:rp[i + 1]] = Lint[i, p.f[i]:i + 1]
    return p, vals, Lv, Aint, Lint


@pytest.mark.parametrize("n,a,w,seed", [(40, 4, 3, 1), (150, 9, 12, 2), (90, 30, 0, 3), (200, 2, 31, 4)])
def test_planted_integer_factor_is_exact(n, a, w, seed):
    p, vals, Lv, Aint, Lint = _planted(n, a, w, seed)
    assert np.abs(Aint).max() < 2 ** 40
    L, info = oracle.factor(p.f, vals)
    assert info == 0
    assert np.array_equal(L, Lv)              # bit-exact: every step is exact
    ld = oracle.logdet(p.f, L)
    ld_exact = 2.0 * math.fsum(math.log(float(d)) for d in np.diag(Lint))
    assert abs(ld - ld_exact) <= 1e-14 * max(1.0, abs(ld_exact))
    # integer solution recovered
    rng = np.random.default_rng(seed + 100)
    x = rng.integers(-9, 10, size=p.N)
    b = (Aint @ x).astype(np.float64)
    xs = oracle.solve(p.f, L, b)
    cond = np.linalg.cond(Aint.astype(float))
    assert np.max(np.abs(xs - x)) <= 1e-14 * cond * max(1, np.abs(x).max())


@pytest.mark.parametrize("a", [1, 3])
def test_logdet_pure_arrowhead_closed_form(a):
    """Half-width 0: det A = prod d_i * det(C - Z^T D^{-1} Z)."""
    n = 3000
    p = I.make_pattern(n, a, 0)
    rng = np.random.default_rng(11)
    d = rng.uniform(1.0, 3.0, size=n)
    Z = rng.standard_normal((n, a)) * 0.1
    C = np.eye(a) * (1.0 + np.sum(Z * Z / d[:, None], axis=0).max() * 4) + 0.01 * np.ones((a, a))
    rp = p.row_ptr()
    vals = np.empty(rp[-1])
    vals[rp[:n]] = d
    for r in range(a):
        i = n + r
        vals[rp[i]:rp[i] + n] = Z[:, r]
        vals[rp[i] + n:rp[i + 1]] = C[r, :r + 1]
    S = C - Z.T @ (Z / d[:, None])
    if a == 1:
        ld_exact = math.fsum(np.log(d)) + math.log(float(S[0, 0]))
    else:
        sgn, lds = np.linalg.slogdet(S)
        assert sgn > 0
        ld_exact = math.fsum(np.log(d)) + lds
    L, info = oracle.factor(p.f, vals)
    assert info == 0
    ld = oracle.logdet(p.f, L)
    assert abs(ld - ld_exact) <= 1e-13 * abs(ld_exact)


@pytest.mark.parametrize("n", [2000, 100_000])
def test_logdet_toeplitz_band_eigenvector_arrow(n):
    """Tridiagonal Toeplitz band (delta, beta) with arrow columns that are
    scaled eigenvectors: logdet is known in closed form at any n."""
    delta, beta = 4.0, -1.3
    ks = [1, 7, n // 2]
    # scaled so that gamma^2 (n+1)/2 stays O(1): the Schur complement is positive
    gam = [g * math.sqrt(2.0 / (n + 1)) for g in (0.5, 0.25, 0.8)]
    Cd = [3.0, 2.0, 5.0]
    a = len(ks)
    p = I.make_pattern(n, a, 1)
    rp = p.row_ptr()
    vals = np.empty(rp[-1])
    vals[0] = delta
    vals[rp[1:n] ] = beta
    vals[rp[1:n] + 1] = delta
    idx = np.arange(1, n + 1)
    lam = lambda k: delta + 2 * beta * math.cos(k * math.pi / (n + 1))
    for c in range(a):
        i = n + c
        vals[rp[i]:rp[i] + n] = gam[c] * np.sin(idx * ks[c] * math.pi / (n + 1))
        vals[rp[i] + n:rp[i + 1] - 1] = 0.0
        vals[rp[i + 1] - 1] = Cd[c]
    ld_exact = math.fsum(math.log(lam(k)) for k in range(1, n + 1))
    for c in range(a):
        ld_exact += math.log(Cd[c] - gam[c] ** 2 * (n + 1) / (2 * lam(ks[c])))
    L, info = oracle.factor(p.f, vals)
    assert info == 0
    ld = oracle.logdet(p.f, L)
    assert abs(ld - ld_exact) <= 1e-12 * abs(ld_exact), (ld, ld_exact)


def test_solve_backward_error_and_lapack():
    p = I.make_pattern(1500, 20, 37)
    v = I.make_values(p, seed=5)
    A = I.to_dense(p, v)
    L, info = oracle.factor(p.f, v)
    B = I.rhs(p.N, 3, seed=6)
    X = oracle.solve(p.f, L, B)
    Xref = np.linalg.solve(A, B)
    assert np.linalg.norm(X - Xref) / np.linalg.norm(Xref) <= 1e-13
    u = 2.0 ** -53
    for c in range(3):
        r = B[:, c] - A @ X[:, c]
        be = np.linalg.norm(r) / (np.linalg.norm(A, 2) * np.linalg.norm(X[:, c]) + np.linalg.norm(B[:, c]))
        assert be <= 10 * (37 + 20) * u
    # symv agrees with the dense product
    assert np.allclose(oracle.symv(p.f, v, X), A @ X, rtol=1e-14, atol=1e-12)


def test_permutation_invariance_of_logdet_and_solution():
    """Reversing the band order (arrow kept last) changes L but not logdet or x."""
    n, a, w = 800, 6, 21
    p = I.make_pattern(n, a, w)
    v = I.make_values(p, seed=12)
    A = I.to_dense(p, v)
    perm = np.concatenate([np.arange(n)[::-1], np.arange(n, n + a)])
    Ap = A[np.ix_(perm, perm)]
    rp = p.row_ptr()
    vp = np.empty_like(v)
    for i in range(p.N):
        vp[rp[i]:rp[i + 1]] = Ap[i, p.f[i]:i + 1]   # reversed band keeps the same envelope
    assert np.allclose(I.to_dense(p, vp), Ap)
    L1, _ = oracle.factor(p.f, v)
    L2, _ = oracle.factor(p.f, vp)
    ld1, ld2 = oracle.logdet(p.f, L1), oracle.logdet(p.f, L2)
    assert abs(ld1 - ld2) <= 1e-12 * abs(ld1)
    b = I.rhs(p.N, 1, seed=13)[:, 0]
    x1 = oracle.solve(p.f, L1, b)
    x2p = oracle.solve(p.f, L2, b[perm])
    x2 = np.empty_like(x2p)
    x2[perm] = x2p
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) <= 1e-12


@pytest.mark.parametrize("bad", [0, 17, 403, 410])
def test_non_spd_reports_first_failing_column(bad):
    p = I.make_pattern(400, 12, 9)
    v = I.make_values(p, seed=3)
    rp = p.row_ptr()
    v[rp[bad + 1] - 1] = -1.0
    _, info = oracle.factor(p.f, v)
    assert info == bad + 1


def test_factor_residual_matches_dense():
    p = I.make_pattern(300, 8, 11)
    v = I.make_values(p, seed=4)
    L, _ = oracle.factor(p.f, v)
    A = I.to_dense(p, v)
    assert oracle.factor_residual(p.f, v, L) <= 1e-15
    # a planted perturbation: the residual function must agree with dense numpy
    rp = p.row_ptr()
    L2 = L.copy()
    L2[rp[150] + 3] += 1e-6
    L2[rp[p.N - 1] + 40] -= 2e-6
    Ld = _dense_L(p, L2)
    ref = np.linalg.norm(Ld @ Ld.T - A) / np.linalg.norm(A)
    got = oracle.factor_residual(p.f, v, L2)
    assert ref > 1e-9 and abs(got - ref) <= 1e-6 * ref
    # row subsets: the arrow rows alone see the second perturbation only
    rows = np.arange(p.n, p.N)
    assert oracle.factor_residual(p.f, v, L2, rows) > 1e-9


def test_generators_are_spd_and_seeded():
    p = I.make_pattern(300, 7, [5, 30, 12], seg=100)
    v1 = I.make_values(p, seed=21)
    v2 = I.make_values(p, seed=21)
    assert np.array_equal(v1, v2)
    A = I.to_dense(p, v1)
    assert np.linalg.eigvalsh(A).min() > 0.9          # dominance margin is 1
    vl = I.make_values(p, seed=22, law="laplacian", kappa=1e6)
    Al = I.to_dense(p, vl)
    ev = np.linalg.eigvalsh(Al)
    off = np.abs(Al).sum(axis=1) - np.abs(np.diag(Al))
    eps = 2 * off.max() / 1e6
    assert abs(ev.min() - eps) <= 1e-6 * eps + 1e-12
    assert ev.max() / ev.min() <= 1.01e6
