"""The parity metrics of the GPU tests, checked on the CPU: the per-tile-
column factor error must see an error confined to one block column that the
normwise error of the whole factor dilutes, and must agree with the same
quantity computed on dense matrices."""
import numpy as np

from paper_2501_02483_amd import inputs as I

from gpu_util import col_tile_err, rel, rel_cols


def _dense_lower(f, v):
    N = f.shape[0]
    D = np.zeros((N, N))
    rp = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.arange(N) - f + 1, out=rp[1:])
    for i in range(N):
        D[i, f[i]:i + 1] = v[rp[i]:rp[i + 1]]
    return D


def test_col_tile_err_matches_dense_definition():
    p = I.make_pattern(300, 7, [5, 40, 12], seg=60)
    rng = np.random.default_rng(3)
    Lo = rng.standard_normal(p.nnz)
    L = Lo * (1 + 1e-9 * rng.standard_normal(p.nnz))
    T = 32
    Do, D = _dense_lower(p.f, Lo), _dense_lower(p.f, L)
    want = max(np.linalg.norm((D - Do)[:, k:k + T]) / np.linalg.norm(Do[:, k:k + T])
               for k in range(0, p.N, T) if np.linalg.norm(Do[:, k:k + T]) > 0)
    assert abs(col_tile_err(L, Lo, p.f, T) - want) <= 1e-12 * want


def test_col_tile_err_sees_one_bad_block_column():
    p = I.make_pattern(2000, 10, 50)
    rng = np.random.default_rng(4)
    Lo = rng.standard_normal(p.nnz)
    L = Lo.copy()
    D = _dense_lower(p.f, np.arange(p.nnz, dtype=np.float64))
    # perturb every stored entry of columns 640..703 (tile column 10 at T = 64)
    idx = D[:, 640:704][D[:, 640:704] > 0].astype(np.int64)
    idx = np.concatenate([idx, D[640:704, 640:704].diagonal().astype(np.int64)])
    L[idx] *= 1 + 1e-10
    whole = rel(L, Lo)
    col = col_tile_err(L, Lo, p.f, 64)
    assert col > 0.9e-10 and whole < 0.3 * col


def test_rel_cols_takes_the_worst_column():
    X = np.ones((100, 3))
    Y = X.copy()
    Y[:, 1] *= 1 + 1e-8
    assert abs(rel_cols(Y, X) - 1e-8) < 1e-12
    assert rel(Y, X) < rel_cols(Y, X)
