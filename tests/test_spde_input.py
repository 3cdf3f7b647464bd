"""The spatio-temporal (SPDE-shaped) generator and its analysis on the host:
the pattern is the stated stencil (lower triangle, no duplicates, diagonal
first in each column), the matrix is SPD, the row profile holds the same
matrix as the CSC arrays, and the C ABI analyzes it with every ordering."""
import numpy as np
import pytest

import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I


def _dense_csc(g):
    N = g["N"]
    A = np.zeros((N, N))
    cp, ri, v = g["colptr"], g["rowind"], g["values"]
    for j in range(N):
        A[ri[cp[j]:cp[j + 1]], j] = v[cp[j]:cp[j + 1]]
    return np.tril(A) + np.tril(A, -1).T


def test_spde_pattern_structure_and_spd():
    nx, ny, nt, a = 7, 6, 5, 4
    g = I.spde_space_time(nx, ny, nt, a, seed=3)
    N, n = g["N"], g["n"]
    cp, ri = g["colptr"], g["rowind"]
    cols = np.repeat(np.arange(N), np.diff(cp))
    assert len(set(zip(ri.tolist(), cols.tolist()))) == len(ri)
    assert np.all(ri >= cols)
    assert np.all(ri[cp[:-1]] == np.arange(N))          # diagonal first in each column
    A = _dense_csc(g)
    assert np.array_equal(A, I.to_dense(g["pattern"], g["profile_values"]))
    assert np.all(np.linalg.eigvalsh(A) > 0)
    # an interior node of an interior time step: 13-point stencil at t-1, t, t+1
    t, yy, xx = 2, 3, 3
    i = t * nx * ny + yy * nx + xx
    nb = set(np.nonzero(A[i, :n])[0].tolist()) - {i}
    expect = set()
    for dt in (-1, 0, 1):
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                if abs(dx) + abs(dy) <= 2 and (dt, dy, dx) != (0, 0, 0):
                    expect.add((t + dt) * nx * ny + (yy + dy) * nx + (xx + dx))
    assert nb == expect
    assert np.all(A[i, n:] != 0)                          # coupled to every arrow row


@pytest.mark.parametrize("ordering", [S.STILES_ORDER_AUTO, S.STILES_ORDER_NONE, S.STILES_ORDER_ADAPTABLE_ND])
def test_spde_analyze(ordering):
    g = I.spde_space_time(14, 12, 9, 6, seed=4)
    sym = S.Symbolic.from_csc(g["N"], g["a"], g["colptr"], g["rowind"], tile=32, ordering=ordering)
    info = sym.info
    assert info.N == g["N"]
    p = np.sort(sym.perm())
    assert np.array_equal(p, np.arange(g["N"]))
    # the work of the natural envelope is what the rate counts
    assert info.flops_alg > 0 and info.flops_exec >= info.flops_alg * 0.5
    if ordering == S.STILES_ORDER_ADAPTABLE_ND:
        assert info.nd_parts >= 2
