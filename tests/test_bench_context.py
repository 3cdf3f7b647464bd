"""bench.py's LAPACK context row (band Cholesky through scipy plus the arrow
by blocked substitution), checked on the CPU: its log-determinant equals
that of the dense matrix, also with the last row block shorter than the
half-width and with a half-width of n - 1 (one block)."""
import os
import sys

import numpy as np
import pytest

from paper_2501_02483_amd import inputs as I

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


@pytest.mark.parametrize("n,a,w", [(2000, 10, 50), (3001, 7, 130), (500, 3, 499), (64, 1, 1)])
def test_lapack_context_logdet_matches_dense(n, a, w):
    pytest.importorskip("scipy")
    p = I.make_pattern(n, a, w)
    v = I.make_values(p, seed=n + a)
    r = bench.lapack_banded(p, v)
    assert r["w"] == w
    _, ld = np.linalg.slogdet(I.to_dense(p, v))
    assert abs(r["logdet"] - ld) <= 1e-12 * abs(ld)
