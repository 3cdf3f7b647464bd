"""Adaptable nested dissection in the host analysis (Section III-A): the
permutation keeps the arrow last and in order, the band partitions do not
couple to each other, the symbolic tile pattern covers the element-level fill
of P A P^T (dense boolean elimination), the envelope size matches a brute-
force permutation of the entries, and the algorithmic flop count does not
depend on the partitioning.  Host only (no GPU)."""
import numpy as np
import pytest

import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from permute_util import filled_lower, permute_profile, profile_entries

ND = S.STILES_ORDER_ADAPTABLE_ND


def _tile_of(g, n, T):
    return np.where(g < n, g // T, (n + T - 1) // T + (g - n) // T)


@pytest.mark.parametrize("n,a,w,seg,T,parts", [
    (700, 9, 20, None, 32, 2),
    (900, 12, [10, 40, 25], 150, 32, 3),
    (1100, 0, 30, None, 32, 4),
    (1300, 40, [5, 60], 200, 64, 0),
    (1000, 5, 12, None, 32, 5),
])
def test_nd_structure(n, a, w, seg, T, parts):
    p = I.make_pattern(n, a, w, seg=seg)
    base = S.Symbolic.from_pattern(p, tile=T)
    sym = S.Symbolic.from_pattern(p, tile=T, ordering=ND, nd_parts=parts)
    info = sym.info
    assert info.ordering_used == ND
    assert info.nd_parts >= 2
    if parts:
        assert info.nd_parts == parts
    N = p.N
    perm = sym.perm()
    assert np.array_equal(np.sort(perm), np.arange(N))
    # original arrow rows last, in order
    if a:
        assert np.array_equal(perm[N - a:], np.arange(n, N))
    nb = info.n          # band rows of P A P^T (the separators joined the arrow)
    assert nb < n and info.arrow == N - nb
    vals = I.make_values(p, seed=3)
    f2, v2 = permute_profile(p.f, vals, perm)
    assert info.nnz_L == int(np.sum(np.arange(N) - f2 + 1))
    assert info.flops_alg == base.info.flops_alg
    # partitions: maximal runs of band rows of P A P^T with no coupling between runs
    rows, cols, _ = profile_entries(p.f, vals)
    iperm = np.empty(N, dtype=np.int64)
    iperm[perm] = np.arange(N)
    pi, pj = iperm[rows], iperm[cols]
    hi, lo = np.maximum(pi, pj), np.minimum(pi, pj)
    # a band row's lower entries stay inside its partition: find partition starts
    # from the permutation (new rows whose original predecessor is not adjacent)
    starts = [0] + [q for q in range(1, nb) if abs(perm[q] - perm[q - 1]) != 1]
    assert len(starts) == info.nd_parts
    part_of = np.zeros(nb, dtype=np.int64)
    for k, s0 in enumerate(starts):
        part_of[s0:] = k
    band = hi < nb
    assert np.array_equal(part_of[hi[band]], part_of[lo[band]])
    # partitions before the last are whole tile rows
    for s0 in starts[1:]:
        assert s0 % T == 0
    # the symbolic tile pattern covers the element-level fill
    Lb = filled_lower(N, hi, lo)
    r, c = np.nonzero(Lb)
    need = set(zip(_tile_of(r, nb, T).tolist(), _tile_of(c, nb, T).tolist()))
    trow_ptr = S.stiles_symbolic_export(sym.handle, "trow_ptr")
    tcol = S.stiles_symbolic_export(sym.handle, "tcol")
    have = set()
    for m in range(len(trow_ptr) - 1):
        for t in range(trow_ptr[m], trow_ptr[m + 1]):
            have.add((m, int(tcol[t])))
    assert need <= have
    assert len(have) <= 1.1 * len(need) + 2


def test_nd_csc_matches_profile():
    """The CSC entry point reaches the same partitioning as the row-profile
    one when partial RCM brings no improvement."""
    p = I.make_pattern(1500, 20, [15, 50, 30], seg=300)
    vals = I.make_values(p, seed=1)
    colptr, rowind, _ = I.to_lower_csc(p, vals)
    s_csc = S.Symbolic.from_csc(p.N, p.a, colptr, rowind, tile=32, ordering=ND, nd_parts=3)
    s_prof = S.Symbolic.from_pattern(p, tile=32, ordering=ND, nd_parts=3)
    assert s_csc.info.ordering_used == ND
    assert np.array_equal(s_csc.perm(), s_prof.perm())
    assert s_csc.info.tiles == s_prof.info.tiles
    assert s_csc.info.nnz_L == s_prof.info.nnz_L


def test_nd_infeasible_falls_back():
    """Too short a band for two partitions: the ordering is not applied."""
    p = I.make_pattern(100, 4, 30)
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=ND, nd_parts=2)
    assert sym.info.ordering_used == S.STILES_ORDER_NONE
    assert sym.info.nd_parts == 1
    assert np.array_equal(sym.perm(), np.arange(p.N))
