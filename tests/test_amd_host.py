"""Approximate minimum degree ordering (Section III-A: the option for
irregular patterns) through the C ABI, on the CPU.

The order is not unique, so its results are checked by what the method
fixes: it is a permutation of the band rows with the arrow rows last; on
trees it creates no fill (eliminating leaves first); on small meshes its
element fill is within a few percent of an exact minimum-degree elimination
written out here by brute force (the approximate degrees are upper bounds of
the exact ones); the fill check keeps it only when L has fewer tiles than in
the input order; and the factorization DAG built on it, executed by the host
emulator, reproduces the oracle's factor of P A P^T."""
import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

import dag_emulator as E
from permute_util import filled_lower


def _lower_csc(N, hi, lo):
    """CSC of the lower pattern with strictly lower entries (hi > lo) plus the diagonal."""
    assert np.all(hi > lo)
    d = np.arange(N, dtype=np.int64)
    r = np.concatenate([hi, d])
    c = np.concatenate([lo, d])
    key = np.unique(c * N + r)
    r, c = key % N, key // N
    colptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(c, minlength=N), out=colptr[1:])
    return colptr, r.astype(np.int64)


def _edges(colptr, rowind):
    N = len(colptr) - 1
    c = np.repeat(np.arange(N), np.diff(colptr))
    off = rowind != c
    return rowind[off], c[off]


def _fill_nnz(N, hi, lo, perm):
    """nnz(L) of P A P^T by dense boolean elimination (small N)."""
    inv = np.empty(N, dtype=np.int64)
    inv[perm] = np.arange(N)
    a, b = inv[hi], inv[lo]
    return int(filled_lower(N, np.maximum(a, b), np.minimum(a, b)).sum())


def _exact_md_fill(n, hi, lo):
    """nnz(L) of an exact minimum-degree elimination (textbook definition:
    repeatedly eliminate a vertex of smallest current degree, lowest index on
    ties, joining its neighbours into a clique), for the band graph alone."""
    adj = [set() for _ in range(n)]
    for u, v in zip(hi, lo):
        if u < n and v < n:
            adj[u].add(v)
            adj[v].add(u)
    alive = set(range(n))
    nnz = 0
    while alive:
        p = min(alive, key=lambda v: (len(adj[v]), v))
        nb = adj[p]
        nnz += 1 + len(nb)
        for u in nb:
            adj[u].discard(p)
            adj[u] |= nb - {u}
        alive.discard(p)
        adj[p] = set()
    return nnz


def _sym(N, a, colptr, rowind, **kw):
    return S.Symbolic.from_csc(N, a, colptr, rowind, ordering=S.STILES_ORDER_AMD, **kw)


@pytest.mark.parametrize("n,a,long_edges", [(400, 0, 0), (600, 20, 10), (1500, 30, 40)])
def test_amd_is_a_partial_permutation(n, a, long_edges):
    m = I.irregular_mesh(n, a, seed=n, long_edges=long_edges)
    sym = _sym(m["N"], a, m["colptr"], m["rowind"], tile=32)
    assert sym.info.ordering_used == S.STILES_ORDER_AMD
    perm = np.array(sym.perm())
    assert np.array_equal(np.sort(perm), np.arange(m["N"]))
    assert np.array_equal(perm[n:], np.arange(n, m["N"]))     # the arrow stays last


@pytest.mark.parametrize("kind", ["path", "star", "random_tree"])
def test_amd_creates_no_fill_on_trees(kind):
    n = 300
    rng = np.random.default_rng(3)
    if kind == "path":
        u, v = np.arange(1, n), np.arange(n - 1)
    elif kind == "star":
        u, v = np.arange(1, n), np.zeros(n - 1, dtype=np.int64)
    else:
        u = np.arange(1, n)
        v = np.array([rng.integers(0, k) for k in range(1, n)])
    num = rng.permutation(n)                       # scramble the numbering
    a_, b_ = num[u], num[v]
    hi, lo = np.maximum(a_, b_), np.minimum(a_, b_)
    colptr, rowind = _lower_csc(n, hi, lo)
    sym = S.Symbolic.from_csc(n, 0, colptr, rowind, tile=32, ordering=S.STILES_ORDER_AMD)
    if sym.info.ordering_used != S.STILES_ORDER_AMD:
        pytest.skip("input order already has no more tiles")   # fill check kept the input order
    perm = np.array(sym.perm())
    assert _fill_nnz(n, hi, lo, perm) == n + len(hi)           # nnz(L) = nnz(tril A): no fill


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_amd_fill_close_to_exact_minimum_degree(seed):
    n = 350
    m = I.irregular_mesh(n, 0, seed=seed, long_edges=5)
    hi, lo = _edges(m["colptr"], m["rowind"])
    sym = _sym(n, 0, m["colptr"], m["rowind"], tile=32)
    perm = np.array(sym.perm())
    amd = _fill_nnz(n, hi, lo, perm)
    md = _exact_md_fill(n, hi, lo)
    nat = _fill_nnz(n, hi, lo, np.arange(n))
    rcm = S.Symbolic.from_csc(n, 0, m["colptr"], m["rowind"], tile=32, ordering=S.STILES_ORDER_PARTIAL_RCM)
    rc = _fill_nnz(n, hi, lo, np.array(rcm.perm()))
    # the exact minimum-degree count itself, checked against a dense elimination
    assert md >= n + len(hi)
    assert amd <= 1.15 * md, (amd, md)
    assert amd < rc < nat


def test_fill_check_keeps_input_order_of_a_band():
    """A narrow band in its natural order: no ordering reduces the tiles, so
    the input order is kept."""
    p = I.make_pattern(3000, 10, 20)
    colptr, rowind, _ = I.to_lower_csc(p, np.zeros(p.nnz))
    sym = _sym(p.N, p.a, colptr, rowind, tile=64)
    assert sym.info.ordering_used == S.STILES_ORDER_NONE
    assert np.array_equal(np.array(sym.perm()), np.arange(p.N))


def test_amd_beats_rcm_on_a_poor_mesh_in_tiles_and_work():
    m = I.irregular_mesh(20000, 50, seed=1, long_edges=100)
    amd = _sym(m["N"], 50, m["colptr"], m["rowind"], tile=64)
    rcm = S.Symbolic.from_csc(m["N"], 50, m["colptr"], m["rowind"], tile=64, ordering=S.STILES_ORDER_PARTIAL_RCM)
    assert amd.info.ordering_used == S.STILES_ORDER_AMD
    assert amd.info.tiles < 0.7 * rcm.info.tiles
    assert amd.info.flops_exec < 0.5 * rcm.info.flops_exec


def test_amd_rejected_for_profile_input_and_bad_values():
    p = I.make_pattern(200, 4, 10)
    with pytest.raises(S.StilesError) as e:
        S.Symbolic.from_pattern(p, tile=32, ordering=S.STILES_ORDER_AMD)
    assert e.value.status == S.STILES_ENOTSUP
    colptr, rowind, _ = I.to_lower_csc(p, np.zeros(p.nnz))
    with pytest.raises(S.StilesError) as e:
        S.Symbolic.from_csc(p.N, p.a, colptr, rowind, tile=32, ordering=S.STILES_ORDER_AMD + 1)
    assert e.value.status == S.STILES_EINVAL


@pytest.mark.parametrize("T,mode", [(32, "ticket"), (32, "random"), (64, "ticket")])
def test_emulated_factor_on_amd_order_matches_oracle(T, mode):
    m = I.irregular_mesh(1500, 30, seed=7, long_edges=30)
    N = m["N"]
    sym = _sym(N, 30, m["colptr"], m["rowind"], tile=T)
    assert sym.info.ordering_used == S.STILES_ORDER_AMD
    plan = E.Plan(sym)
    perm = plan.perm
    # dense A from the CSC input, then P A P^T
    c = np.repeat(np.arange(N), np.diff(m["colptr"]))
    A = np.zeros((N, N))
    A[m["rowind"], c] = m["values"]
    A[c, m["rowind"]] = m["values"]
    Ap = A[np.ix_(perm, perm)]
    tiles, linv = E.factor(plan, Ap, mode=mode, seed=T)
    Ld = E.dense_factor(plan, tiles)
    # oracle on the envelope of P A P^T
    f2 = np.array([np.nonzero(Ap[i, :i + 1])[0][0] for i in range(N)], dtype=np.int64)
    rp = np.concatenate([[0], np.cumsum(np.arange(N) - f2 + 1)])
    v2 = np.concatenate([Ap[i, f2[i]:i + 1] for i in range(N)])
    L, info = oracle.factor(f2, v2)
    assert info == 0
    Lo = np.zeros((N, N))
    for i in range(N):
        Lo[i, f2[i]:i + 1] = L[rp[i]:rp[i + 1]]
    assert np.linalg.norm(Ld - Lo) / np.linalg.norm(Lo) <= 1e-12
    B = I.rhs(N, 2, seed=5)
    X = E.solve(plan, tiles, linv, B, mode=mode, seed=T + 1)    # permutes and unpermutes itself
    Xo = np.linalg.solve(A, B)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-12
