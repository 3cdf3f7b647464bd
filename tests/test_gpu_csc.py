"""The CSC entry point on the GPU (value map scatter): natural order, a
scrambled band that partial RCM recovers, adaptable ND, and a pattern that is
sparse inside its envelope.  Solutions and log-determinants do not depend on
the ordering, so they are compared with the oracle on the unscrambled
matrix; bar 1e-12 normwise relative."""
import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import rel, say, to_device_cols
from permute_util import profile_entries

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _csc(N, rows, cols, vals):
    """Lower CSC (diagonal first, rows ascending) from lower entries."""
    order = np.lexsort((rows, cols))
    colptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(cols, minlength=N), out=colptr[1:])
    return colptr, rows[order].astype(np.int64), np.ascontiguousarray(vals[order])


def _oracle(p, vals, B):
    L, info = oracle.factor(p.f, vals, nthreads=8)
    assert info == 0
    return oracle.logdet(p.f, L), oracle.solve(p.f, L, B)


def _run(N, a, colptr, rowind, cvals, B, **opt):
    import torch
    sym = S.Symbolic.from_csc(N, a, colptr, rowind, **opt)
    fac = S.Factor(sym, nrhs_max=B.shape[1])
    fac.factorize(torch.from_numpy(cvals).cuda())
    assert fac.info() == 0
    ld = fac.logdet().item()
    dB = to_device_cols(B)
    fac.solve(dB)
    return sym, ld, dB.cpu().numpy()


@pytest.mark.parametrize("ordering,parts", [(S.STILES_ORDER_AUTO, 0), (S.STILES_ORDER_ADAPTABLE_ND, 3)])
def test_csc_natural_and_nd(ordering, parts):
    p = I.make_pattern(3000, 24, [20, 90, 45], seg=600)
    vals = I.make_values(p, seed=31)
    B = I.rhs(p.N, 3, seed=8)
    ld_o, X_o = _oracle(p, vals, B)
    colptr, rowind, cvals = I.to_lower_csc(p, vals)
    say("[gpu csc] ordering %d parts %d" % (ordering, parts))
    sym, ld, X = _run(p.N, p.a, colptr, rowind, cvals, B, tile=64, ordering=ordering, nd_parts=parts)
    if ordering == S.STILES_ORDER_ADAPTABLE_ND:
        assert sym.info.nd_parts == parts
    assert rel(X, X_o) <= TOL
    assert abs(ld - ld_o) <= TOL * abs(ld_o)


@pytest.mark.parametrize("ordering", [S.STILES_ORDER_AUTO, S.STILES_ORDER_ADAPTABLE_ND])
def test_csc_scrambled_band_recovered(ordering):
    """A band matrix under a random symmetric permutation of its band rows:
    partial RCM brings the band back (fewer tiles), and the results match
    the oracle of the unscrambled matrix."""
    p = I.make_pattern(2500, 16, 30)
    vals = I.make_values(p, seed=12)
    B = I.rhs(p.N, 2, seed=3)
    ld_o, X_o = _oracle(p, vals, B)
    rng = np.random.default_rng(5)
    q = np.arange(p.N)
    q[:p.n] = rng.permutation(p.n)          # old index -> scrambled index (arrow kept last)
    r, c, v = profile_entries(p.f, vals)
    rr, cc = q[r], q[c]
    hi, lo = np.maximum(rr, cc), np.minimum(rr, cc)
    colptr, rowind, cvals = _csc(p.N, hi, lo, v)
    Bs = np.empty_like(B)
    Bs[q] = B
    say("[gpu csc] scrambled band, ordering %d" % ordering)
    sym, ld, Xs = _run(p.N, p.a, colptr, rowind, cvals, Bs, tile=32, ordering=ordering)
    assert sym.info.ordering_used in (S.STILES_ORDER_PARTIAL_RCM, S.STILES_ORDER_ADAPTABLE_ND)
    X = Xs[q]
    assert rel(X, X_o) <= TOL
    assert abs(ld - ld_o) <= TOL * abs(ld_o)


def test_csc_sparse_inside_envelope():
    """Entries missing inside the envelope (fill appears in L): the factor
    still matches the oracle, which stores the envelope with explicit zeros."""
    p = I.make_pattern(2000, 12, 60)
    rng = np.random.default_rng(9)
    r, c, _ = profile_entries(p.f, np.zeros(p.nnz))
    off = r != c
    keep = ~off | (rng.random(p.nnz) < 0.6)
    r, c = r[keep], c[keep]
    v = np.where(r == c, 0.0, rng.standard_normal(len(r)))
    # diagonal dominance on the kept entries: |row| + |column| sums + 1
    d = np.zeros(p.N)
    np.add.at(d, r[r != c], np.abs(v[r != c]))
    np.add.at(d, c[r != c], np.abs(v[r != c]))
    v[r == c] = d[r[r == c]] + 1.0
    # the oracle's envelope values: zeros where entries were dropped
    rp = p.row_ptr()
    env = np.zeros(p.nnz)
    env[rp[r] + (c - p.f[r])] = v
    B = I.rhs(p.N, 2, seed=4)
    ld_o, X_o = _oracle(p, env, B)
    colptr, rowind, cvals = _csc(p.N, r, c, v)
    say("[gpu csc] sparse inside the envelope")
    sym, ld, X = _run(p.N, p.a, colptr, rowind, cvals, B, tile=64, ordering=S.STILES_ORDER_NONE)
    assert rel(X, X_o) <= TOL
    assert abs(ld - ld_o) <= TOL * abs(ld_o)


@pytest.mark.parametrize("T", [32, 64])
def test_csc_amd_order_on_a_poor_mesh(T):
    """An irregular mesh with long-range couplings, numbered at random: the
    approximate minimum degree order is kept (fewer tiles than the input
    order and than partial RCM).  L matches the oracle's factor of P A P^T
    (per tile column), X and logdet the oracle of the same matrix."""
    import torch
    from gpu_util import col_tile_err
    m = I.irregular_mesh(20000, 50, seed=1, long_edges=100)
    N, a = m["N"], m["a"]
    sym = S.Symbolic.from_csc(N, a, m["colptr"], m["rowind"], tile=T, ordering=S.STILES_ORDER_AMD)
    rcm = S.Symbolic.from_csc(N, a, m["colptr"], m["rowind"], tile=T, ordering=S.STILES_ORDER_PARTIAL_RCM)
    say("[gpu csc] AMD order, irregular mesh N=%d T=%d: %d tiles (partial RCM %d)" % (
        N, T, sym.info.tiles, rcm.info.tiles))
    assert sym.info.ordering_used == S.STILES_ORDER_AMD and sym.info.tiles < rcm.info.tiles
    perm = np.array(sym.perm())
    # oracle on the envelope of P A P^T, built from the entries of A
    iperm = np.empty(N, dtype=np.int64)
    iperm[perm] = np.arange(N)
    c = iperm[np.repeat(np.arange(N), np.diff(m["colptr"]))]
    r = iperm[m["rowind"]]
    hi, lo = np.maximum(r, c), np.minimum(r, c)
    f2 = np.arange(N, dtype=np.int64)
    np.minimum.at(f2, hi, lo)
    rp = np.concatenate([[0], np.cumsum(np.arange(N) - f2 + 1)])
    v2 = np.zeros(int(rp[-1]))
    v2[rp[hi] + (lo - f2[hi])] = m["values"]
    L_o, info = oracle.factor(f2, v2, nthreads=8)
    assert info == 0
    B = I.rhs(N, 3, seed=21)
    X_o = np.empty_like(B)
    X_o[perm] = oracle.solve(f2, L_o, B[perm])
    ld_o = oracle.logdet(f2, L_o)
    fac = S.Factor(sym, nrhs_max=3)
    fac.factorize(torch.from_numpy(m["values"]).cuda())
    assert fac.info() == 0
    eL = col_tile_err(fac.extract().cpu().numpy(), L_o, f2, T)
    dB = to_device_cols(B)
    fac.solve(dB)
    ld = fac.logdet().item()
    say("   errors: L per tile column %.2e  X %.2e  logdet %.2e" % (
        eL, rel(dB.cpu().numpy(), X_o), abs(ld - ld_o) / abs(ld_o)))
    assert eL <= TOL
    assert rel(dB.cpu().numpy(), X_o) <= TOL
    assert abs(ld - ld_o) <= TOL * abs(ld_o)
