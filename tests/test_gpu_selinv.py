"""Selected inversion on the GPU against the oracle's Takahashi recursion:
every selected entry (natural ordering: the whole envelope; adaptable ND: the
entries of the stored tiles, against the oracle run on P A P^T built by brute
force) and the diagonal of A^{-1} in the original ordering.  Bar: 1e-12
normwise relative for the entries, 1e-12 relative per diagonal entry (FP64
factor); 1e-5 for a mixed-precision factor, which is inverted as computed."""
import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import rel, say
from permute_util import permute_profile

pytestmark = pytest.mark.gpu

TOL = 1e-12
ND = S.STILES_ORDER_ADAPTABLE_ND


def _oracle_selinv(f, vals):
    L, info = oracle.factor(f, vals, nthreads=8)
    assert info == 0
    return oracle.selinv(f, L, nthreads=8)


def _diag_of(f, env):
    f = np.asarray(f)
    rp = np.concatenate([[0], np.cumsum(np.arange(len(f)) - f + 1)])
    return env[rp[1:] - 1]


def _stored_mask(sym, f):
    """Envelope entries (row-profile order of P A P^T) inside stored tiles."""
    h = sym.handle
    trow_ptr = S.stiles_symbolic_export(h, "trow_ptr")
    tcol = S.stiles_symbolic_export(h, "tcol")
    row_base = S.stiles_symbolic_export(h, "row_base")
    row_cnt = S.stiles_symbolic_export(h, "row_cnt")
    N = len(f)
    tile_of = np.empty(N, dtype=np.int64)
    for m in range(len(row_base)):
        tile_of[row_base[m]:row_base[m] + row_cnt[m]] = m
    stored = set()
    for m in range(len(trow_ptr) - 1):
        for t in range(trow_ptr[m], trow_ptr[m + 1]):
            stored.add((m, int(tcol[t])))
    lens = np.arange(N) - f + 1
    rows = np.repeat(np.arange(N), lens)
    rp = np.concatenate([[0], np.cumsum(lens)])
    cols = f[rows] + (np.arange(rp[-1]) - rp[rows])
    tr, tc = tile_of[rows], tile_of[cols]
    keys = tr * (len(row_base) + 1) + tc
    ok = np.array(sorted(a * (len(row_base) + 1) + b for a, b in stored))
    return np.isin(keys, ok)


NATURAL = [
    # n, arrow, widths, segment, tile
    (2000, 10, 50, None, 64),
    (3001, 33, [10, 120, 60], 400, 32),
    (1500, 0, 40, None, 64),
    (700, 70, 0, None, 32),
    (5000, 100, [30, 150, 80, 40], 600, 64),
]


@pytest.mark.parametrize("case", NATURAL, ids=lambda c: "n%d_a%d_T%d" % (c[0], c[1], c[4]))
def test_selinv_natural(case):
    import torch
    n, a, w, seg, T = case
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + a + T)
    ref = _oracle_selinv(p.f, vals)
    sym = S.Symbolic.from_pattern(p, tile=T, ordering=S.STILES_ORDER_NONE)
    say("[gpu selinv] natural n=%d a=%d T=%d" % (n, a, T))
    fac = S.Factor(sym)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    si = S.SelInv(fac).compute()
    env = si.extract().cpu().numpy()
    d = si.diag().cpu().numpy()
    e_env = rel(env, ref)
    d_ref = _diag_of(p.f, ref)
    e_d = np.max(np.abs(d - d_ref) / d_ref)
    say("   errors: entries %.2e  diagonal %.2e" % (e_env, e_d))
    assert e_env <= TOL and e_d <= TOL


ND_CASES = [
    # n, arrow, widths, segment, tile, parts
    (3000, 20, [20, 90, 40], 500, 64, 2),
    (3001, 33, [10, 120, 60], 400, 32, 3),
    (5000, 70, [30, 150, 80, 40], 600, 64, 0),
]


@pytest.mark.parametrize("case", ND_CASES, ids=lambda c: "n%d_a%d_T%d_P%d" % (c[0], c[1], c[4], c[5]))
def test_selinv_nd(case):
    import torch
    n, a, w, seg, T, parts = case
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + 5)
    sym = S.Symbolic.from_pattern(p, tile=T, ordering=ND, nd_parts=parts)
    assert sym.info.ordering_used == ND
    say("[gpu selinv] nd n=%d a=%d T=%d P=%d" % (n, a, T, sym.info.nd_parts))
    ref = _oracle_selinv(p.f, vals)
    f2, v2 = permute_profile(p.f, vals, sym.perm())
    ref2 = _oracle_selinv(f2, v2)
    fac = S.Factor(sym)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    si = S.SelInv(fac).compute()
    env = si.extract().cpu().numpy()
    mask = _stored_mask(sym, f2)
    e_env = rel(env[mask], ref2[mask])
    d = si.diag().cpu().numpy()
    d_ref = _diag_of(p.f, ref)
    e_d = np.max(np.abs(d - d_ref) / d_ref)
    say("   errors: stored entries %.2e  diagonal %.2e" % (e_env, e_d))
    assert e_env <= TOL and e_d <= TOL


def test_selinv_recompute_after_refactorization():
    """New values through the same handles: the second selected inverse is
    that of the new matrix (the executor's counters re-arm)."""
    import torch
    p = I.make_pattern(2500, 16, [12, 70], seg=500)
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=ND, nd_parts=2)
    fac = S.Factor(sym)
    si = S.SelInv(fac)
    say("[gpu selinv] recompute")
    for seed in (41, 42):
        vals = I.make_values(p, seed=seed)
        fac.factorize(torch.from_numpy(vals).cuda())
        si.compute()
        d = si.diag().cpu().numpy()
        d_ref = _diag_of(p.f, _oracle_selinv(p.f, vals))
        assert np.max(np.abs(d - d_ref) / d_ref) <= TOL


def test_selinv_csc_scrambled_band():
    """CSC input with partial RCM: the diagonal in the original ordering."""
    import torch
    from permute_util import profile_entries
    p = I.make_pattern(2500, 16, 30)
    vals = I.make_values(p, seed=12)
    ref = _diag_of(p.f, _oracle_selinv(p.f, vals))
    rng = np.random.default_rng(5)
    q = np.arange(p.N)
    q[:p.n] = rng.permutation(p.n)
    r, c, v = profile_entries(p.f, vals)
    rr, cc = q[r], q[c]
    hi, lo = np.maximum(rr, cc), np.minimum(rr, cc)
    order = np.lexsort((hi, lo))
    colptr = np.zeros(p.N + 1, dtype=np.int64)
    np.cumsum(np.bincount(lo, minlength=p.N), out=colptr[1:])
    sym = S.Symbolic.from_csc(p.N, p.a, colptr, hi[order].astype(np.int64), tile=32)
    assert sym.info.ordering_used == S.STILES_ORDER_PARTIAL_RCM
    say("[gpu selinv] csc scrambled band")
    fac = S.Factor(sym)
    fac.factorize(torch.from_numpy(np.ascontiguousarray(v[order])).cuda())
    assert fac.info() == 0
    d = S.SelInv(fac).compute().diag().cpu().numpy()
    assert np.max(np.abs(d[q] - ref) / ref) <= TOL


def test_selinv_mixed_precision_factor():
    import torch
    p = I.make_pattern(4000, 40, [30, 100], seg=800)
    vals = I.make_values(p, seed=21)
    d_ref = _diag_of(p.f, _oracle_selinv(p.f, vals))
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=ND, nd_parts=3)
    fac = S.Factor(sym, S.STILES_MIXED32)
    say("[gpu selinv] mixed-precision factor")
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    d = S.SelInv(fac).compute().diag().cpu().numpy()
    e = np.max(np.abs(d - d_ref) / d_ref)
    say("   diagonal error %.2e" % e)
    assert e <= 1e-5


def test_selinv_failed_factorization():
    """Not SPD: before the failure is known the diagonal is NaN; once
    stiles_factor_info has reported it, compute is refused (ESTATE)."""
    import torch
    p = I.make_pattern(2000, 10, 40)
    vals = I.make_values(p, seed=9)
    rp = p.row_ptr()
    vals[rp[1501] - 1] = -2.0
    sym = S.Symbolic.from_pattern(p, tile=64)
    fac = S.Factor(sym)
    si = S.SelInv(fac)
    say("[gpu selinv] non-SPD")
    fac.factorize(torch.from_numpy(vals).cuda())
    si.compute()
    assert torch.isnan(si.diag()).all()
    assert fac.info() > 0
    with pytest.raises(S.StilesError) as e:
        si.compute()
    assert e.value.status == S.STILES_ESTATE
