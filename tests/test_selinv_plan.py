"""CPU checks of the selected-inversion plan through the C ABI (no GPU): the
SWE / SW / SDIAG task DAG, executed by the host emulator in ticket order and
in random topological orders on the emulated factor, reproduces the oracle's
selected inverse (natural order: every envelope entry; adaptable ND: the
diagonal in the original ordering and every stored entry against the dense
inverse)."""
import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

import dag_emulator as E

SHAPES = [
    # n, a, widths, seg, tile
    (300, 5, 7, None, 32),
    (700, 40, 60, None, 64),
    (1000, 0, 30, None, 32),
    (400, 70, 0, None, 32),
    (2000, 100, [10, 130, 40, 90], 500, 32),
]


def _dense_sigma(plan, sigma):
    """Dense symmetric Sigma (permuted order) on the stored tiles; NaN elsewhere."""
    D = np.full((plan.N, plan.N), np.nan)
    for t in range(len(plan.tcol)):
        m, j = plan.trow[t], plan.tcol[t]
        rb, cb, rc, cc = plan.row_base[m], plan.row_base[j], plan.row_cnt[m], plan.row_cnt[j]
        D[rb:rb + rc, cb:cb + cc] = sigma[t][:rc, :cc]
        D[cb:cb + cc, rb:rb + rc] = sigma[t][:rc, :cc].T
    return D


def _envelope(p, D):
    rp = p.row_ptr()
    out = np.empty(rp[-1])
    for i in range(p.N):
        out[rp[i]:rp[i + 1]] = D[i, p.f[i]:i + 1]
    return out


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%d_a%d_T%d" % (s[0], s[1], s[4]))
@pytest.mark.parametrize("mode", ["ticket", "random"])
def test_emulated_selinv_matches_oracle(shape, mode):
    n, a, w, seg, T = shape
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + 3 * a)
    sym = S.Symbolic.from_pattern(p, tile=T)
    plan = E.Plan(sym)
    tiles, linv = E.factor(plan, I.to_dense(p, vals), mode=mode, seed=n)
    sigma = E.selinv(plan, tiles, linv, mode=mode, seed=n + 2)
    L, info = oracle.factor(p.f, vals)
    assert info == 0
    ref = oracle.selinv(p.f, L)
    got = _envelope(p, _dense_sigma(plan, sigma))
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-12


@pytest.mark.parametrize("parts", [2, 3, 0])
def test_emulated_selinv_under_nd(parts):
    p = I.make_pattern(3000, 24, [20, 90, 45], seg=600)
    vals = I.make_values(p, seed=31)
    sym = S.Symbolic.from_pattern(p, tile=32, ordering=S.STILES_ORDER_ADAPTABLE_ND, nd_parts=parts)
    assert sym.info.nd_parts >= 2
    plan = E.Plan(sym)
    A = I.to_dense(p, vals)
    Ap = A[np.ix_(plan.perm, plan.perm)]
    tiles, linv = E.factor(plan, Ap, mode="random", seed=parts)
    sigma = E.selinv(plan, tiles, linv, mode="random", seed=parts + 5)
    D = _dense_sigma(plan, sigma)
    inv_p = np.linalg.inv(Ap)
    mask = ~np.isnan(D)
    assert np.linalg.norm(D[mask] - inv_p[mask]) / np.linalg.norm(inv_p[mask]) <= 1e-12
    # the diagonal in the original ordering against the oracle
    L, info = oracle.factor(p.f, vals)
    assert info == 0
    Sg = oracle.selinv(p.f, L)
    rp = p.row_ptr()
    d_ref = Sg[rp[1:] - 1]
    d = np.empty(p.N)
    d[plan.perm] = np.diag(D)
    assert np.max(np.abs(d - d_ref) / d_ref) <= 1e-12


def test_selinv_plan_counts():
    """One SW task per off-diagonal tile, one SDIAG per tile column; the
    algorithmic count is sum_j 2 eta_j (eta_j + 1) over the envelope."""
    p = I.make_pattern(900, 20, 40)
    sym = S.Symbolic.from_pattern(p, tile=32)
    plan = E.Plan(sym)
    itask, _, _ = plan.selinv_tables()
    types = itask[:, 0] & 0xff
    assert np.sum(types == E.SW) == len(plan.tcol) - plan.ntr
    assert np.sum(types == E.SDIAG) == plan.ntr
    ntasks, falg, fexec = S.stiles_selinv_query(sym.handle)
    assert ntasks == len(itask)
    eta = np.zeros(p.N, dtype=np.int64)
    for i in range(p.N):
        eta[p.f[i]:i] += 1
    assert falg == pytest.approx(float(np.sum(2.0 * eta * (eta + 1.0))), rel=1e-15)
    assert fexec >= falg
