"""stiles_factorize_solve: factorization and solve as one launch of the
merged task graph.  The factor, the solution and the log-determinant must be
bitwise those of stiles_factorize + stiles_solve (same tasks, same
accumulation orders), and match the oracle within 1e-12."""
import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import oracle_reference, rel, say, to_device_cols

pytestmark = pytest.mark.gpu

CASES = [
    # n, arrow, widths, segment, tile, ordering, parts, nrhs
    (3000, 20, [20, 90, 40], 500, 64, S.STILES_ORDER_NONE, 0, 1),
    (3001, 33, [10, 120, 60], 400, 32, S.STILES_ORDER_NONE, 0, 8),
    (5000, 70, [30, 150, 80, 40], 600, 64, S.STILES_ORDER_ADAPTABLE_ND, 0, 8),
    (4000, 0, 50, None, 64, S.STILES_ORDER_ADAPTABLE_ND, 3, 16),
    (2500, 100, [8, 60], 250, 32, S.STILES_ORDER_ADAPTABLE_ND, 5, 20),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_T%d_o%d_P%d_r%d" % (c[0], c[4], c[5], c[6], c[7]))
def test_factorize_solve_matches_separate_calls(case):
    import torch
    n, a, w, seg, T, ordering, parts, nrhs = case
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + T)
    B = I.rhs(p.N, nrhs, seed=13)
    ref = oracle_reference(p, vals, B)
    sym = S.Symbolic.from_pattern(p, tile=T, ordering=ordering, nd_parts=parts)
    say("[gpu factorize_solve] n=%d T=%d ordering %d P=%d nrhs %d" % (n, T, ordering, sym.info.nd_parts, nrhs))
    dv = torch.from_numpy(vals).cuda()
    one = S.Factor(sym, nrhs_max=nrhs)
    one.factorize(dv)
    X1 = to_device_cols(B)
    one.solve(X1)
    both = S.Factor(sym, nrhs_max=nrhs)
    X2 = to_device_cols(B)
    both.factorize_solve(dv, X2)
    assert both.info() == 0
    assert torch.equal(X1, X2)
    assert torch.equal(one.logdet(), both.logdet())
    if ordering == S.STILES_ORDER_NONE:
        assert torch.equal(one.extract(), both.extract())
    eX = rel(X2.cpu().numpy(), ref["X"])
    say("   X error %.2e" % eX)
    assert eX <= 1e-12
    # the same workspace again (counters re-armed), new values
    vals2 = I.make_values(p, seed=n + T + 1)
    X3 = to_device_cols(B)
    both.factorize_solve(torch.from_numpy(vals2).cuda(), X3)
    ref2 = oracle_reference(p, vals2, B)
    assert rel(X3.cpu().numpy(), ref2["X"]) <= 1e-12


def test_factorize_solve_failure_and_mixed():
    import torch
    p = I.make_pattern(2000, 10, 40)
    vals = I.make_values(p, seed=9)
    rp = p.row_ptr()
    vals[rp[1501] - 1] = -2.0
    sym = S.Symbolic.from_pattern(p, tile=64)
    fac = S.Factor(sym)
    b = torch.ones(p.N, dtype=torch.float64, device="cuda")
    say("[gpu factorize_solve] non-SPD and mixed precision")
    fac.factorize_solve(torch.from_numpy(vals).cuda(), b)
    assert fac.info() > 0
    assert torch.isnan(b).all()
    mixed = S.Factor(sym, S.STILES_MIXED32)
    b = torch.ones(p.N, dtype=torch.float64, device="cuda")
    mixed.factorize_solve(torch.from_numpy(vals).cuda(), b)
    assert mixed.info() == fac.info()
    assert torch.isnan(b).all()


@pytest.mark.parametrize("ordering,nrhs", [(S.STILES_ORDER_NONE, 3), (S.STILES_ORDER_ADAPTABLE_ND, 20)],
                         ids=["natural_r3", "nd_r20"])
def test_mixed_factorize_solve_matches_separate_calls(ordering, nrhs):
    """Mixed precision in one launch: the merged launch's solve is the first
    iterate of the FP64 refinement; the refined X is bitwise that of
    stiles_factorize + stiles_solve (right-hand sides beyond 16 included)
    and matches the oracle."""
    import torch
    p = I.make_pattern(8000, 40, [30, 160, 90], seg=900)
    vals = I.make_values(p, seed=21)
    B = I.rhs(p.N, nrhs, seed=22)
    ref = oracle_reference(p, vals, B)
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=ordering)
    say("[gpu factorize_solve] mixed precision, ordering %d, %d RHS" % (ordering, nrhs))
    dv = torch.from_numpy(vals).cuda()
    one = S.Factor(sym, S.STILES_MIXED32, nrhs_max=nrhs)
    one.factorize(dv)
    X1 = to_device_cols(B)
    rep = one.solve(X1)
    assert rep.converged == 1
    both = S.Factor(sym, S.STILES_MIXED32, nrhs_max=nrhs)
    X2 = to_device_cols(B)
    both.factorize_solve(dv, X2)
    assert both.info() == 0
    assert torch.equal(X1, X2)
    eX = rel(X2.cpu().numpy(), ref["X"])
    say("   X error %.2e" % eX)
    assert eX <= 1e-12


def test_ticket_order_does_not_change_results():
    """The ticket order (sched_workers: list schedule on 512 or 64 workgroups,
    or the earliest-start order) changes only the speed: factor, merged
    solve and log-determinant are bitwise equal across orders."""
    import torch
    p = I.make_pattern(6000, 40, [20, 110, 50], seg=700)
    vals = I.make_values(p, seed=77)
    B = I.rhs(p.N, 4, seed=78)
    dv = torch.from_numpy(vals).cuda()
    out = []
    for sw in (0, -1, 64):
        sym = S.Symbolic.from_pattern(p, tile=64, ordering=S.STILES_ORDER_ADAPTABLE_ND, nd_parts=4, sched_workers=sw)
        say("[gpu ticket order] sched_workers=%d" % sw)
        fac = S.Factor(sym, nrhs_max=4)
        X = to_device_cols(B)
        fac.factorize_solve(dv, X)
        ld = fac.logdet().item()
        assert fac.info() == 0
        out.append((fac.extract().cpu().numpy(), X.cpu().numpy(), ld))
    for L, X, ld in out[1:]:
        assert np.array_equal(L, out[0][0]) and np.array_equal(X, out[0][1]) and ld == out[0][2]


def test_merged_trace_records_every_task():
    """stiles_factor_set_merged_trace: one record per task of the merged DAG,
    start >= claim and end >= start, task type in the record."""
    import torch
    p = I.make_pattern(3000, 20, [20, 90, 40], seg=500)
    vals = I.make_values(p, seed=5)
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=S.STILES_ORDER_ADAPTABLE_ND, nd_parts=3)
    tasks = S.stiles_symbolic_export(sym.handle, "mtask").reshape(-1, 8)
    fac = S.Factor(sym, nrhs_max=2)
    tr = torch.zeros(len(tasks) * 4, dtype=torch.int64, device="cuda")
    say("[gpu merged trace] %d tasks" % len(tasks))
    S.stiles_factor_set_merged_trace(fac.handle, tr)
    X = to_device_cols(I.rhs(p.N, 2, seed=6))
    fac.factorize_solve(torch.from_numpy(vals).cuda(), X)
    S.stiles_factor_set_merged_trace(fac.handle, None)
    a = tr.cpu().numpy().reshape(-1, 4).astype(np.uint64)
    assert (a[:, 0] > 0).all() and (a[:, 1] >= a[:, 0]).all() and (a[:, 2] >= a[:, 1]).all()
    assert np.array_equal((a[:, 3] >> np.uint64(24)) & np.uint64(0xff), (tasks[:, 0] & 0xff).astype(np.uint64))
