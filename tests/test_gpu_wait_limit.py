"""Bounded executor waits (Algorithm 2's progress check with a deadline).

A host-set deadline far below any task's duration makes the waits give up:
the launch is abandoned, every workgroup skips its remaining tasks and exits
normally (the kernels return; nothing hangs), stiles_factor_info reports
STILES_ETIMEOUT, solve and logdet refuse the factor, and once the default
deadline is restored the same workspace factors correctly again (the
progress counters were re-armed by the abandoned launch).  Covered: the
factorization, the merged factorization + solve, a batch, the solve alone
and the selected inversion."""
import numpy as np
import pytest

import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import oracle_reference, rel, say, to_device_cols

pytestmark = pytest.mark.gpu

TINY = 1e-8   # one tick of the 100 MHz device clock


def _case():
    p = I.make_pattern(5000, 40, [30, 150, 80], seg=700)
    vals = I.make_values(p, seed=77)
    B = I.rhs(p.N, 4, seed=78)
    return p, vals, B, oracle_reference(p, vals, B)


def _expect_timeout(fac):
    import torch
    torch.cuda.synchronize()
    with pytest.raises(S.StilesError) as e:
        fac.info()
    assert e.value.status == S.STILES_ETIMEOUT


def test_factorize_timeout_then_recovers():
    import torch
    p, vals, B, ref = _case()
    dv = torch.from_numpy(vals).cuda()
    for ordering in (S.STILES_ORDER_NONE, S.STILES_ORDER_ADAPTABLE_ND):
        sym = S.Symbolic.from_pattern(p, tile=64, ordering=ordering, nd_parts=3)
        fac = S.Factor(sym, nrhs_max=4)
        say("[gpu wait limit] factorize, ordering %d, deadline one tick" % ordering)
        fac.set_wait_limit(TINY)
        fac.factorize(dv)
        _expect_timeout(fac)
        X = to_device_cols(B)
        with pytest.raises(S.StilesError) as e:
            fac.solve(X)
        assert e.value.status == S.STILES_ESTATE
        fac.set_wait_limit(0)
        for _ in range(2):
            fac.factorize(dv)
            assert fac.info() == 0
            X = to_device_cols(B)
            fac.solve(X)
            assert rel(X.cpu().numpy(), ref["X"]) <= 1e-12
            assert abs(fac.logdet().item() - ref["logdet"]) <= 1e-12 * abs(ref["logdet"])


def test_merged_and_solve_timeout_then_recover():
    import torch
    p, vals, B, ref = _case()
    dv = torch.from_numpy(vals).cuda()
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=S.STILES_ORDER_ADAPTABLE_ND, nd_parts=3)
    fac = S.Factor(sym, nrhs_max=4)
    say("[gpu wait limit] merged factorization + solve, deadline one tick")
    fac.set_wait_limit(TINY)
    X = to_device_cols(B)
    fac.factorize_solve(dv, X)
    _expect_timeout(fac)
    assert torch.isnan(X).all()
    fac.set_wait_limit(0)
    X = to_device_cols(B)
    fac.factorize_solve(dv, X)
    assert fac.info() == 0
    assert rel(X.cpu().numpy(), ref["X"]) <= 1e-12
    # the solve launch alone: a good factor, then a solve past its deadline
    say("[gpu wait limit] solve alone, deadline one tick")
    fac.set_wait_limit(TINY)
    X = to_device_cols(B)
    fac.solve(X)
    _expect_timeout(fac)
    fac.set_wait_limit(0)
    fac.factorize(dv)
    assert fac.info() == 0
    X = to_device_cols(B)
    fac.solve(X)
    assert rel(X.cpu().numpy(), ref["X"]) <= 1e-12


def test_batch_and_selinv_timeout_then_recover():
    import torch
    pats = [I.make_pattern(3000, 16, 60), I.make_pattern(2200, 8, 90), I.make_pattern(4000, 30, 40)]
    vals = [I.make_values(q, seed=90 + i) for i, q in enumerate(pats)]
    dv = [torch.from_numpy(v).cuda() for v in vals]
    facs = [S.Factor(S.Symbolic.from_pattern(q, tile=64)) for q in pats]
    batch = S.Batch(facs)
    say("[gpu wait limit] batch of 3, deadline one tick")
    facs[0].set_wait_limit(TINY)
    batch.factorize(dv)
    torch.cuda.synchronize()
    statuses = []
    for f in facs:
        try:
            statuses.append(f.info())
        except S.StilesError as e:
            statuses.append(e.status)
    assert S.STILES_ETIMEOUT in statuses
    facs[0].set_wait_limit(0)
    batch.factorize(dv)
    lds = batch.logdet().cpu().numpy()
    for q, v, f, ld in zip(pats, vals, facs, lds):
        assert f.info() == 0
        ref = oracle_reference(q, v)
        assert abs(ld - ref["logdet"]) <= 1e-12 * abs(ref["logdet"])
    # selected inversion of a good factor, past its deadline
    say("[gpu wait limit] selected inversion, deadline one tick")
    f0 = facs[2]
    f0.factorize(dv[2])
    assert f0.info() == 0
    si = S.SelInv(f0)
    f0.set_wait_limit(TINY)
    d = si.compute().diag()
    _expect_timeout(f0)
    assert torch.isnan(d).all()
    f0.set_wait_limit(0)
    f0.factorize(dv[2])
    assert f0.info() == 0
    d = si.compute().diag().cpu().numpy()
    assert np.isfinite(d).all() and (d > 0).all()
