"""POTRF tasks that also form the panel tile below the diagonal
(option fuse_panel; off by default).  The panel's products run in the same
order as in a separate TRSM task, so the factor, the solution and the
log-determinant are bitwise those of the unfused plan, and match the FP64
oracle within 1e-12 (natural order: L as well; adaptable ND: X and logdet
against the unpermuted oracle); mixed precision keeps its refined accuracy."""
import numpy as np
import pytest

import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import oracle_reference, rel, rel_cols, say, to_device_cols

pytestmark = pytest.mark.gpu

CASES = [
    # n, arrow, widths, segment, tile, ordering, parts, nrhs
    (4000, 40, [20, 200, 90, 130], 700, 64, S.STILES_ORDER_NONE, 0, 4),
    (3001, 33, [10, 120, 60], 400, 32, S.STILES_ORDER_NONE, 0, 3),
    (6000, 70, [30, 250, 80, 160], 600, 64, S.STILES_ORDER_ADAPTABLE_ND, 4, 8),
]


def _run(sym, dv, B, precision=S.STILES_FP64):
    import torch
    fac = S.Factor(sym, precision, nrhs_max=B.shape[1])
    fac.factorize(dv)
    assert fac.info() == 0
    X = to_device_cols(B)
    fac.solve(X)
    both = S.Factor(sym, precision, nrhs_max=B.shape[1])
    X2 = to_device_cols(B)
    both.factorize_solve(dv, X2)
    assert both.info() == 0
    if precision == S.STILES_FP64:
        assert torch.equal(X, X2)
    return fac.extract(), X, fac.logdet()


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_T%d_o%d_P%d" % (c[0], c[4], c[5], c[6]))
def test_panel_fusion_bitwise_and_oracle(case):
    import torch
    n, a, w, seg, T, ordering, parts, nrhs = case
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + 7)
    B = I.rhs(p.N, nrhs, seed=23)
    ref = oracle_reference(p, vals, B)
    on = S.Symbolic.from_pattern(p, tile=T, ordering=ordering, nd_parts=parts, fuse_panel=1)
    off = S.Symbolic.from_pattern(p, tile=T, ordering=ordering, nd_parts=parts)
    say("[gpu panel] n=%d T=%d ordering %d P=%d: %d panels fused" % (n, T, ordering, on.info.nd_parts,
                                                                     on.info.panels_fused))
    assert on.info.panels_fused > 0 and off.info.panels_fused == 0
    dv = torch.from_numpy(vals).cuda()
    L1, X1, ld1 = _run(on, dv, B)
    L0, X0, ld0 = _run(off, dv, B)
    assert torch.equal(L1, L0) and torch.equal(X1, X0) and torch.equal(ld1, ld0)
    eX = rel_cols(X1.cpu().numpy(), ref["X"])
    eld = abs(ld1.item() - ref["logdet"]) / abs(ref["logdet"])
    say("   errors: X %.2e  logdet %.2e" % (eX, eld))
    assert eX <= 1e-12 and eld <= 1e-12
    if ordering == S.STILES_ORDER_NONE:
        assert rel(L1.cpu().numpy(), ref["L"]) <= 1e-12


def test_panel_fusion_mixed_precision():
    import torch
    p = I.make_pattern(20000, 60, 200)
    vals = I.make_values(p, seed=4)
    B = I.rhs(p.N, 4, seed=104)
    ref = oracle_reference(p, vals, B)
    sym = S.Symbolic.from_pattern(p, tile=64, fuse_panel=1)
    say("[gpu panel] mixed precision, %d panels fused" % sym.info.panels_fused)
    fac = S.Factor(sym, S.STILES_MIXED32, nrhs_max=4)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    eL = rel(fac.extract().cpu().numpy(), ref["L"])
    dB = to_device_cols(B)
    rep = fac.solve(dB)
    eX = rel(dB.cpu().numpy(), ref["X"])
    say("   factor %.2e x %.2e iters %d" % (eL, eX, rep.iterations))
    assert rep.converged == 1 and eL <= 1e-5 and eX <= 1e-12
