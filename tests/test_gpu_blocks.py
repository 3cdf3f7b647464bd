"""2 x 2 block update tasks (option ublock: two tile rows of two adjacent
band tile columns share their operand tiles).  With blocks on, the factor,
the solution and the log-determinant match the FP64 oracle within 1e-12
(natural order: L as well; adaptable ND: X and logdet against the
unpermuted oracle), the merged factorization + solve launch is bitwise the
separate launches, and the mixed-precision mode (FP32 block products on the
FP32 copies of the factor) keeps the accuracy of the plain mixed path."""
import numpy as np
import pytest

import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import oracle_reference, rel, rel_cols, say, to_device_cols

pytestmark = pytest.mark.gpu

TOL = 1e-12

CASES = [
    # n, arrow, widths, segment, tile, ordering, parts, ublock, nrhs
    (4000, 40, [20, 200, 90, 130], 700, 64, S.STILES_ORDER_NONE, 0, 6, 4),
    (4000, 40, [20, 200, 90, 130], 700, 64, S.STILES_ORDER_NONE, 0, 1, 2),
    (3001, 33, [10, 120, 60], 400, 32, S.STILES_ORDER_NONE, 0, 4, 3),
    (6000, 70, [30, 250, 80, 160], 600, 64, S.STILES_ORDER_ADAPTABLE_ND, 4, 6, 8),
    (6000, 70, [30, 250, 80, 160], 600, 64, S.STILES_ORDER_ADAPTABLE_ND, 2, 15, 8),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_T%d_o%d_P%d_ub%d" % (c[0], c[4], c[5], c[6], c[7]))
def test_block_updates_match_oracle(case):
    import torch
    n, a, w, seg, T, ordering, parts, ub, nrhs = case
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + ub)
    B = I.rhs(p.N, nrhs, seed=17)
    ref = oracle_reference(p, vals, B)
    sym = S.Symbolic.from_pattern(p, tile=T, ordering=ordering, nd_parts=parts, ublock=ub)
    say("[gpu blocks] n=%d T=%d ordering %d P=%d ublock %d: %d blocks" % (
        n, T, ordering, sym.info.nd_parts, ub, sym.info.update_blocks))
    assert sym.info.update_blocks > 0
    dv = torch.from_numpy(vals).cuda()
    fac = S.Factor(sym, nrhs_max=nrhs)
    fac.factorize(dv)
    assert fac.info() == 0
    X = to_device_cols(B)
    fac.solve(X)
    eX = rel_cols(X.cpu().numpy(), ref["X"])
    ld = fac.logdet().item()
    eld = abs(ld - ref["logdet"]) / abs(ref["logdet"])
    say("   errors: X %.2e  logdet %.2e" % (eX, eld))
    assert eX <= TOL and eld <= TOL
    if ordering == S.STILES_ORDER_NONE:
        eL = rel(fac.extract().cpu().numpy(), ref["L"])
        say("   error L %.2e" % eL)
        assert eL <= TOL
    both = S.Factor(sym, nrhs_max=nrhs)
    X2 = to_device_cols(B)
    both.factorize_solve(dv, X2)
    assert both.info() == 0
    assert torch.equal(X, X2)
    assert torch.equal(fac.logdet(), both.logdet())


def test_block_updates_mixed_precision():
    import torch
    p = I.make_pattern(20000, 60, 200)
    vals = I.make_values(p, seed=4)
    B = I.rhs(p.N, 4, seed=104)
    ref = oracle_reference(p, vals, B)
    sym = S.Symbolic.from_pattern(p, tile=64, ublock=6)
    say("[gpu blocks] mixed precision, %d blocks" % sym.info.update_blocks)
    assert sym.info.update_blocks > 0
    fac = S.Factor(sym, S.STILES_MIXED32, nrhs_max=4)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    eL = rel(fac.extract().cpu().numpy(), ref["L"])
    ld = fac.logdet().item()
    eld = abs(ld - ref["logdet"]) / abs(ref["logdet"])
    dB = to_device_cols(B)
    rep = fac.solve(dB)
    eX = rel(dB.cpu().numpy(), ref["X"])
    say("   factor %.2e logdet %.2e x %.2e iters %d" % (eL, eld, eX, rep.iterations))
    assert rep.converged == 1
    assert eL <= 1e-5 and eld <= 1e-6 and eX <= 1e-12
