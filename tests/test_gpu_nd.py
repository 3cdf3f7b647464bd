"""Adaptable nested dissection on the GPU: the factor of P A P^T matches the
oracle's factor of the same permuted matrix (built by brute force from the
entries), and the solution and log-determinant, which do not depend on the
ordering, match the oracle on the original matrix.  Bar as for the natural
ordering: 1e-12 normwise relative, for the whole factor and for each of its
tile columns (||dL(:,k)||_F / ||L_o(:,k)||_F), and for each right-hand side."""
import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import col_tile_err, oracle_reference, rel, rel_cols, say, to_device_cols
from permute_util import permute_profile

pytestmark = pytest.mark.gpu

TOL = 1e-12
ND = S.STILES_ORDER_ADAPTABLE_ND

CASES = [
    # n, arrow, widths, segment, tile, parts, nrhs
    (3000, 20, [20, 90, 40], 500, 64, 2, 1),
    (3001, 33, [10, 120, 60], 400, 32, 3, 4),
    (4000, 0, 50, None, 64, 4, 2),
    (5000, 70, [30, 150, 80, 40], 600, 64, 0, 8),
    (2500, 100, [8, 60], 250, 32, 5, 3),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_a%d_T%d_P%d" % (c[0], c[1], c[4], c[5]))
def test_nd_factor_solve_logdet(case):
    import torch
    n, a, w, seg, T, parts, nrhs = case
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + T + parts)
    B = I.rhs(p.N, nrhs, seed=11)
    sym = S.Symbolic.from_pattern(p, tile=T, ordering=ND, nd_parts=parts)
    say("[gpu nd] case n=%d a=%d T=%d parts=%d -> P=%d band=%d arrow=%d" % (
        n, a, T, parts, sym.info.nd_parts, sym.info.n, sym.info.arrow))
    assert sym.info.ordering_used == ND
    ref = oracle_reference(p, vals, B)
    f2, v2 = permute_profile(p.f, vals, sym.perm())
    L2, info2 = oracle.factor(f2, v2, nthreads=8)
    assert info2 == 0
    fac = S.Factor(sym, S.STILES_FP64, nrhs_max=nrhs)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    L = fac.extract().cpu().numpy()
    eL = rel(L, L2)
    eLc = col_tile_err(L, L2, f2, T)
    ld = fac.logdet().item()
    dB = to_device_cols(B)
    fac.solve(dB)
    X = dB.cpu().numpy()
    eX = rel_cols(X, ref["X"])
    eld = abs(ld - ref["logdet"]) / abs(ref["logdet"])
    say("   errors: L %.2e (worst tile column %.2e)  X %.2e  logdet %.2e" % (eL, eLc, eX, eld))
    assert eL <= TOL and eLc <= TOL and eX <= TOL and eld <= TOL


def test_nd_non_spd_reports_permuted_column():
    """A non-positive pivot is reported as a 1-based column of P A P^T; the
    oracle factor of the permuted matrix fails at the same column."""
    import torch
    p = I.make_pattern(2000, 10, 40)
    vals = I.make_values(p, seed=9)
    rp = p.row_ptr()
    vals[rp[1500 + 1] - 1] = -2.0
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=ND, nd_parts=3)
    f2, v2 = permute_profile(p.f, vals, sym.perm())
    _, info2 = oracle.factor(f2, v2, nthreads=8)
    fac = S.Factor(sym)
    say("[gpu nd] non-SPD")
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == info2 > 0


def test_nd_mixed_precision_solve():
    """Mixed mode under the ND ordering: refined solution at FP64 accuracy."""
    import torch
    p = I.make_pattern(4000, 40, [30, 100], seg=800)
    vals = I.make_values(p, seed=21)
    B = I.rhs(p.N, 2, seed=5)
    ref = oracle_reference(p, vals, B)
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=ND, nd_parts=3)
    fac = S.Factor(sym, S.STILES_MIXED32, nrhs_max=2)
    say("[gpu nd] mixed")
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    dB = to_device_cols(B)
    fac.solve(dB)
    assert rel(dB.cpu().numpy(), ref["X"]) <= 1e-12
    assert abs(fac.logdet().item() - ref["logdet"]) <= 1e-6 * abs(ref["logdet"])


def test_nd_in_batch_equals_single():
    """An ND factor inside a batch (per-matrix scatter) equals its single run."""
    import torch
    pats = [I.make_pattern(2500, 16, 60), I.make_pattern(1800, 8, 30)]
    vals = [I.make_values(q, seed=70 + i) for i, q in enumerate(pats)]
    syms = [S.Symbolic.from_pattern(pats[0], tile=64, ordering=ND, nd_parts=2),
            S.Symbolic.from_pattern(pats[1], tile=64)]
    facs = [S.Factor(s) for s in syms]
    dv = [torch.from_numpy(v).cuda() for v in vals]
    say("[gpu nd] batch")
    b = S.Batch(facs)
    b.factorize(dv)
    lds = b.logdet()
    torch.cuda.synchronize()
    for i, (s, f) in enumerate(zip(syms, facs)):
        assert f.info() == 0
        one = S.Factor(s)
        one.factorize(dv[i])
        assert torch.equal(one.extract(), f.extract())
        assert torch.equal(one.logdet(), lds[i:i + 1])
