"""Parity of the HIP path (through the C ABI) with the FP64 oracle on seeded
inputs that span several tiles and ragged edges.  Bar (normwise, relative):
factor L <= 1e-12, solution X <= 1e-12, logdet <= 1e-12."""
import numpy as np
import pytest

import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import oracle_reference, rel, say, to_device_cols

pytestmark = pytest.mark.gpu

TOL = 1e-12

CASES = [
    # n, arrow, half-width (or widths), segment, tile, nrhs, tree ratio
    (100, 5, 7, None, 32, 1, 2),
    (2000, 10, 50, None, 64, 1, 2),          # the n=2,000 / w=50 / a=10 workload
    (1000, 0, 30, None, 64, 2, 2),           # band only
    (500, 64, 40, None, 64, 3, 2),           # arrow exactly one tile
    (777, 33, 100, None, 32, 4, 2),          # ragged band and arrow
    (300, 3, 0, None, 64, 1, 2),             # pure arrowhead (diagonal band)
    (3001, 70, [10, 200, 60], 1000, 64, 8, 2),  # variable bandwidth
    (3001, 70, [10, 200, 60], 1000, 64, 8, 0),  # same, arrow corner without the tree
    (1500, 130, 129, None, 32, 16, 2),       # three arrow tile rows at T=32... and 5
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d_a%d_T%d_r%d" % (c[0], c[1], c[4], c[6]))
def test_factor_solve_logdet_match_oracle(case):
    import torch
    n, a, w, seg, T, nrhs, ratio = case
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + a + T)
    B = I.rhs(p.N, nrhs, seed=7)
    say("[gpu parity] case n=%d a=%d w=%s T=%d nrhs=%d tree_ratio=%d" % (n, a, w, T, nrhs, ratio))
    ref = oracle_reference(p, vals, B)
    sym = S.Symbolic.from_pattern(p, tile=T, tree_min_ratio=ratio)
    fac = S.Factor(sym, S.STILES_FP64, nrhs_max=nrhs)
    dv = torch.from_numpy(vals).cuda()
    fac.factorize(dv)
    assert fac.info() == 0
    L = fac.extract().cpu().numpy()
    eL = rel(L, ref["L"])
    ld = fac.logdet().item()
    dB = to_device_cols(B)
    fac.solve(dB)
    X = dB.cpu().numpy()
    eX = rel(X, ref["X"])
    eld = abs(ld - ref["logdet"]) / abs(ref["logdet"])
    say("   errors: L %.2e  X %.2e  logdet %.2e" % (eL, eX, eld))
    assert eL <= TOL
    assert eX <= TOL
    assert eld <= TOL


def test_refactorize_same_workspace_new_values():
    import torch
    p = I.make_pattern(1200, 20, 45)
    sym = S.Symbolic.from_pattern(p, tile=64)
    fac = S.Factor(sym)
    for seed in (1, 2, 3):
        say("[gpu parity] refactorize seed", seed)
        vals = I.make_values(p, seed=seed)
        ref = oracle_reference(p, vals)
        fac.factorize(torch.from_numpy(vals).cuda())
        assert fac.info() == 0
        assert rel(fac.extract().cpu().numpy(), ref["L"]) <= TOL
        assert abs(fac.logdet().item() - ref["logdet"]) <= TOL * abs(ref["logdet"])


@pytest.mark.parametrize("bad", [0, 70, 1023, 1210])
def test_non_spd_reports_first_failing_column(bad):
    import torch
    p = I.make_pattern(1200, 20, 45)
    vals = I.make_values(p, seed=5)
    rp = p.row_ptr()
    vals[rp[bad + 1] - 1] = -1.0
    say("[gpu parity] non-SPD pivot at", bad)
    ref = oracle_reference(p, vals)
    assert ref["info"] == bad + 1
    sym = S.Symbolic.from_pattern(p, tile=64)
    fac = S.Factor(sym)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == bad + 1
    with pytest.raises(S.StilesError):
        fac.logdet()
