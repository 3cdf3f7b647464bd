"""Out-of-core (streamed) factorization: the band is factored segment by
segment, each segment in core with the next segment's coupling rows after
its own and the arrow as its arrow, its Schur complement seeding the next
one.  L (whole
factor, and per tile column) and the log-determinant match the FP64 oracle
within 1e-12 for several segment lengths and both tile sizes, one segment
reproduces the in-core factor, the device footprint of a segment stays
below that of the whole factorization, and a non-SPD row is reported at
its own index."""
import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import col_tile_err, rel, say

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _oracle(p, vals):
    L, info = oracle.factor(p.f, vals, nthreads=8)
    assert info == 0
    return L, oracle.logdet(p.f, L)


@pytest.mark.parametrize("seg,T", [(700, 64), (2500, 64), (1000, 32), (600, 64), (0, 64)],
                         ids=["seg700_T64", "seg2500_T64", "seg1000_T32", "seg600_T64", "one_segment_T64"])
def test_ooc_matches_oracle(seg, T):
    # the half-width grows at rows 700 (20 -> 200) and 2,100 (90 -> 130):
    # segments of 600 and 1,000 rows end 100 and 100 rows before such a
    # row, so the rows that couple back across the boundary are not
    # contiguous there (80 and 10 rows in between do not)
    p = I.make_pattern(20000, 40, [20, 200, 90, 130], seg=700)
    vals = I.make_values(p, seed=77)
    L_o, ld_o = _oracle(p, vals)
    seg_rows = seg or p.n
    L, ld, info, peak = S.stiles_factorize_ooc(p.n, p.a, p.f[:p.n], vals, seg_rows, tile=T)
    eL, eC = rel(L, L_o), col_tile_err(L, L_o, p.f, T)
    say("[gpu ooc] n=%d seg=%d T=%d: peak %.1f MB, L %.2e (per tile column %.2e), logdet %.2e" % (
        p.n, seg_rows, T, peak / 2 ** 20, eL, eC, abs(ld - ld_o) / abs(ld_o)))
    assert info == 0
    assert eL <= TOL and eC <= TOL
    assert abs(ld - ld_o) <= TOL * abs(ld_o)


def test_ooc_one_segment_is_the_in_core_factor_and_segments_save_memory():
    import torch
    p = I.make_pattern(30000, 60, 250)
    vals = I.make_values(p, seed=5)
    L1, ld1, _, peak1 = S.stiles_factorize_ooc(p.n, p.a, p.f[:p.n], vals, p.n, tile=64)
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=S.STILES_ORDER_NONE)
    fac = S.Factor(sym)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    assert np.array_equal(fac.extract().cpu().numpy(), L1)
    L4, ld4, _, peak4 = S.stiles_factorize_ooc(p.n, p.a, p.f[:p.n], vals, 3000, tile=64)
    say("[gpu ooc] one segment %.1f MB, segments of 3,000 rows %.1f MB; |dL| %.2e" % (
        peak1 / 2 ** 20, peak4 / 2 ** 20, rel(L4, L1)))
    assert peak4 < peak1 / 4
    assert rel(L4, L1) <= TOL and abs(ld4 - ld1) <= TOL * abs(ld1)


def test_ooc_writes_every_entry_of_a_reused_output_and_repeats_bitwise():
    """The factor goes into a caller's array (filled with NaN first): every
    entry is written, and a second call into the same array gives the same
    bits (the host assembly and scatter run on several threads, each on its
    own rows)."""
    p = I.make_pattern(12000, 30, [60, 220, 140], seg=3000)
    vals = I.make_values(p, seed=12)
    out = np.full(p.nnz, np.nan)
    L, ld, info, _ = S.stiles_factorize_ooc(p.n, p.a, p.f[:p.n], vals, 2500, tile=64, out=out)
    assert info == 0 and L is out
    assert not np.isnan(out).any()
    first = out.copy()
    out[:] = np.nan
    _, ld2, _, _ = S.stiles_factorize_ooc(p.n, p.a, p.f[:p.n], vals, 2500, tile=64, out=out)
    assert np.array_equal(out, first) and ld2 == ld
    Lo, info_o = oracle.factor(p.f, vals)
    assert info_o == 0 and rel(out, Lo) <= TOL
    with pytest.raises(ValueError):
        S.stiles_factorize_ooc(p.n, p.a, p.f[:p.n], vals, 2500, tile=64, out=np.empty(p.nnz - 1))


def test_ooc_reports_the_failing_row():
    p = I.make_pattern(8000, 20, 100)
    vals = I.make_values(p, seed=9)
    bad = 5321
    rp = p.row_ptr()
    vals[rp[bad + 1] - 1] = -1.0                 # a negative pivot in segment 3
    _, info_o = oracle.factor(p.f, vals)
    L, ld, info, _ = S.stiles_factorize_ooc(p.n, p.a, p.f[:p.n], vals, 2000, tile=64)
    say("[gpu ooc] planted non-SPD row %d: info %d (oracle %d)" % (bad, info, info_o))
    assert info == info_o == bad + 1
    assert np.isnan(ld)


def test_ooc_full_size_variable_band():
    """The default workload's matrix (n = 200,000, a = 100) in segments of
    20,000 rows, natural order."""
    p = I.variable_band()
    vals = I.make_values(p, seed=2)
    L_o, ld_o = _oracle(p, vals)
    L, ld, info, peak = S.stiles_factorize_ooc(p.n, p.a, p.f[:p.n], vals, 20000, tile=64)
    eC = col_tile_err(L, L_o, p.f, 64)
    say("[gpu ooc] full size n=%d, segments of 20,000 rows: peak %.1f MB, L per tile column %.2e, logdet %.2e" % (
        p.n, peak / 2 ** 20, eC, abs(ld - ld_o) / abs(ld_o)))
    assert info == 0 and eC <= TOL and abs(ld - ld_o) <= TOL * abs(ld_o)
