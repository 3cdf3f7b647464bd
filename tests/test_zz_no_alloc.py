"""stiles_logdet_static: the log-determinant for callers that cannot allocate
device memory, with its per-tile-row partials in the library's fixed device
array.  Checked through the C ABI against stiles_logdet on the same factor
(bitwise: the same kernels sum in the same order) and against the oracle, on
two calls in a row, the second with a smaller matrix (fewer tile rows, so
stale partials of the first call must not leak into the second); a failed
factor gives NaN from both; a factor with more tile rows than the array
holds is rejected before anything runs."""
import numpy as np
import pytest

import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import oracle_reference, say

pytestmark = pytest.mark.gpu


def _factor(p, vals, tile, ordering):
    import torch
    sym = S.Symbolic.from_pattern(p, tile=tile, ordering=ordering)
    fac = S.Factor(sym)
    fac.factorize(torch.from_numpy(vals).cuda())
    return sym, fac


def _both(fac):
    import torch
    ref = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    out = torch.full((1,), -2.0, dtype=torch.float64, device="cuda")
    S.stiles_logdet(fac.handle, ref)
    S.stiles_logdet_static(fac.handle, out)
    torch.cuda.synchronize()
    return out.item(), ref.item()


def test_logdet_static_two_calls_second_smaller():
    cases = [
        # (pattern, value seed, tile, ordering): the second has fewer tile rows
        (I.make_pattern(60000, 40, [60, 300, 120], seg=4000), 11, 32, S.STILES_ORDER_ADAPTABLE_ND),
        (I.make_pattern(3000, 10, 50), 12, 64, S.STILES_ORDER_NONE),
    ]
    rows = []
    for p, seed, tile, ordering in cases:
        vals = I.make_values(p, seed=seed)
        sym, fac = _factor(p, vals, tile, ordering)
        rows.append(sym.info.tile_rows)
        say("[gpu no-alloc] logdet_static n=%d tile=%d tile rows=%d" % (p.n, tile, sym.info.tile_rows))
        assert fac.info() == 0
        got, ref = _both(fac)
        ld_o = oracle_reference(p, vals)["logdet"]
        say("   static %.17g  workspace %.17g  oracle %.17g" % (got, ref, ld_o))
        assert got == ref
        assert abs(got - ld_o) <= 1e-12 * abs(ld_o)
    assert rows[1] < rows[0]


def test_logdet_static_failed_factor_and_size_limit():
    import torch
    p = I.make_pattern(2000, 8, 30)
    vals = I.make_values(p, seed=13)
    vals[p.row_ptr()[700 + 1] - 1] = -5.0          # a negative pivot in row 700
    sym, fac = _factor(p, vals, 64, S.STILES_ORDER_NONE)
    say("[gpu no-alloc] logdet_static on a failed factorization")
    got, ref = _both(fac)          # launched before the failure is known: NaN
    assert np.isnan(got) and np.isnan(ref)
    assert fac.info() == 701
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(S.StilesError) as e:   # known failed: refused
        S.stiles_logdet_static(fac.handle, out)
    assert e.value.status == S.STILES_ESTATE
    # more tile rows than the fixed array holds: rejected, nothing written
    n = S.STILES_STATIC_LOGDET_MAX_ROWS * 32 + 1
    big = I.make_pattern(n, 1, 1)
    sym = S.Symbolic.from_pattern(big, tile=32)
    assert sym.info.tile_rows > S.STILES_STATIC_LOGDET_MAX_ROWS
    fac = S.Factor(sym)
    say("[gpu no-alloc] logdet_static size limit (%d tile rows)" % sym.info.tile_rows)
    out = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(S.StilesError) as e:
        S.stiles_logdet_static(fac.handle, out)
    assert e.value.status == S.STILES_ENOTSUP
    torch.cuda.synchronize()
    assert out.item() == 7.0
