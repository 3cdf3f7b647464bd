"""Batched persistent launch (many independent factorizations in one kernel):
each matrix matches the oracle, and equals its single-launch factorization
bit for bit (same symbolic object, fixed per-tile accumulation order)."""
import numpy as np
import pytest

import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import oracle_reference, rel, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("T", [32, 64])
def test_batch_matches_oracle_and_single(T):
    import torch
    rng = np.random.default_rng(17)
    pats, vals = [], []
    for b in range(10):
        n = int(rng.integers(200, 3000))
        w = int(rng.integers(8, 200))
        a = int(rng.integers(0, 70))
        pats.append(I.make_pattern(n, a, w, name="b%d" % b))
        vals.append(I.make_values(pats[-1], seed=3000 + b))
    say("[gpu batch] T=%d sizes %s" % (T, [(p.n, p.a) for p in pats]))
    syms = [S.Symbolic.from_pattern(p, tile=T) for p in pats]
    facs = [S.Factor(s) for s in syms]
    dvals = [torch.from_numpy(v).cuda() for v in vals]
    S.factorize_batch(facs, dvals)
    torch.cuda.synchronize()
    Lb = []
    for p, v, f in zip(pats, vals, facs):
        assert f.info() == 0
        L = f.extract().cpu().numpy()
        Lb.append(L)
        ref = oracle_reference(p, v)
        assert rel(L, ref["L"]) <= 1e-12
        assert abs(f.logdet().item() - ref["logdet"]) <= 1e-12 * abs(ref["logdet"])
    # the same matrices factored one at a time: bitwise identical
    for p, v, s, L in zip(pats, dvals, syms, Lb):
        f1 = S.Factor(s)
        f1.factorize(v)
        assert np.array_equal(f1.extract().cpu().numpy(), L)


def test_batch_reuse_and_failure_isolated():
    """A non-SPD matrix in the batch reports its own failure; the others are unaffected."""
    import torch
    pats = [I.make_pattern(900, 12, 40), I.make_pattern(1500, 5, 70), I.make_pattern(600, 0, 20)]
    vals = [I.make_values(p, seed=40 + i) for i, p in enumerate(pats)]
    bad = vals[1].copy()
    rp = pats[1].row_ptr()
    bad[rp[777 + 1] - 1] = -5.0
    syms = [S.Symbolic.from_pattern(p, tile=64) for p in pats]
    facs = [S.Factor(s) for s in syms]
    say("[gpu batch] failure isolation")
    S.factorize_batch(facs, [torch.from_numpy(v).cuda() for v in (vals[0], bad, vals[2])])
    assert facs[0].info() == 0 and facs[2].info() == 0
    assert facs[1].info() == 778
    for i in (0, 2):
        ref = oracle_reference(pats[i], vals[i])
        assert rel(facs[i].extract().cpu().numpy(), ref["L"]) <= 1e-12
    # the workspaces are reusable after the batch (counters re-armed)
    S.factorize_batch(facs, [torch.from_numpy(v).cuda() for v in vals])
    assert [f.info() for f in facs] == [0, 0, 0]


def test_batch_logdet_and_refactorize():
    """Batched scatter + batched log-determinant: every value equals the
    single-factor stiles_logdet bit for bit, a failed matrix gives NaN, and a
    second factorize with new value arrays (new pointers) is picked up."""
    import torch
    rng = np.random.default_rng(23)
    pats = [I.make_pattern(int(rng.integers(100, 2500)), int(rng.integers(0, 40)), int(rng.integers(5, 120)))
            for _ in range(7)]
    vals = [I.make_values(p, seed=500 + i) for i, p in enumerate(pats)]
    syms = [S.Symbolic.from_pattern(p, tile=64) for p in pats]
    facs = [S.Factor(s) for s in syms]
    batch = S.Batch(facs)
    dvals = [torch.from_numpy(v).cuda() for v in vals]
    say("[gpu batch] batched logdet, %d matrices" % len(pats))
    batch.factorize(dvals)
    lds = batch.logdet()
    torch.cuda.synchronize()
    for i, f in enumerate(facs):
        assert f.info() == 0
        one = f.logdet()
        assert torch.equal(one, lds[i:i + 1])
        ref = oracle_reference(pats[i], vals[i])
        assert abs(lds[i].item() - ref["logdet"]) <= 1e-12 * abs(ref["logdet"])
    # new arrays (other pointers): one matrix made indefinite
    vals2 = [I.make_values(p, seed=900 + i) for i, p in enumerate(pats)]
    rp = pats[3].row_ptr()
    vals2[3][rp[pats[3].N // 2 + 1] - 1] = -1.0
    dvals2 = [torch.from_numpy(v).cuda() for v in vals2]
    batch.factorize(dvals2)
    lds2 = batch.logdet()
    torch.cuda.synchronize()
    for i, f in enumerate(facs):
        if i == 3:
            assert f.info() > 0
            assert torch.isnan(lds2[i]).item()
            continue
        assert f.info() == 0
        ref = oracle_reference(pats[i], vals2[i])
        assert abs(lds2[i].item() - ref["logdet"]) <= 1e-12 * abs(ref["logdet"])


def test_batch_workgroup_cap_keeps_results_bitwise():
    """A batch launch takes its first factor's workgroup cap (so batches on
    different streams can share the GPU); fewer workgroups claim the same
    tickets, so every factor is bitwise the uncapped one."""
    import torch
    from paper_2501_02483_amd import autotune
    pats = [I.make_pattern(n, a, w, name="c%d" % i)
            for i, (n, a, w) in enumerate([(4000, 20, 90), (2500, 8, 40), (6000, 30, 150), (1200, 5, 16)])]
    vals = [torch.from_numpy(I.make_values(p, seed=40 + i)).cuda() for i, p in enumerate(pats)]
    out = []
    for cap in (0, 24):
        syms = autotune.batch_symbolics(pats, 64, 40)
        facs = [S.Factor(s) for s in syms]
        facs[0].set_max_workgroups(cap)
        batch = S.Batch(facs)
        batch.factorize(vals)
        lds = batch.logdet()
        torch.cuda.synchronize()
        assert all(f.info() == 0 for f in facs)
        out.append(([f.extract().cpu() for f in facs], lds.cpu()))
    say("[gpu batch] cap 24 workgroups vs the full GPU")
    for a, b in zip(out[0][0], out[1][0]):
        assert torch.equal(a, b)
    assert torch.equal(out[0][1], out[1][1])
