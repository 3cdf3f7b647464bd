"""Parity at the benchmarked sizes, in the launch configurations the bench
times: the variable-bandwidth matrix (n = 200,000, arrow 100, 8 right-hand
sides) under the natural ordering and under adaptable ND -- including the
merged factorization + solve launch exactly as the bench times it -- the
512-matrix batch and the n = 500,000 mixed-precision workload.  The oracle
runs on the full inputs on the host cores (a few seconds each).  Every
solution and log-determinant is compared in full; errors are normwise
relative (per right-hand side for X), and the natural-order factor is
checked both as a whole and per tile column (the largest
||dL(:,k)||_F / ||L_o(:,k)||_F over the tile columns k)."""
import os

import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import col_tile_err, oracle_solve_cols, rel, rel_cols, say, to_device_cols

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


@pytest.fixture(scope="module")
def varband():
    p = I.variable_band()
    vals = I.make_values(p, seed=2)
    B = I.rhs(p.N, 8, seed=102)
    say("[gpu fullsize] oracle on the variable-band matrix (N=%d)" % p.N)
    L, info = oracle.factor(p.f, vals, nthreads=_threads())
    assert info == 0
    return p, vals, B, L, oracle.logdet(p.f, L), oracle.solve(p.f, L, B)


@pytest.mark.parametrize("ordering,parts", [(S.STILES_ORDER_NONE, 0), (S.STILES_ORDER_ADAPTABLE_ND, 0)],
                         ids=["natural", "nd"])
def test_varband_full_size(varband, ordering, parts):
    import torch
    p, vals, B, Lref, ldref, Xref = varband
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=ordering, nd_parts=parts)
    say("[gpu fullsize] varband T=64 ordering=%d parts=%d" % (ordering, sym.info.nd_parts))
    fac = S.Factor(sym, nrhs_max=8)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    ld = fac.logdet().item()
    dB = to_device_cols(B)
    fac.solve(dB)
    eX = rel_cols(dB.cpu().numpy(), Xref)
    eld = abs(ld - ldref) / abs(ldref)
    say("   errors: X %.2e (worst right-hand side)  logdet %.2e" % (eX, eld))
    assert eX <= TOL and eld <= TOL
    if ordering == S.STILES_ORDER_NONE:
        Lg = fac.extract().cpu().numpy()
        eL = rel(Lg, Lref)
        eLc = col_tile_err(Lg, Lref, p.f, 64)
        say("   error L %.2e, worst tile column %.2e" % (eL, eLc))
        assert eL <= TOL and eLc <= TOL


def test_merged_launch_full_size(varband):
    """The bench's step exactly: automatic adaptable ND, T = 64, the merged
    factorization + solve launch with 8 right-hand sides.  X (every column)
    and logdet against the oracle within 1e-12, and X bitwise equal to
    separate factorize + solve launches on the same symbolic object."""
    import torch
    p, vals, B, Lref, ldref, Xref = varband
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=S.STILES_ORDER_ADAPTABLE_ND)
    say("[gpu fullsize] merged launch, varband T=64, %d partitions, 8 RHS" % sym.info.nd_parts)
    dv = torch.from_numpy(vals).cuda()
    fac = S.Factor(sym, nrhs_max=8)
    Xm = to_device_cols(B)
    fac.factorize_solve(dv, Xm)
    assert fac.info() == 0
    ld = fac.logdet().item()
    eX = rel_cols(Xm.cpu().numpy(), Xref)
    eld = abs(ld - ldref) / abs(ldref)
    say("   errors: X %.2e (worst right-hand side)  logdet %.2e" % (eX, eld))
    assert eX <= TOL and eld <= TOL
    sep = S.Factor(sym, nrhs_max=8)
    sep.factorize(dv)
    Xs = to_device_cols(B)
    sep.solve(Xs)
    assert sep.info() == 0
    assert torch.equal(Xm, Xs), "merged launch differs from separate launches"
    assert torch.equal(fac.logdet(), sep.logdet())


@pytest.fixture(scope="module")
def varband_selinv(varband):
    p, vals, B, L, ldref, Xref = varband
    say("[gpu fullsize] oracle selected inversion (N=%d)" % p.N)
    return oracle.selinv(p.f, L, nthreads=_threads())


@pytest.mark.parametrize("ordering", [S.STILES_ORDER_NONE, S.STILES_ORDER_ADAPTABLE_ND], ids=["natural", "nd"])
def test_varband_selinv_full_size(varband, varband_selinv, ordering):
    """Selected inversion at the benchmarked size: the diagonal of A^{-1}
    (original ordering) against the oracle's Takahashi recursion, entry by
    entry; under the natural ordering every envelope entry as well."""
    import torch
    p, vals = varband[0], varband[1]
    Sref = varband_selinv
    rp = p.row_ptr()
    dref = Sref[rp[1:] - 1]
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=ordering)
    say("[gpu fullsize] selinv ordering=%d parts=%d" % (ordering, sym.info.nd_parts))
    fac = S.Factor(sym)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    si = S.SelInv(fac).compute()
    d = si.diag().cpu().numpy()
    ed = float(np.max(np.abs(d - dref) / dref))
    say("   diagonal error %.2e" % ed)
    assert ed <= TOL
    if ordering == S.STILES_ORDER_NONE:
        e = rel(si.extract().cpu().numpy(), Sref)
        say("   entries error %.2e" % e)
        assert e <= TOL


def test_batch512_full_size():
    """All 512 matrices of the batched workload (device-generated values,
    read back for the oracle): every log-determinant within 1e-12."""
    import torch

    from paper_2501_02483_amd.devgen import DevicePattern
    pats = I.batch_patterns()
    dvals = [DevicePattern(q).values(q.meta["value_seed"]) for q in pats]
    syms = [S.Symbolic.from_pattern(q, tile=64) for q in pats]
    facs = [S.Factor(s) for s in syms]
    batch = S.Batch(facs)
    say("[gpu fullsize] batch of %d" % len(pats))
    batch.factorize(dvals)
    lds = batch.logdet().cpu().numpy()
    worst = 0.0
    for q, v, f, ld in zip(pats, dvals, facs, lds):
        assert f.info() == 0
        L, info = oracle.factor(q.f, v.cpu().numpy(), nthreads=_threads())
        assert info == 0
        ref = oracle.logdet(q.f, L)
        worst = max(worst, abs(ld - ref) / abs(ref))
    say("   worst logdet error %.2e" % worst)
    assert worst <= TOL


def test_small_bench_configuration():
    """The n = 2,000 / half-width 50 / arrow 10 workload as the bench runs it
    (T = 64, adaptable ND with the automatic partition count, 1 RHS)."""
    import torch
    p = I.single_small()
    vals = I.make_values(p, seed=1)
    B = I.rhs(p.N, 1, seed=101)
    L, info = oracle.factor(p.f, vals, nthreads=_threads())
    assert info == 0
    X_o = oracle.solve(p.f, L, B)
    ld_o = oracle.logdet(p.f, L)
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=S.STILES_ORDER_ADAPTABLE_ND)
    say("[gpu fullsize] small workload, %d partitions" % sym.info.nd_parts)
    fac = S.Factor(sym)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    dB = to_device_cols(B)
    fac.solve(dB)
    assert rel(dB.cpu().numpy(), X_o) <= TOL
    assert abs(fac.logdet().item() - ld_o) <= TOL * abs(ld_o)


def test_mixed_full_size():
    """The n = 500,000 / half-width 1,000 / arrow 200 Laplacian workload
    (κ ≈ 1e6) in mixed precision, as the bench runs it (adaptable ND, 16
    right-hand sides, FP64 refinement): all sixteen solutions (each column)
    and the log-determinant against the oracle on the device-drawn values."""
    import torch

    from paper_2501_02483_amd.devgen import DevicePattern
    p = I.mixed_large()
    dv = DevicePattern(p).values(4, law="laplacian", kappa=1e6)
    B = torch.randn(16, p.N, dtype=torch.float64, device="cuda",
                    generator=torch.Generator("cuda").manual_seed(104)).t()
    sym = S.Symbolic.from_pattern(p, tile=64, ordering=S.STILES_ORDER_ADAPTABLE_ND)
    say("[gpu fullsize] mixed n=500,000, %d partitions" % sym.info.nd_parts)
    fac = S.Factor(sym, S.STILES_MIXED32, nrhs_max=16)
    fac.factorize(dv)
    assert fac.info() == 0
    X = B.clone()
    rep = fac.solve(X)
    ld = fac.logdet().item()
    vals = dv.cpu().numpy()
    Bh = np.ascontiguousarray(B.cpu().numpy())
    Xh = np.ascontiguousarray(X.cpu().numpy())
    del fac, dv
    say("   oracle factorization (host)")
    L, info = oracle.factor(p.f, vals, nthreads=_threads())
    assert info == 0
    ld_o = oracle.logdet(p.f, L)
    X_o = oracle_solve_cols(p.f, L, Bh)
    eX = rel_cols(Xh, X_o)
    eld = abs(ld - ld_o) / abs(ld_o)
    say("   errors: X %.2e (worst of 16 right-hand sides)  logdet %.2e  refinement steps %d  "
        "backward error %.2e" % (eX, eld, rep.iterations, rep.backward_error))
    assert rep.converged == 1
    assert max(rep.per_rhs[0]) == rep.backward_error
    assert eX <= 1e-9 and eld <= 1e-6
