"""Parity at the benchmarked sizes, in the launch configurations the bench
times: the variable-bandwidth matrix (n = 200,000, arrow 100, 8 right-hand
sides) under the natural ordering and under adaptable ND, and the 512-matrix
batch.  The oracle runs on the full inputs on the host cores (a few seconds
each); solutions and log-determinants are compared in full, the natural-order
factor element by element."""
import os

import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import rel, say, to_device_cols

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
    eX = rel(dB.cpu().numpy(), Xref)
    eld = abs(ld - ldref) / abs(ldref)
    say("   errors: X %.2e  logdet %.2e" % (eX, eld))
    assert eX <= TOL and eld <= TOL
    if ordering == S.STILES_ORDER_NONE:
        eL = rel(fac.extract().cpu().numpy(), Lref)
        say("   error L %.2e" % eL)
        assert eL <= TOL


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
