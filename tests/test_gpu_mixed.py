"""Mixed precision: FP32 MFMA tile updates, FP64 POTRF/TRSM/corner/logdet, and
FP64 iterative refinement of solves against the resident original matrix.
Accuracy is stated against the FP64 oracle (forward error of x; factor and
logdet errors are those of the FP32 updates and are not refined)."""
import numpy as np
import pytest

import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import oracle_reference, rel, say, to_device_cols

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("law,kappa", [("dominant", None), ("laplacian", 1e6)])
def test_mixed_refinement_reaches_fp64_accuracy(law, kappa):
    import torch
    p = I.make_pattern(20000, 60, 200)
    vals = I.make_values(p, seed=4, law=law, kappa=kappa or 1e6)
    B = I.rhs(p.N, 4, seed=104)
    say("[gpu mixed] law=%s n=%d" % (law, p.n))
    ref = oracle_reference(p, vals, B)
    sym = S.Symbolic.from_pattern(p, tile=64)
    fac = S.Factor(sym, S.STILES_MIXED32, nrhs_max=4)
    fac.factorize(torch.from_numpy(vals).cuda())
    assert fac.info() == 0
    L = fac.extract().cpu().numpy()
    eL = rel(L, ref["L"])
    ld = fac.logdet().item()
    eld = abs(ld - ref["logdet"]) / abs(ref["logdet"])
    dB = to_device_cols(B)
    rep = fac.solve(dB)
    X = dB.cpu().numpy()
    eX = rel(X, ref["X"])
    say("   factor %.2e logdet %.2e x %.2e iters %d converged %d berr %.2e" % (
        eL, eld, eX, rep.iterations, rep.converged, rep.backward_error))
    assert rep.converged == 1
    assert eL <= 1e-5
    assert eld <= 1e-6
    if law == "dominant":
        assert eX <= 1e-12
    else:
        # kappa ~ 1e6: both solutions are accurate to about kappa * u
        assert eX <= 1e-9
