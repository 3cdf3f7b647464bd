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


def test_corner_accumulation_placement_and_scaled_law():
    """The arrow-corner accumulation in FP64 (STILES_MIXED32) and in FP32
    (STILES_MIXED32_FULL): the errors of each against the FP64 oracle on the
    Laplacian law (kappa ~ 1e6, wide arrow, corner sums over every band
    column); and the literal "scaled diagonal" input S A0 S (host
    scale_values, s_i = 10^(-3 u_i)), benign for FP32 updates because the
    factorization's rounding follows the condition of the diagonally scaled
    matrix.  Every variant's refined solution is accurate; the errors of
    factor and logdet are stated."""
    import torch
    p = I.make_pattern(20000, 200, 150)
    B = I.rhs(p.N, 2, seed=106)
    lap = I.make_values(p, seed=6, law="laplacian", kappa=1e6)
    scaled = I.scale_values(p, I.make_values(p, seed=7), seed=8)
    for name, vals in (("laplacian", lap), ("scaled", scaled)):
        ref = oracle_reference(p, vals, B)
        sym = S.Symbolic.from_pattern(p, tile=64)
        assert sym.info.tree_used == 1
        errs = {}
        for prec, pname in ((S.STILES_MIXED32, "corner FP64"), (S.STILES_MIXED32_FULL, "corner FP32")):
            fac = S.Factor(sym, prec, nrhs_max=2)
            fac.factorize(torch.from_numpy(vals).cuda())
            assert fac.info() == 0
            eL = rel(fac.extract().cpu().numpy(), ref["L"])
            eld = abs(fac.logdet().item() - ref["logdet"]) / abs(ref["logdet"])
            dB = to_device_cols(B)
            rep = fac.solve(dB)
            eX = rel(dB.cpu().numpy(), ref["X"])
            errs[pname] = (eL, eld, eX)
            say("[gpu mixed] %s, %s: factor %.2e logdet %.2e x %.2e (refinement steps %d, backward error %.2e)"
                % (name, pname, eL, eld, eX, rep.iterations, rep.backward_error))
            assert rep.converged == 1
            assert eX <= 1e-9
            assert eL <= 1e-3 and eld <= 1e-4
        assert errs["corner FP64"][0] <= 1e-5
