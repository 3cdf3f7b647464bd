"""Spatio-temporal (SPDE-shaped) CSC input on the GPU: entries sparse inside
the envelope, a 13-point spatial stencil coupled over adjacent time steps and
a dense arrow.  Solution, log-determinant and the diagonal of A^{-1} are
ordering-invariant, so they are compared with the oracle run on the natural
order's row profile (zeros stored where the envelope has no entry); bar
1e-12."""
import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

from gpu_util import rel, say, to_device_cols

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def spde_cases():
    out = {}
    for key, (nx, ny, nt, a) in {"small": (12, 12, 8, 5), "medium": (20, 20, 20, 20)}.items():
        g = I.spde_space_time(nx, ny, nt, a, seed=7)
        p = g["pattern"]
        L, info = oracle.factor(p.f, g["profile_values"], nthreads=8)
        assert info == 0
        B = I.rhs(g["N"], 3, seed=17)
        Sg = oracle.selinv(p.f, L, nthreads=8)
        rp = p.row_ptr()
        out[key] = (g, B, oracle.solve(p.f, L, B), oracle.logdet(p.f, L), Sg[rp[1:] - 1])
    return out


@pytest.mark.parametrize("key", ["small", "medium"])
@pytest.mark.parametrize("ordering", [S.STILES_ORDER_AUTO, S.STILES_ORDER_ADAPTABLE_ND], ids=["auto", "nd"])
@pytest.mark.parametrize("tile", [32, 64])
def test_spde_factor_solve_logdet_selinv(spde_cases, key, ordering, tile):
    import torch
    g, B, Xo, ldo, do = spde_cases[key]
    sym = S.Symbolic.from_csc(g["N"], g["a"], g["colptr"], g["rowind"], tile=tile, ordering=ordering)
    say("[gpu spde] %s ordering %d -> used %d, %d partitions, T=%d, %d tiles" % (
        key, ordering, sym.info.ordering_used, sym.info.nd_parts, tile, sym.info.tiles))
    fac = S.Factor(sym, nrhs_max=3)
    fac.factorize(torch.from_numpy(g["values"]).cuda())
    assert fac.info() == 0
    dB = to_device_cols(B)
    fac.solve(dB)
    ld = fac.logdet().item()
    d = S.SelInv(fac).compute().diag().cpu().numpy()
    eX, eld, ed = rel(dB.cpu().numpy(), Xo), abs(ld - ldo) / abs(ldo), float(np.max(np.abs(d - do) / do))
    say("   errors: X %.2e  logdet %.2e  diag(A^-1) %.2e" % (eX, eld, ed))
    assert eX <= TOL and eld <= TOL and ed <= TOL
