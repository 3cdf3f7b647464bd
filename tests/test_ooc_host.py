"""Argument checks of the out-of-core factorization (host only: every check
happens before the first device call)."""
import numpy as np
import pytest

import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I


def _call(n, a, f, vals, seg, tile=64):
    return S.stiles_factorize_ooc(n, a, f, vals, seg, tile=tile, stream=0)


@pytest.fixture(autouse=True)
def _no_torch_stream(monkeypatch):
    # the calls below fail before any stream is used
    monkeypatch.setattr(S, "_stream", lambda stream=None: None)


def test_segments_narrower_than_the_band_are_rejected():
    p = I.make_pattern(3000, 10, 200)
    vals = np.zeros(p.nnz)
    with pytest.raises(S.StilesError) as e:
        _call(p.n, p.a, p.f[:p.n], vals, 150)
    assert e.value.status == S.STILES_EINVAL and "argument 5" in str(e.value)


@pytest.mark.parametrize("bad", ["n", "first_col", "seg", "tile"])
def test_invalid_arguments(bad):
    p = I.make_pattern(500, 4, 20)
    f = p.f[:p.n].copy()
    vals = np.zeros(p.nnz)
    n, seg, tile = p.n, 200, 64
    if bad == "n":
        n = 0
    elif bad == "first_col":
        f[10] = 11
    elif bad == "seg":
        seg = 0
    else:
        tile = 48
    with pytest.raises(S.StilesError) as e:
        _call(n, p.a, f, vals, seg, tile)
    assert e.value.status == (S.STILES_ENOTSUP if bad == "tile" else S.STILES_EINVAL)
