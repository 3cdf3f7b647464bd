"""Helpers shared by the GPU tests: run the HIP path through the C ABI binding
and compare with the FP64 oracle."""
import sys

import numpy as np

import oracle
from paper_2501_02483_amd import inputs as I


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_device_cols(B):
    """(N, nrhs) numpy -> column-major float64 CUDA tensor of shape (N, nrhs)."""
    import torch
    t = torch.empty((B.shape[1], B.shape[0]), dtype=torch.float64, device="cuda")
    t.copy_(torch.from_numpy(np.ascontiguousarray(B.T)))
    return t.t()


def rel(a, b):
    """Normwise relative error ||a - b||_F / ||b||_F (one number for the whole
    array, not an element-by-element bound)."""
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def rel_cols(a, b):
    """Largest normwise relative error over the columns (right-hand sides)."""
    a = np.asarray(a).reshape(a.shape[0], -1)
    b = np.asarray(b).reshape(b.shape[0], -1)
    return max(rel(a[:, c], b[:, c]) for c in range(b.shape[1]))


def col_tile_err(L, Lo, f, T):
    """Per-tile-column error of a factor in row-profile order (row i holds
    columns f[i]..i): max over tile columns k of ||dL(:, kT:(k+1)T)||_F /
    ||Lo(:, kT:(k+1)T)||_F, so that a wrong block column cannot hide in the
    norm of the whole factor."""
    f = np.asarray(f, dtype=np.int64)
    N = f.shape[0]
    lens = np.arange(N, dtype=np.int64) - f + 1
    rp = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(lens, out=rp[1:])
    num = np.zeros((N + T - 1) // T)
    den = np.zeros_like(num)
    # rows in blocks, to bound the temporary index arrays
    step = 1 << 14
    for r0 in range(0, N, step):
        r1 = min(N, r0 + step)
        e0, e1 = rp[r0], rp[r1]
        col = np.arange(e0, e1, dtype=np.int64) - np.repeat(rp[r0:r1] - f[r0:r1], lens[r0:r1])
        tc = col // T
        d = np.asarray(L[e0:e1], dtype=np.float64) - np.asarray(Lo[e0:e1], dtype=np.float64)
        num += np.bincount(tc, weights=d * d, minlength=num.shape[0])
        lo = np.asarray(Lo[e0:e1], dtype=np.float64)
        den += np.bincount(tc, weights=lo * lo, minlength=num.shape[0])
    ok = den > 0
    return float(np.max(np.sqrt(num[ok] / den[ok]))) if ok.any() else 0.0


def oracle_solve_cols(f, L, B, workers=16):
    """oracle.solve on each column of B in parallel host threads (the
    oracle's solve is sequential; ctypes releases the GIL during the call)."""
    from concurrent.futures import ThreadPoolExecutor
    B = np.asarray(B, dtype=np.float64).reshape(B.shape[0], -1)
    with ThreadPoolExecutor(max_workers=min(workers, B.shape[1])) as ex:
        cols = list(ex.map(lambda c: oracle.solve(f, L, np.ascontiguousarray(B[:, c])), range(B.shape[1])))
    return np.stack(cols, axis=1)


def oracle_reference(p, vals, B=None):
    L, info = oracle.factor(p.f, vals, nthreads=8)
    out = {"L": L, "info": info}
    if info == 0:
        out["logdet"] = oracle.logdet(p.f, L)
        if B is not None:
            out["X"] = oracle.solve(p.f, L, B)
    return out
