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
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def oracle_reference(p, vals, B=None):
    L, info = oracle.factor(p.f, vals, nthreads=8)
    out = {"L": L, "info": info}
    if info == 0:
        out["logdet"] = oracle.logdet(p.f, L)
        if B is not None:
            out["X"] = oracle.solve(p.f, L, B)
    return out
