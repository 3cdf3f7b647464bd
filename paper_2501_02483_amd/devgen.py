"""Device-side synthetic values for band-plus-arrow envelopes (libstiles_gen.so).

Input generation only (no factorization arithmetic): off-diagonals are
counter-based normals (Philox4x32-10 + Box-Muller) indexed by their position
in row-profile order, the diagonal is the absolute row sum plus one.  Used by
the serving workload to draw a fresh matrix per request on the GPU.
"""
import ctypes
import os

import numpy as np

_LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libstiles_gen.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError("libstiles_gen.so is not built")
        lib = ctypes.CDLL(_LIB)
        lib.stiles_gen_offdiag.restype = ctypes.c_int
        lib.stiles_gen_offdiag.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                           ctypes.c_int64, ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                                           ctypes.c_void_p, ctypes.c_void_p]
        lib.stiles_gen_diag.restype = ctypes.c_int
        lib.stiles_gen_diag.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_double,
                                        ctypes.c_void_p, ctypes.c_void_p]
        _lib = lib
    return _lib


class DevicePattern:
    """Row pointers and first columns of a pattern, resident on the device."""

    def __init__(self, pattern, device="cuda"):
        import torch
        self.pattern = pattern
        f = pattern.f
        N = pattern.N
        self.N = N
        self.nnz = pattern.nnz
        self.rp = torch.from_numpy(pattern.row_ptr()).to(device)
        self.f = torch.from_numpy(np.ascontiguousarray(f)).to(device)
        i = np.arange(N)
        band = f > 0
        self.wmax = int((i[band] - f[band]).max()) if band.any() else 0
        self.full0 = pattern.n if pattern.a > 0 else N
        # rows before full0 with f == 0 but beyond wmax would be missed: widen
        early = (f == 0) & (i < self.full0)
        if early.any():
            self.wmax = max(self.wmax, int(i[early].max()))
        self.tmp = torch.empty(2 * N, dtype=torch.float64, device=device)

    def values(self, seed, out=None, stream=None, law="dominant", kappa=1e6, tmp=None, decades=3.0):
        """Seeded values on the device; law "dominant" (diagonal = |row| + 1)
        or "laplacian" (-|z| off-diagonals, diagonal = |row| + eps with
        eps = 2 max|row| / kappa, so that the smallest eigenvalue is eps), or
        "scaled": the dominant matrix A0 scaled symmetrically, S A0 S with
        s_i = 10^(-decades u_i), u_i ~ U[0, 1) from torch's generator seeded
        with `seed` (condition number up to ~10^(2 decades) while the
        diagonally scaled matrix stays well conditioned).
        tmp: scratch of at least 2N doubles; calls that may overlap on
        different streams must each pass their own (the default is shared)."""
        import torch
        if law == "scaled":
            v = self.values(seed, out=out, stream=stream, law="dominant", tmp=tmp)
            st = stream if stream is not None else torch.cuda.current_stream()
            with torch.cuda.stream(st):
                g = torch.Generator(device=v.device).manual_seed(int(seed))
                s = torch.pow(10.0, -decades * torch.rand(self.N, dtype=torch.float64, device=v.device,
                                                          generator=g))
                # entry e of row i sits at column f_i + (e - rp_i); rows in blocks
                rp = self.rp
                step = 1 << 14
                for r0 in range(0, self.N, step):
                    r1 = min(self.N, r0 + step)
                    lens = rp[r0 + 1:r1 + 1] - rp[r0:r1]
                    rows = torch.repeat_interleave(torch.arange(r0, r1, device=v.device), lens)
                    lo, hi = int(rp[r0]), int(rp[r1])
                    cols = torch.arange(lo, hi, device=v.device) - rp[rows] + self.f[rows]
                    v[lo:hi] *= s[rows] * s[cols]
            return v
        if out is None:
            out = torch.empty(self.nnz, dtype=torch.float64, device=self.rp.device)
        if tmp is None:
            tmp = self.tmp
        elif tmp.numel() < 2 * self.N or tmp.dtype != torch.float64:
            raise ValueError("tmp needs 2N float64 entries")
        st = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p(st.cuda_stream)
        lib = _load()
        err = lib.stiles_gen_offdiag(self.rp.data_ptr(), self.f.data_ptr(), self.N, self.wmax, self.full0, int(seed),
                                     1 if law == "laplacian" else 0, out.data_ptr(), tmp.data_ptr(), h)
        if err == 0:
            if law == "laplacian":
                with torch.cuda.stream(st):
                    tot = tmp[:self.N] + tmp[self.N:2 * self.N]
                    shift = 2.0 * float(tot.max()) / kappa
            else:
                shift = 1.0
            err = lib.stiles_gen_diag(self.rp.data_ptr(), self.N, tmp.data_ptr(), shift, out.data_ptr(), h)
        if err != 0:
            raise RuntimeError("device value generation failed (%d)" % err)
        return out
