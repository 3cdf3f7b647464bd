"""MI355X (gfx950) sparse tile Cholesky for SPD block-arrowhead matrices with
variable bandwidth (the sTiles method, arXiv 2501.02483).

This module is a thin ctypes binding of libstiles.so: the functions named
stiles_* marshal arguments to the C ABI of include/stiles.h and nothing else;
every step of the factorization, solve and log-determinant runs in the
library's HIP kernels.  PyTorch provides device memory and streams only.
The convenience classes Symbolic and Factor wrap the same calls.
"""
import ctypes
import os

import numpy as np

__all__ = [
    "STILES_FP64", "STILES_MIXED32", "StilesError", "Symbolic", "Factor", "load_library",
    "stiles_default_opts", "stiles_analyze", "stiles_analyze_profile", "stiles_symbolic_query",
    "stiles_symbolic_perm", "stiles_symbolic_destroy", "stiles_workspace_size", "stiles_workspace_init",
    "stiles_factorize", "stiles_factorize_batch", "stiles_batch_workspace_size", "stiles_factor_info",
    "stiles_solve", "stiles_logdet", "stiles_factor_set_max_workgroups", "stiles_factor_release",
    "stiles_status_string", "stiles_last_error_arg", "factorize_batch", "stiles_factor_extract",
    "stiles_factor_set_timing", "stiles_factor_kernel_ms", "stiles_factor_set_trace",
    "stiles_symbolic_export", "stiles_batch_create", "stiles_batch_factorize", "stiles_batch_logdet",
    "stiles_batch_destroy", "Batch", "SelInv", "stiles_selinv_query", "stiles_selinv_workspace_size",
    "stiles_selinv_create", "stiles_selinv_compute", "stiles_selinv_diag", "stiles_selinv_extract",
    "stiles_selinv_set_timing", "stiles_selinv_kernel_ms", "stiles_selinv_set_trace", "stiles_selinv_destroy",
    "stiles_factorize_solve", "stiles_factor_set_merged_trace", "stiles_factor_set_wait_limit",
    "stiles_logdet_static", "STILES_STATIC_LOGDET_MAX_ROWS", "stiles_factorize_ooc",
]

# STILES_LIBRARY names another build of the same library (the host-sanitized
# one, see sanitize.py); the default is the in-tree libstiles.so
LIB_PATH = os.environ.get("STILES_LIBRARY") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libstiles.so")

STILES_OK = 0
STILES_EINVAL = -1
STILES_ENOTSUP = -2
STILES_ENOMEM = -3
STILES_EDEVICE = -4
STILES_ESTATE = -5
STILES_ETIMEOUT = -6
STILES_ORDER_AUTO = 0
STILES_ORDER_NONE = 1
STILES_ORDER_PARTIAL_RCM = 2
STILES_ORDER_ADAPTABLE_ND = 3
STILES_ORDER_AMD = 4
STILES_FP64 = 0
STILES_MIXED32 = 1
STILES_MIXED32_FULL = 2
STILES_STATIC_LOGDET_MAX_ROWS = 65536

# every symbol include/stiles.h declares
EXPORTED = [
    "stiles_default_opts", "stiles_status_string", "stiles_last_error_arg", "stiles_analyze",
    "stiles_analyze_profile", "stiles_symbolic_query", "stiles_symbolic_perm", "stiles_symbolic_destroy",
    "stiles_workspace_size", "stiles_workspace_init", "stiles_factorize", "stiles_batch_workspace_size",
    "stiles_factorize_batch", "stiles_factor_info", "stiles_solve", "stiles_logdet",
    "stiles_factor_set_max_workgroups", "stiles_factor_release", "stiles_factor_extract",
    "stiles_factor_set_timing", "stiles_factor_kernel_ms", "stiles_factor_set_trace",
    "stiles_symbolic_export", "stiles_batch_create", "stiles_batch_factorize", "stiles_batch_logdet",
    "stiles_batch_destroy", "stiles_selinv_query", "stiles_selinv_workspace_size", "stiles_selinv_create",
    "stiles_selinv_compute", "stiles_selinv_diag", "stiles_selinv_extract", "stiles_selinv_set_timing",
    "stiles_selinv_kernel_ms", "stiles_selinv_set_trace", "stiles_selinv_destroy", "stiles_factorize_solve",
    "stiles_factor_set_merged_trace", "stiles_factor_set_wait_limit", "stiles_logdet_static",
    "stiles_factorize_ooc",
]


class stiles_opts(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("ordering", ctypes.c_int32), ("tree_min_ratio", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("refine_tol", ctypes.c_double), ("refine_max_iter", ctypes.c_int32),
                ("nd_parts", ctypes.c_int32), ("sched_workers", ctypes.c_int32), ("ublock", ctypes.c_int32)]


class stiles_symbolic_info(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("n", ctypes.c_int64), ("arrow", ctypes.c_int64),
                ("tile", ctypes.c_int32), ("ordering_used", ctypes.c_int32),
                ("tile_rows", ctypes.c_int64), ("band_tile_rows", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("nnz_L", ctypes.c_int64), ("flops_alg", ctypes.c_double), ("flops_exec", ctypes.c_double),
                ("factor_tasks", ctypes.c_int64), ("solve_tasks", ctypes.c_int64),
                ("corner_accumulations", ctypes.c_int64), ("tree_used", ctypes.c_int32),
                ("nd_parts", ctypes.c_int32), ("nnz_L_alg", ctypes.c_int64), ("update_blocks", ctypes.c_int64),
                ("nd_chain", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class stiles_solve_report(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32), ("backward_error", ctypes.c_double),
                ("backward_errors", ctypes.POINTER(ctypes.c_double)),
                ("rhs_iterations", ctypes.POINTER(ctypes.c_int32))]


_lib = None
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def load_library(path=LIB_PATH):
    """Load libstiles.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libstiles.so is not built (%s): run __graft_entry__.build() or "
                           "python paper_2501_02483_amd/build.py" % path)
    # torch first: its HIP runtime is then the one the library's HIP calls
    # bind to (the library loaded first would bring a second runtime into
    # the process, which does not see the device torch has opened)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    sig = {
        "stiles_default_opts": (None, [ctypes.POINTER(stiles_opts)]),
        "stiles_status_string": (ctypes.c_char_p, [_i32]),
        "stiles_last_error_arg": (_i32, []),
        "stiles_analyze": (_i32, [_i64, _i64, _vp, _vp, ctypes.POINTER(stiles_opts), ctypes.POINTER(_vp)]),
        "stiles_analyze_profile": (_i32, [_i64, _i64, _vp, ctypes.POINTER(stiles_opts), ctypes.POINTER(_vp)]),
        "stiles_symbolic_query": (_i32, [_vp, ctypes.POINTER(stiles_symbolic_info)]),
        "stiles_symbolic_perm": (_i32, [_vp, _vp]),
        "stiles_symbolic_destroy": (None, [_vp]),
        "stiles_workspace_size": (_i32, [_vp, _i32, _i64, ctypes.POINTER(ctypes.c_size_t)]),
        "stiles_workspace_init": (_i32, [_vp, _i32, _i64, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
        "stiles_factorize": (_i32, [_vp, _vp, _vp]),
        "stiles_batch_workspace_size": (_i32, [_i32, _vp, ctypes.POINTER(ctypes.c_size_t)]),
        "stiles_factorize_batch": (_i32, [_i32, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
        "stiles_factor_info": (_i32, [_vp, _vp, ctypes.POINTER(_i64)]),
        "stiles_solve": (_i32, [_vp, _i64, _vp, _i64, _vp, ctypes.POINTER(stiles_solve_report)]),
        "stiles_logdet": (_i32, [_vp, _vp, _vp]),
        "stiles_logdet_static": (_i32, [_vp, _vp, _vp]),
        "stiles_factorize_ooc": (_i32, [_i64, _i64, _vp, _vp, _i64, _i32, _vp, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_size_t), _vp]),
        "stiles_factor_set_max_workgroups": (_i32, [_vp, _i32]),
        "stiles_factor_set_wait_limit": (_i32, [_vp, ctypes.c_double]),
        "stiles_factor_release": (None, [_vp]),
        "stiles_factor_extract": (_i32, [_vp, _vp, _vp]),
        "stiles_factor_set_timing": (_i32, [_vp, _i32]),
        "stiles_factor_kernel_ms": (_i32, [_vp, _i32, ctypes.POINTER(ctypes.c_float)]),
        "stiles_factor_set_trace": (_i32, [_vp, _vp, _vp, _vp]),
        "stiles_factor_set_merged_trace": (_i32, [_vp, _vp, _vp]),
        "stiles_symbolic_export": (_i32, [_vp, _i32, _vp, ctypes.POINTER(_i64)]),
        "stiles_batch_create": (_i32, [_i32, _vp, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
        "stiles_batch_factorize": (_i32, [_vp, _vp, _vp]),
        "stiles_batch_logdet": (_i32, [_vp, _vp, _vp]),
        "stiles_batch_destroy": (None, [_vp]),
        "stiles_selinv_query": (_i32, [_vp, ctypes.POINTER(_i64), ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]),
        "stiles_selinv_workspace_size": (_i32, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
        "stiles_selinv_create": (_i32, [_vp, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]),
        "stiles_selinv_compute": (_i32, [_vp, _vp]),
        "stiles_selinv_diag": (_i32, [_vp, _vp, _vp]),
        "stiles_selinv_extract": (_i32, [_vp, _vp, _vp]),
        "stiles_selinv_set_timing": (_i32, [_vp, _i32]),
        "stiles_selinv_kernel_ms": (_i32, [_vp, ctypes.POINTER(ctypes.c_float)]),
        "stiles_selinv_set_trace": (_i32, [_vp, _vp, _vp]),
        "stiles_factorize_solve": (_i32, [_vp, _vp, _i64, _vp, _i64, _vp]),
        "stiles_selinv_destroy": (None, [_vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class StilesError(RuntimeError):
    def __init__(self, status, where):
        lib = load_library()
        arg = lib.stiles_last_error_arg()
        msg = "%s: %s" % (where, lib.stiles_status_string(status).decode())
        if status == STILES_EINVAL and arg:
            msg += " (argument %d)" % arg
        super().__init__(msg)
        self.status = status
        self.arg = arg


def _check(st, where):
    if st != STILES_OK:
        raise StilesError(st, where)


def _ptr(a):
    """Address of a numpy array or torch tensor (contiguous)."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------- raw C-ABI wrappers

def stiles_default_opts(tile=64, ordering=STILES_ORDER_AUTO, tree_min_ratio=2, chunk=0, refine_tol=0.0,
                        refine_max_iter=0, nd_parts=0, sched_workers=0, ublock=0):
    o = stiles_opts()
    load_library().stiles_default_opts(ctypes.byref(o))
    o.tile, o.ordering, o.tree_min_ratio, o.chunk = tile, ordering, tree_min_ratio, chunk
    o.refine_tol, o.refine_max_iter, o.nd_parts = refine_tol, refine_max_iter, nd_parts
    o.sched_workers = sched_workers
    o.ublock = ublock
    return o


def stiles_analyze(N, arrow, colptr, rowind, opts=None):
    colptr = np.ascontiguousarray(colptr, dtype=np.int64)
    rowind = np.ascontiguousarray(rowind, dtype=np.int64)
    h = _vp()
    _check(load_library().stiles_analyze(N, arrow, _ptr(colptr), _ptr(rowind),
                                         ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)),
           "stiles_analyze")
    return h


def stiles_analyze_profile(n_band, arrow, first_col, opts=None):
    first_col = np.ascontiguousarray(first_col, dtype=np.int64)
    h = _vp()
    _check(load_library().stiles_analyze_profile(n_band, arrow, _ptr(first_col) if n_band > 0 else None,
                                                 ctypes.byref(opts) if opts is not None else None, ctypes.byref(h)),
           "stiles_analyze_profile")
    return h


def stiles_symbolic_query(sym):
    info = stiles_symbolic_info()
    _check(load_library().stiles_symbolic_query(sym, ctypes.byref(info)), "stiles_symbolic_query")
    return info


def stiles_symbolic_perm(sym, N):
    p = np.empty(N, dtype=np.int64)
    _check(load_library().stiles_symbolic_perm(sym, _ptr(p)), "stiles_symbolic_perm")
    return p


EXPORT_KINDS = {"ftask": (0, np.int32), "fsucc": (1, np.int32), "fpairs": (2, np.int32), "stask": (3, np.int32),
                "ssucc": (4, np.int32), "spairs": (5, np.int32), "trow_ptr": (6, np.int32), "tcol": (7, np.int32),
                "row_base": (8, np.int64), "row_cnt": (9, np.int32), "npart": (10, np.int32),
                "itask": (11, np.int32), "isucc": (12, np.int32), "ilist": (13, np.int32),
                "mtask": (14, np.int32), "msucc": (15, np.int32), "mpairs": (16, np.int32),
                "tile_has_a": (17, np.int32)}


def stiles_symbolic_export(sym, kind):
    which, dt = EXPORT_KINDS[kind]
    lib = load_library()
    n = _i64()
    _check(lib.stiles_symbolic_export(sym, which, None, ctypes.byref(n)), "stiles_symbolic_export")
    out = np.empty(max(n.value, 1), dtype=dt)
    _check(lib.stiles_symbolic_export(sym, which, _ptr(out), ctypes.byref(n)), "stiles_symbolic_export")
    return out[:n.value]


def stiles_symbolic_destroy(sym):
    load_library().stiles_symbolic_destroy(sym)


def stiles_workspace_size(sym, precision, nrhs_max):
    b = ctypes.c_size_t()
    _check(load_library().stiles_workspace_size(sym, precision, nrhs_max, ctypes.byref(b)), "stiles_workspace_size")
    return b.value


def stiles_workspace_init(sym, precision, nrhs_max, d_ws, ws_bytes, stream=None):
    h = _vp()
    _check(load_library().stiles_workspace_init(sym, precision, nrhs_max, _ptr(d_ws), ws_bytes, _stream(stream),
                                                ctypes.byref(h)), "stiles_workspace_init")
    return h


def stiles_factorize(fac, d_values, stream=None):
    _check(load_library().stiles_factorize(fac, _ptr(d_values), _stream(stream)), "stiles_factorize")


def stiles_batch_workspace_size(facs):
    arr = (_vp * len(facs))(*[f.value for f in facs])
    b = ctypes.c_size_t()
    _check(load_library().stiles_batch_workspace_size(len(facs), arr, ctypes.byref(b)), "stiles_batch_workspace_size")
    return b.value


def stiles_factorize_batch(facs, d_values, d_batch_ws, batch_bytes, stream=None):
    arr = (_vp * len(facs))(*[f.value for f in facs])
    vals = (_vp * len(facs))(*[_ptr(v) for v in d_values])
    _check(load_library().stiles_factorize_batch(len(facs), arr, vals, _ptr(d_batch_ws), batch_bytes,
                                                 _stream(stream)), "stiles_factorize_batch")


def stiles_factor_info(fac, stream=None):
    v = _i64()
    _check(load_library().stiles_factor_info(fac, _stream(stream), ctypes.byref(v)), "stiles_factor_info")
    return v.value


def stiles_solve(fac, nrhs, d_B, ldb, stream=None):
    """Returns the report; rep.per_rhs = (backward errors, iteration counts),
    one entry per right-hand side."""
    rep = stiles_solve_report()
    berr = (ctypes.c_double * nrhs)()
    its = (ctypes.c_int32 * nrhs)()
    rep.backward_errors = ctypes.cast(berr, ctypes.POINTER(ctypes.c_double))
    rep.rhs_iterations = ctypes.cast(its, ctypes.POINTER(ctypes.c_int32))
    _check(load_library().stiles_solve(fac, nrhs, _ptr(d_B), ldb, _stream(stream), ctypes.byref(rep)), "stiles_solve")
    rep.per_rhs = (list(berr), list(its))
    return rep


def stiles_factorize_solve(fac, d_values, nrhs, d_B, ldb, stream=None):
    _check(load_library().stiles_factorize_solve(fac, _ptr(d_values), nrhs, _ptr(d_B), ldb, _stream(stream)),
           "stiles_factorize_solve")


def stiles_logdet(fac, d_out, stream=None):
    _check(load_library().stiles_logdet(fac, _ptr(d_out), _stream(stream)), "stiles_logdet")


def stiles_factorize_ooc(n_band, arrow, first_col, values, seg_rows, tile=64, stream=None, out=None):
    """Out-of-core factorization (host arrays in row-profile order): returns
    (L as a host array in the same layout, logdet, info, peak device bytes
    of one segment).  `out`: a float64 host array of values' size to receive
    L (reused across calls), else one is allocated."""
    first_col = np.ascontiguousarray(first_col, dtype=np.int64)
    values = np.ascontiguousarray(values, dtype=np.float64)
    if out is None:
        L = np.empty_like(values)
    else:
        if out.dtype != np.float64 or out.shape != values.shape or not out.flags["C_CONTIGUOUS"]:
            raise ValueError("out must be a contiguous float64 array of the values' shape")
        L = out
    ld, info, peak = ctypes.c_double(), _i64(), ctypes.c_size_t()
    _check(load_library().stiles_factorize_ooc(n_band, arrow, _ptr(first_col), _ptr(values), seg_rows, tile,
                                               _ptr(L), ctypes.byref(ld), ctypes.byref(info), ctypes.byref(peak),
                                               _stream(stream)), "stiles_factorize_ooc")
    return L, ld.value, info.value, peak.value


def stiles_logdet_static(fac, d_out, stream=None):
    _check(load_library().stiles_logdet_static(fac, _ptr(d_out), _stream(stream)), "stiles_logdet_static")


def stiles_factor_set_max_workgroups(fac, max_wg):
    _check(load_library().stiles_factor_set_max_workgroups(fac, max_wg), "stiles_factor_set_max_workgroups")


def stiles_factor_set_wait_limit(fac, seconds):
    _check(load_library().stiles_factor_set_wait_limit(fac, float(seconds)), "stiles_factor_set_wait_limit")


def stiles_factor_release(fac):
    load_library().stiles_factor_release(fac)


def stiles_factor_extract(fac, d_L, stream=None):
    _check(load_library().stiles_factor_extract(fac, _ptr(d_L), _stream(stream)), "stiles_factor_extract")


def stiles_factor_set_timing(fac, enable):
    _check(load_library().stiles_factor_set_timing(fac, 1 if enable else 0), "stiles_factor_set_timing")


def stiles_factor_kernel_ms(fac, which):
    v = ctypes.c_float()
    _check(load_library().stiles_factor_kernel_ms(fac, which, ctypes.byref(v)), "stiles_factor_kernel_ms")
    return v.value


def stiles_factor_set_trace(fac, d_factor_trace, d_solve_trace, stream=None):
    _check(load_library().stiles_factor_set_trace(fac, _ptr(d_factor_trace), _ptr(d_solve_trace), _stream(stream)),
           "stiles_factor_set_trace")


def stiles_factor_set_merged_trace(fac, d_trace, stream=None):
    _check(load_library().stiles_factor_set_merged_trace(fac, _ptr(d_trace), _stream(stream)),
           "stiles_factor_set_merged_trace")


def stiles_selinv_query(sym):
    """(tasks, algorithmic flops, executed flops) of the selected inversion."""
    n, fa, fe = _i64(), ctypes.c_double(), ctypes.c_double()
    _check(load_library().stiles_selinv_query(sym, ctypes.byref(n), ctypes.byref(fa), ctypes.byref(fe)),
           "stiles_selinv_query")
    return n.value, fa.value, fe.value


def stiles_selinv_workspace_size(sym):
    b = ctypes.c_size_t()
    _check(load_library().stiles_selinv_workspace_size(sym, ctypes.byref(b)), "stiles_selinv_workspace_size")
    return b.value


def stiles_selinv_create(fac, d_ws, ws_bytes, stream=None):
    h = _vp()
    _check(load_library().stiles_selinv_create(fac, _ptr(d_ws), ws_bytes, _stream(stream), ctypes.byref(h)),
           "stiles_selinv_create")
    return h


def stiles_selinv_compute(si, stream=None):
    _check(load_library().stiles_selinv_compute(si, _stream(stream)), "stiles_selinv_compute")


def stiles_selinv_diag(si, d_diag, stream=None):
    _check(load_library().stiles_selinv_diag(si, _ptr(d_diag), _stream(stream)), "stiles_selinv_diag")


def stiles_selinv_extract(si, d_out, stream=None):
    _check(load_library().stiles_selinv_extract(si, _ptr(d_out), _stream(stream)), "stiles_selinv_extract")


def stiles_selinv_set_timing(si, enable):
    _check(load_library().stiles_selinv_set_timing(si, 1 if enable else 0), "stiles_selinv_set_timing")


def stiles_selinv_kernel_ms(si):
    v = ctypes.c_float()
    _check(load_library().stiles_selinv_kernel_ms(si, ctypes.byref(v)), "stiles_selinv_kernel_ms")
    return v.value


def stiles_selinv_set_trace(si, d_trace, stream=None):
    _check(load_library().stiles_selinv_set_trace(si, _ptr(d_trace), _stream(stream)), "stiles_selinv_set_trace")


def stiles_selinv_destroy(si):
    load_library().stiles_selinv_destroy(si)


def stiles_status_string(st):
    return load_library().stiles_status_string(st).decode()


def stiles_last_error_arg():
    return load_library().stiles_last_error_arg()


# ------------------------------------------------------- convenience classes

class Symbolic:
    """Reordering + symbolic tile factorization of one sparsity pattern."""

    def __init__(self, handle):
        self.handle = handle
        self.info = stiles_symbolic_query(handle)

    @classmethod
    def from_profile(cls, n_band, arrow, first_col, **opt):
        return cls(stiles_analyze_profile(n_band, arrow, first_col, stiles_default_opts(**opt)))

    @classmethod
    def from_pattern(cls, pattern, **opt):
        return cls.from_profile(pattern.n, pattern.a, pattern.band_first_col, **opt)

    @classmethod
    def from_csc(cls, N, arrow, colptr, rowind, **opt):
        return cls(stiles_analyze(N, arrow, colptr, rowind, stiles_default_opts(**opt)))

    @property
    def N(self):
        return self.info.N

    def perm(self):
        return stiles_symbolic_perm(self.handle, self.info.N)

    def workspace_size(self, precision=STILES_FP64, nrhs_max=1):
        return stiles_workspace_size(self.handle, precision, nrhs_max)

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.stiles_symbolic_destroy(self.handle)
            self.handle = None


class Factor:
    """A resident factor: a device workspace (torch uint8 tensor) bound to a
    symbolic object.  factorize() may be called again with new values."""

    def __init__(self, sym, precision=STILES_FP64, nrhs_max=1, device="cuda", stream=None, workspace=None):
        import torch
        self.sym = sym
        self.precision = precision
        self.nrhs_max = nrhs_max
        self.bytes = sym.workspace_size(precision, nrhs_max)
        if workspace is None:
            workspace = torch.empty(self.bytes + 256, dtype=torch.uint8, device=device)
        self.workspace = workspace
        base = workspace.data_ptr()
        self._ws_addr = (base + 255) // 256 * 256
        if self._ws_addr + self.bytes > base + workspace.numel():
            raise ValueError("workspace tensor too small")
        h = _vp()
        _check(load_library().stiles_workspace_init(sym.handle, precision, nrhs_max, ctypes.c_void_p(self._ws_addr),
                                                    self.bytes, _stream(stream), ctypes.byref(h)),
               "stiles_workspace_init")
        self.handle = h

    def set_max_workgroups(self, n):
        stiles_factor_set_max_workgroups(self.handle, n)

    def set_wait_limit(self, seconds):
        stiles_factor_set_wait_limit(self.handle, seconds)

    def factorize(self, d_values, stream=None):
        stiles_factorize(self.handle, d_values, stream)
        return self

    def info(self, stream=None):
        return stiles_factor_info(self.handle, stream)

    def solve(self, B, stream=None):
        """In-place solve of a (N,) or (N, nrhs) float64 device tensor
        (column-major storage, i.e. B.t() contiguous, or a 1-D vector)."""
        if B.dim() == 1:
            rep = stiles_solve(self.handle, 1, B, B.shape[0], stream)
        else:
            if B.stride(0) != 1:
                raise ValueError("B must be column-major (use X.t().contiguous().t())")
            rep = stiles_solve(self.handle, B.shape[1], B, B.stride(1), stream)
        return rep

    def factorize_solve(self, d_values, B, stream=None):
        """factorize(d_values) then an in-place solve of B, as one launch
        (FP64); B as for solve()."""
        if B.dim() == 1:
            stiles_factorize_solve(self.handle, d_values, 1, B, B.shape[0], stream)
        else:
            if B.stride(0) != 1:
                raise ValueError("B must be column-major (use X.t().contiguous().t())")
            stiles_factorize_solve(self.handle, d_values, B.shape[1], B, B.stride(1), stream)
        return self

    def extract(self, stream=None):
        """L in row-profile order of the permuted envelope (device tensor)."""
        import torch
        out = torch.empty(self.sym.info.nnz_L, dtype=torch.float64, device=self.workspace.device)
        stiles_factor_extract(self.handle, out, stream)
        return out

    def logdet(self, out=None, stream=None):
        import torch
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.workspace.device)
        stiles_logdet(self.handle, out, stream)
        return out

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.stiles_factor_release(self.handle)
            self.handle = None


class SelInv:
    """Selected inversion bound to a resident factor: compute() fills Sigma =
    A^{-1} on the factor's tile pattern; diag() and extract() read it out."""

    def __init__(self, factor, stream=None):
        import torch
        self.factor = factor
        self.bytes = stiles_selinv_workspace_size(factor.sym.handle)
        self.ws = torch.empty(self.bytes + 256, dtype=torch.uint8, device=factor.workspace.device)
        addr = (self.ws.data_ptr() + 255) // 256 * 256
        h = _vp()
        _check(load_library().stiles_selinv_create(factor.handle, ctypes.c_void_p(addr), self.bytes, _stream(stream),
                                                   ctypes.byref(h)), "stiles_selinv_create")
        self.handle = h

    def compute(self, stream=None):
        stiles_selinv_compute(self.handle, stream)
        return self

    def diag(self, out=None, stream=None):
        """(A^{-1})_ii in the original ordering (float64 device tensor)."""
        import torch
        if out is None:
            out = torch.empty(self.factor.sym.info.N, dtype=torch.float64, device=self.ws.device)
        stiles_selinv_diag(self.handle, out, stream)
        return out

    def extract(self, stream=None):
        """Selected entries in the layout of Factor.extract()."""
        import torch
        out = torch.empty(self.factor.sym.info.nnz_L, dtype=torch.float64, device=self.ws.device)
        stiles_selinv_extract(self.handle, out, stream)
        return out

    def set_timing(self, enable=True):
        stiles_selinv_set_timing(self.handle, enable)

    def kernel_ms(self):
        return stiles_selinv_kernel_ms(self.handle)

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.stiles_selinv_destroy(self.handle)
            self.handle = None


class Batch:
    """Many factors run in one persistent launch; the merged schedule is
    uploaded once (stiles_batch_create) and reused by every factorize()."""

    def __init__(self, factors, stream=None):
        import torch
        self.factors = list(factors)
        hs = [f.handle for f in self.factors]
        need = stiles_batch_workspace_size(hs)
        self.ws = torch.empty(need + 256, dtype=torch.uint8, device=self.factors[0].workspace.device)
        addr = (self.ws.data_ptr() + 255) // 256 * 256
        arr = (_vp * len(hs))(*[h.value for h in hs])
        h = _vp()
        _check(load_library().stiles_batch_create(len(hs), arr, ctypes.c_void_p(addr), need, _stream(stream),
                                                  ctypes.byref(h)), "stiles_batch_create")
        self.handle = h

    def factorize(self, values, stream=None):
        ptrs = tuple(_ptr(v) for v in values)
        if getattr(self, "_ptrs", None) != ptrs:
            self._ptrs = ptrs
            self._vals = (_vp * len(ptrs))(*ptrs)
        _check(load_library().stiles_batch_factorize(self.handle, self._vals, _stream(stream)), "stiles_batch_factorize")

    def logdet(self, out=None, stream=None):
        """Log-determinants of all matrices (float64 device tensor of length count)."""
        import torch
        if out is None:
            out = torch.empty(len(self.factors), dtype=torch.float64, device=self.ws.device)
        if out.numel() < len(self.factors) or out.dtype != torch.float64:
            raise ValueError("Batch.logdet: out needs %d float64 entries" % len(self.factors))
        stiles_batch_logdet(self.handle, out, stream)
        return out

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.stiles_batch_destroy(self.handle)
            self.handle = None


def stiles_batch_create(facs, d_batch_ws, batch_bytes, stream=None):
    arr = (_vp * len(facs))(*[f.value for f in facs])
    h = _vp()
    _check(load_library().stiles_batch_create(len(facs), arr, _ptr(d_batch_ws), batch_bytes, _stream(stream),
                                              ctypes.byref(h)), "stiles_batch_create")
    return h


def stiles_batch_factorize(batch, d_values, stream=None):
    vals = (_vp * len(d_values))(*[_ptr(v) for v in d_values])
    _check(load_library().stiles_batch_factorize(batch, vals, _stream(stream)), "stiles_batch_factorize")


def stiles_batch_logdet(batch, d_out, stream=None):
    _check(load_library().stiles_batch_logdet(batch, _ptr(d_out), _stream(stream)), "stiles_batch_logdet")


def stiles_batch_destroy(batch):
    load_library().stiles_batch_destroy(batch)


def factorize_batch(factors, values, batch_ws=None, stream=None):
    """One persistent launch over many factors (distinct workspaces, one tile size)."""
    import torch
    hs = [f.handle for f in factors]
    need = stiles_batch_workspace_size(hs)
    if batch_ws is None or batch_ws.numel() < need + 256:
        batch_ws = torch.empty(need + 256, dtype=torch.uint8, device=factors[0].workspace.device)
    addr = (batch_ws.data_ptr() + 255) // 256 * 256
    arr = (_vp * len(hs))(*[h.value for h in hs])
    vals = (_vp * len(hs))(*[_ptr(v) for v in values])
    _check(load_library().stiles_factorize_batch(len(hs), arr, vals, ctypes.c_void_p(addr), need, _stream(stream)),
           "stiles_factorize_batch")
    return batch_ws
