"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only builds input matrices (sparsity profiles and values); it
holds none of the factorization's arithmetic.  Both the HIP path and the CPU
oracle consume exactly the arrays produced here.

Shapes follow the block-arrowhead matrices of the sTiles paper (Section I and
the matrix-properties table of Section V: band of a given half-width plus a
dense trailing arrow of at most ~200 columns).  The paper's INLA matrices are
not available; these generators stand in for them.

Layout ("row profile"): a matrix of order N = n + a is described by
f[0..N-1], the first structurally nonzero column of each lower-triangle row.
Band rows i < n have f[i] = max(0, i - w_i); the a arrow rows have f = 0.
Values are stored row by row, row i holding columns f[i]..i (diagonal last).

Value law: off-diagonal entries are drawn N(0,1) in row-profile order (row i
ascending, column ascending; the arrow rows come last, row-major), from
numpy's PCG64 default_rng(seed).  The diagonal is then set to the absolute
sum of the full symmetric row plus one, which makes the matrix strictly
diagonally dominant, hence SPD (Gershgorin).  The "laplacian" law instead
uses -|N(0,1)| off-diagonals and diagonal = absolute row sum + eps, a weighted
graph Laplacian plus eps*I whose smallest eigenvalue is exactly eps.
"""
import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Pattern:
    """Band-plus-arrow envelope: n band rows, a arrow rows, first columns f."""
    n: int
    a: int
    f: np.ndarray            # int64, length N = n + a
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def N(self):
        return self.n + self.a

    @property
    def band_first_col(self):
        return self.f[: self.n]

    def row_ptr(self):
        lens = np.arange(self.N, dtype=np.int64) - self.f + 1
        rp = np.zeros(self.N + 1, dtype=np.int64)
        np.cumsum(lens, out=rp[1:])
        return rp

    @property
    def nnz(self):
        return int(np.sum(np.arange(self.N, dtype=np.int64) - self.f + 1))


def band_first_cols(n, widths, seg=None):
    """f_i = max(0, i - w(i)); widths is an int (constant half-width) or one
    width per segment of `seg` rows (piecewise-constant half-width)."""
    i = np.arange(n, dtype=np.int64)
    if np.isscalar(widths):
        w = np.full(n, int(widths), dtype=np.int64)
    else:
        widths = np.asarray(widths, dtype=np.int64)
        w = widths[np.minimum(i // seg, widths.shape[0] - 1)]
    return np.maximum(0, i - w)


def make_pattern(n, a, widths, seg=None, name=""):
    f = np.zeros(n + a, dtype=np.int64)
    f[:n] = band_first_cols(n, widths, seg)
    return Pattern(n=n, a=a, f=f, name=name)


def _col_abs_sums(f, rp, absoff, N, chunk=1 << 25):
    """Sum of |A_ki| over lower entries (k, i), k > i, i.e. the upper half of row i."""
    out = np.zeros(N, dtype=np.float64)
    r0 = 0
    while r0 < N:
        r1 = r0
        # grow the row block until it holds about `chunk` entries
        r1 = int(np.searchsorted(rp, rp[r0] + chunk, side="right"))
        r1 = max(r1, r0 + 1)
        r1 = min(r1, N)
        lo, hi = rp[r0], rp[r1]
        lens = (rp[r0 + 1:r1 + 1] - rp[r0:r1])
        rows = np.repeat(np.arange(r0, r1, dtype=np.int64), lens)
        cols = np.arange(lo, hi, dtype=np.int64) - rp[rows] + f[rows]
        out += np.bincount(cols, weights=absoff[lo:hi], minlength=N)
        r0 = r1
    return out


def make_values(pattern, seed, law="dominant", kappa=1e6):
    """Values of an SPD matrix on `pattern` (row-profile order, float64)."""
    f = pattern.f
    N = pattern.N
    rp = pattern.row_ptr()
    nnz = int(rp[-1])
    rng = np.random.default_rng(seed)
    v = np.empty(nnz, dtype=np.float64)
    diag_pos = rp[1:] - 1
    # off-diagonal draws in row-profile order, row by row (chunked to bound memory)
    r0 = 0
    chunk = 1 << 25
    while r0 < N:
        r1 = int(np.searchsorted(rp, rp[r0] + chunk, side="right"))
        r1 = min(max(r1, r0 + 1), N)
        lo, hi = rp[r0], rp[r1]
        mask = np.ones(hi - lo, dtype=bool)
        mask[diag_pos[r0:r1] - lo] = False
        draws = rng.standard_normal(int(hi - lo - (r1 - r0)))
        if law == "laplacian":
            draws = -np.abs(draws)
        seg = v[lo:hi]
        seg[mask] = draws
        seg[~mask] = 0.0
        r0 = r1
    absoff = np.abs(v)
    row_abs = np.add.reduceat(absoff, rp[:-1]) if N > 0 else np.zeros(0)
    col_abs = _col_abs_sums(f, rp, absoff, N)
    tot = row_abs + col_abs
    if law == "dominant":
        v[diag_pos] = tot + 1.0
    elif law == "laplacian":
        gersh = 2.0 * float(tot.max()) if N else 1.0
        eps = gersh / kappa
        v[diag_pos] = tot + eps
    else:
        raise ValueError(law)
    return v


def scale_values(pattern, values, seed, decades=3.0):
    """Symmetric diagonal scaling S A S with s_i = 10^(-decades*u_i), u ~ U[0,1)."""
    rng = np.random.default_rng(seed)
    s = 10.0 ** (-decades * rng.random(pattern.N))
    rp = pattern.row_ptr()
    lens = rp[1:] - rp[:-1]
    rows = np.repeat(np.arange(pattern.N, dtype=np.int64), lens)
    cols = np.arange(rp[-1], dtype=np.int64) - rp[rows] + pattern.f[rows]
    return values * s[rows] * s[cols]


def rhs(N, nrhs, seed):
    """Right-hand sides N(0,1), column-major (N, nrhs)."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.standard_normal((nrhs, N)).T)


# ---------------------------------------------------------------- workloads

def single_small():
    """Plain FP64 single factorize+solve: n=2,000, half-width 50, arrow 10."""
    return make_pattern(2000, 10, 50, name="band2000_w50_a10")


def variable_band(seed=2, n=200_000, seg=5000, wlo=200, whi=800, a=100):
    """Variable bandwidth: half-width piecewise constant per 5,000-row
    segment, uniform in [200, 800]; arrow of 100."""
    rng = np.random.default_rng(seed)
    nseg = (n + seg - 1) // seg
    widths = rng.integers(wlo, whi + 1, size=nseg)
    p = make_pattern(n, a, widths, seg=seg, name="varband%d_a%d" % (n, a))
    p.meta["widths"] = widths
    return p


def batch_patterns(seed=3, count=512, nlo=1000, nhi=20000, wlo=32, whi=256, alo=4, ahi=64):
    """Batch of uneven band-arrowhead matrices (n log-uniform, w, a uniform)."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        n = int(round(math.exp(rng.uniform(math.log(nlo), math.log(nhi)))))
        w = int(rng.integers(wlo, whi + 1))
        a = int(rng.integers(alo, ahi + 1))
        p = make_pattern(n, a, w, name="batch%d" % b)
        p.meta.update(dict(w=w, value_seed=3000 + b))
        out.append(p)
    return out


def mixed_large(n=500_000, w=1000, a=200):
    """Mixed-precision workload: n=500,000, half-width 1,000, arrow 200."""
    return make_pattern(n, a, w, name="band%d_w%d_a%d" % (n, w, a))


def serving_patterns(seed=5):
    """Eight resident patterns for the serving workload."""
    rng = np.random.default_rng(seed)
    specs = [(10_000, 64, 16)]
    for _ in range(6):
        n = int(round(math.exp(rng.uniform(math.log(1e4), math.log(3e5)))))
        w = int(rng.integers(64, 801))
        a = int(rng.integers(16, 201))
        specs.append((n, w, a))
    specs.append((300_000, 800, 200))
    return [make_pattern(n, a, w, name="serve%d" % i) for i, (n, w, a) in enumerate(specs)]


def serving_requests(npat, count, qps, seed=55, value_seed0=5000):
    """Poisson arrivals: (arrival time s, pattern index, op, value seed)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, size=count)
    t = np.cumsum(gaps)
    pats = rng.integers(0, npat, size=count)
    ops = rng.integers(0, 3, size=count)    # 0 factorize, 1 +solve(1 RHS), 2 +logdet
    return [(float(t[i]), int(pats[i]), int(ops[i]), value_seed0 + i) for i in range(count)]


def spde_space_time(nx, ny, nt, a, seed, name=""):
    """Sparse-inside-the-envelope input shaped like the spatio-temporal
    precision matrices INLA factors (Section I): nodes (t, y, x) in time-major,
    then row-major order; node i couples to the nodes of its own and of the
    adjacent time steps within spatial distance |dx| + |dy| <= 2 (the stencil
    of (kappa^2 - Laplacian)^2 on a grid, times an AR(1) coupling in time);
    `a` dense arrow rows (fixed effects).  Values: N(0,1) off the diagonal in
    (row, column) order, diagonal = absolute sum of the full symmetric row + 1.
    Returns a dict: N, n, a, CSC of the lower triangle (colptr, rowind,
    values in CSC order) and the natural order's row profile (a Pattern and
    the values in row-profile order, zeros where the envelope has no entry)."""
    n = nx * ny * nt
    N = n + a
    idx = np.arange(n, dtype=np.int64)
    t, rem = np.divmod(idx, nx * ny)
    y, x = np.divmod(rem, nx)
    rows, cols = [], []
    # lower neighbours: the whole stencil at t - 1, the part before (y, x) at t
    for dt in (-1, 0):
        for dy in range(-2, 3):
            for dx in range(-2, 3):
                if abs(dx) + abs(dy) > 2 or (dt == 0 and (dy, dx) >= (0, 0)):
                    continue
                ok = (t + dt >= 0) & (y + dy >= 0) & (y + dy < ny) & (x + dx >= 0) & (x + dx < nx)
                i = idx[ok]
                rows.append(i)
                cols.append(i + dt * nx * ny + dy * nx + dx)
    return _assemble(n, a, rows, cols, seed, name or "spde%dx%dx%d_a%d" % (nx, ny, nt, a))


def irregular_mesh(n, a, seed, k=6, long_edges=0, name=""):
    """Irregular-pattern input (the case Section III-A names for minimum-degree
    orderings): n points uniform in the unit square, each joined to its k
    nearest neighbours (symmetrized), plus `long_edges` couplings between
    random pairs of points (a poor-quality mesh), numbered in random order
    (no locality in the numbering), plus `a` dense arrow rows.  Values and
    return value as for spde_space_time (the row profile only when it is
    small enough to hold)."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    _, nb = cKDTree(pts).query(pts, k=k + 1)
    num = rng.permutation(n).astype(np.int64)          # node -> row index
    lu = rng.integers(0, n, size=long_edges)
    lv = rng.integers(0, n, size=long_edges)
    keep = lu != lv
    u = np.concatenate([np.repeat(num, k), num[lu[keep]]])
    v = np.concatenate([num[nb[:, 1:].reshape(-1)], num[lv[keep]]])
    hi, lo = np.maximum(u, v), np.minimum(u, v)
    key = np.unique(hi * n + lo)
    return _assemble(n, a, [key // n], [key % n], seed + 1, name or "mesh%d_k%d_l%d_a%d" % (n, k, long_edges, a))


def _assemble(n, a, rows, cols, seed, name):
    """Lower CSC + row profile of an SPD matrix with the given strictly lower
    band entries (rows[i] > cols[i]) and `a` dense arrow rows; off-diagonal
    values N(0,1) in (row, column) order, diagonal = absolute sum of the full
    symmetric row + 1."""
    N = n + a
    rows, cols = list(rows), list(cols)
    # arrow rows: dense
    ar = np.repeat(np.arange(n, N, dtype=np.int64), np.arange(n, N))
    ac = np.concatenate([np.arange(r, dtype=np.int64) for r in range(n, N)]) if a else np.zeros(0, np.int64)
    rows.append(ar)
    cols.append(ac)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    order = np.lexsort((c, r))            # (row, column) order for the draws
    r, c = r[order], c[order]
    rng = np.random.default_rng(seed)
    off = rng.standard_normal(r.shape[0])
    dsum = np.zeros(N)
    np.add.at(dsum, r, np.abs(off))
    np.add.at(dsum, c, np.abs(off))
    dr = np.arange(N, dtype=np.int64)
    R = np.concatenate([r, dr])
    C = np.concatenate([c, dr])
    V = np.concatenate([off, dsum + 1.0])
    co = np.lexsort((R, C))               # CSC: column, then row
    colptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(C, minlength=N), out=colptr[1:])
    f = np.arange(N, dtype=np.int64)
    np.minimum.at(f, R, C)
    pat = Pattern(n=n, a=a, f=f, name=name)
    rp = pat.row_ptr()
    prof = None
    if rp[-1] <= 1 << 28:
        prof = np.zeros(int(rp[-1]))
        prof[rp[R] + (C - f[R])] = V
    return {"N": N, "n": n, "a": a, "colptr": colptr, "rowind": R[co].copy(), "values": np.ascontiguousarray(V[co]),
            "pattern": pat, "profile_values": prof}


# ------------------------------------------------------------ format helpers

def to_dense(pattern, values):
    """Dense symmetric matrix from the lower envelope (small inputs only)."""
    N = pattern.N
    A = np.zeros((N, N))
    rp = pattern.row_ptr()
    for i in range(N):
        A[i, pattern.f[i]:i + 1] = values[rp[i]:rp[i + 1]]
    return np.tril(A) + np.tril(A, -1).T


def to_lower_csc(pattern, values):
    """Lower-triangle CSC (colptr, rowind, values-in-CSC-order) of the envelope."""
    N = pattern.N
    rp = pattern.row_ptr()
    lens = rp[1:] - rp[:-1]
    rows = np.repeat(np.arange(N, dtype=np.int64), lens)
    cols = np.arange(rp[-1], dtype=np.int64) - rp[rows] + pattern.f[rows]
    order = np.lexsort((rows, cols))
    colptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(np.bincount(cols, minlength=N), out=colptr[1:])
    return colptr, rows[order].copy(), np.ascontiguousarray(values[order])
