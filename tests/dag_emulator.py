"""Host emulation of the task DAGs that the GPU executor runs.

The plan (tasks, successor lists, tile pairs, tile pattern) is read from a
symbolic object through stiles_symbolic_export and executed here with numpy
tile operations, in the schedule's ticket order or in a random order among
the tasks whose predecessors are done.  This checks the planner on the CPU:
a missing dependency, a wrong pair list or a wrong tree would change the
result (compared with the FP64 oracle), and a cycle would leave tasks
unexecuted.  Task semantics follow the comments of stiles_internal.h."""
import numpy as np

import paper_2501_02483_amd as S

UPD, PART, TREE, POTRF, TRSM, UPDB = 1, 2, 3, 4, 5, 6
FUPD, FDIAG, BUPD, BDIAG, FPART, FSUM = 8, 9, 10, 11, 12, 13
SWE, SW, SDIAG, TSUM = 16, 17, 18, 19
TF_DIAG, TF_FIRST, TF_ACC, TF_SPLIT = 1 << 8, 1 << 9, 1 << 10, 1 << 11
SIG_TRANS = 1 << 30
MERGED_FDEP, SUCC_FDEP = 1 << 16, 1 << 30
SPLIT_W, SUCC_MID = 1 << 8, 1 << 29


def succ_edge(v):
    """(successor, counter decrement) of a successor entry: an entry with
    SUCC_FDEP (an early predecessor of a two-stage task; in the merged DAG
    also factorization task -> solve task) subtracts MERGED_FDEP, one with
    SUCC_MID (merged DAG: early solve predecessor of a two-stage diagonal
    step) SPLIT_W."""
    v = int(v)
    if v & SUCC_FDEP:
        return v & ~SUCC_FDEP, MERGED_FDEP
    if v & SUCC_MID:
        return v & ~SUCC_MID, SPLIT_W
    return v, 1


class Plan:
    def __init__(self, sym):
        h = sym.handle
        ex = lambda k: S.stiles_symbolic_export(h, k)
        self.T = sym.info.tile
        self.ftask = ex("ftask").reshape(-1, 8)
        self.fsucc = ex("fsucc")
        self.fpairs = ex("fpairs").reshape(-1, 2)
        self.stask = ex("stask").reshape(-1, 8)
        self.ssucc = ex("ssucc")
        self.spairs = ex("spairs").reshape(-1, 2)
        self.trow_ptr = ex("trow_ptr")
        self.tcol = ex("tcol")
        self.row_base = ex("row_base")
        self.row_cnt = ex("row_cnt")
        self.npart = int(ex("npart")[0])
        self.ntr = len(self.trow_ptr) - 1
        self.trow = np.repeat(np.arange(self.ntr), np.diff(self.trow_ptr))
        self.perm = sym.perm()
        self.N = sym.info.N
        self._sym = sym

    def selinv_tables(self):
        ex = lambda k: S.stiles_symbolic_export(self._sym.handle, k)
        return ex("itask").reshape(-1, 8), ex("isucc"), ex("ilist")


def _order(tasks, succ, mode, rng):
    n = len(tasks)
    if mode == "ticket":
        # ticket order must be topological: every successor has a larger index
        for t in range(n):
            for q in range(tasks[t, 5], tasks[t, 6]):
                assert succ_edge(succ[q])[0] > t
        return list(range(n))
    rem = tasks[:, 7].copy()
    ready = [t for t in range(n) if rem[t] == 0]
    out = []
    while ready:
        i = int(rng.integers(len(ready)))
        t = ready.pop(i)
        out.append(t)
        for q in range(tasks[t, 5], tasks[t, 6]):
            s, dec = succ_edge(succ[q])
            rem[s] -= dec
            assert rem[s] >= 0
            if rem[s] == 0:
                ready.append(s)
    assert len(out) == n, "DAG has a cycle or a wrong predecessor count"
    return out


def scatter(plan, Aperm):
    """Tile store of the permuted dense matrix (lower triangle), unit padding."""
    T = plan.T
    tiles = np.zeros((len(plan.tcol), T, T))
    for t in range(len(plan.tcol)):
        m, j = plan.trow[t], plan.tcol[t]
        rb, cb, rc, cc = plan.row_base[m], plan.row_base[j], plan.row_cnt[m], plan.row_cnt[j]
        blk = np.zeros((T, T))
        blk[:rc, :cc] = Aperm[rb:rb + rc, cb:cb + cc]
        if m == j:
            blk = np.tril(blk)
            for r in range(rc, T):
                blk[r, r] = 1.0
        tiles[t] = blk
    return tiles


def update_block(w, P, tiles, done=None):
    """UPDB: a 2 x 2 block of targets (ra,k), (rb,k), (ra,k+1), (rb,k+1)
    (-1: absent); per column j the operands (ra,j), (rb,j), (k,j), (k+1,j).
    `done` (merged emulation): the operand tiles must be final."""
    words = P.reshape(-1)[2 * w[2]:2 * w[2] + 4 + 4 * w[3]]
    tg = words[:4]
    ops = words[4:].reshape(-1, 4)
    if done is not None:
        o = ops.reshape(-1)
        assert done[o[o >= 0]].all(), "block update read a tile before it was final"
    for q in range(4):
        if tg[q] < 0:
            continue
        use = [o for o in ops if o[q & 1] >= 0 and o[2 + (q >> 1)] >= 0]   # -1: absent operand
        if not use:
            continue
        acc = sum(tiles[o[q & 1]] @ tiles[o[2 + (q >> 1)]].T for o in use)
        diag = (w[0] & TF_DIAG) and q != 1
        tiles[tg[q]] -= np.tril(acc) if diag else acc


def factor(plan, Aperm, mode="ticket", seed=0):
    rng = np.random.default_rng(seed)
    T = plan.T
    tiles = scatter(plan, Aperm)
    linv = np.zeros((plan.ntr, T, T))
    part = np.zeros((max(plan.npart, 1), T, T))
    P = plan.fpairs
    for t in _order(plan.ftask, plan.fsucc, mode, rng):
        w = plan.ftask[t]
        typ = w[0] & 0xff
        if typ in (UPD, PART):
            acc = sum(tiles[P[p, 0]] @ tiles[P[p, 1]].T for p in range(w[2], w[3]))
            if typ == UPD:
                if w[0] & TF_DIAG:
                    tiles[w[1]] -= np.tril(acc)
                else:
                    tiles[w[1]] -= acc
            elif w[0] & TF_ACC:
                part[w[4]] += acc
            else:
                part[w[4]] = acc
        elif typ == UPDB:
            update_block(w, P, tiles)
        elif typ == TREE:
            s = part[w[2]] + (part[w[3]] if w[3] >= 0 else 0.0)
            if w[4] >= 0:
                part[w[4]] = s
            else:
                tiles[w[1]] -= s
        elif typ == POTRF:
            C = tiles[w[1]].copy()
            for p in range(w[3], w[4]):
                C -= tiles[P[p, 0]] @ tiles[P[p, 1]].T
            Cs = np.tril(C) + np.tril(C, -1).T
            L = np.linalg.cholesky(Cs)
            tiles[w[1]] = L
            linv[w[2]] = np.linalg.inv(L)
        elif typ == TRSM:
            C = tiles[w[1]].copy()
            for p in range(w[3], w[4]):
                C -= tiles[P[p, 0]] @ tiles[P[p, 1]].T
            tiles[w[1]] = C @ linv[w[2]].T
        else:
            raise AssertionError("unknown factor task type %d" % typ)
    return tiles, linv


def dense_factor(plan, tiles):
    """Dense lower factor of the permuted matrix from the tile store."""
    L = np.zeros((plan.N, plan.N))
    for t in range(len(plan.tcol)):
        m, j = plan.trow[t], plan.tcol[t]
        rb, cb, rc, cc = plan.row_base[m], plan.row_base[j], plan.row_cnt[m], plan.row_cnt[j]
        L[rb:rb + rc, cb:cb + cc] = tiles[t][:rc, :cc]
    return np.tril(L)


def _split_order(tasks, succ, rng, late_of=None, eager=False):
    """A random topological order of the solve DAG in which every two-stage
    diagonal step (TF_SPLIT) is two sub-tasks: stage 0 after its early
    predecessors (the successor entries with SUCC_FDEP), stage 1 after
    stage 0 and its late predecessor.  Items are (task, stage), stage None
    for a single-stage task.  late_of (task -> predecessor) overrides which
    predecessor counts as late; eager runs a ready stage 0 before anything
    else (the first stages as early as their predecessors allow)."""
    n = len(tasks)
    split = [bool(tasks[t, 0] & TF_SPLIT) for t in range(n)]
    preds = [[] for _ in range(n)]
    late = {}
    for t in range(n):
        for q in range(tasks[t, 5], tasks[t, 6]):
            x, dec = succ_edge(succ[q])
            preds[x].append(t)
            if split[x] and dec == 1:
                assert x not in late, "a two-stage step has one late predecessor"
                late[x] = t
    if late_of is not None:
        late.update(late_of)
    nodes = []
    for t in range(n):
        nodes += [(t, 0), (t, 1)] if split[t] else [(t, None)]
    final = lambda t: (t, 1) if split[t] else (t, None)
    need = {}
    for t in range(n):
        if split[t]:
            assert t in late
            need[(t, 0)] = {final(x) for x in preds[t] if x != late[t]}
            need[(t, 1)] = {(t, 0), final(late[t])}
        else:
            need[(t, None)] = {final(x) for x in preds[t]}
    done, out = set(), []
    ready = [v for v in nodes if not need[v]]
    waiting = {v: set(need[v]) for v in nodes if need[v]}
    users = {}
    for v, ps in waiting.items():
        for u in ps:
            users.setdefault(u, []).append(v)
    while ready:
        first = [i for i, v in enumerate(ready) if v[1] == 0] if eager else []
        v = ready.pop(first[0] if first else int(rng.integers(len(ready))))
        out.append(v)
        done.add(v)
        for u in users.get(v, []):
            waiting[u].discard(v)
            if not waiting[u]:
                ready.append(u)
    assert len(out) == len(nodes), "split DAG has a cycle"
    return out


def solve(plan, tiles, linv, B, mode="ticket", seed=0, late_of=None):
    """Forward and backward sweeps by the plan's solve tasks.  mode "ticket",
    "random" (whole tasks), "split": two-stage diagonal steps run as two
    sub-tasks (their first fused product before the late predecessor) in a
    random order, or "split_eager": the same with every first stage run as
    soon as it is ready; backward blocks not yet written read as NaN."""
    rng = np.random.default_rng(seed)
    T, ntr = plan.T, plan.ntr
    nrhs = B.shape[1]
    Y = np.zeros((ntr, T, nrhs))
    Bp = B[plan.perm]
    for m in range(ntr):
        rb, rc = plan.row_base[m], plan.row_cnt[m]
        Y[m, :rc] = Bp[rb:rb + rc]
    Z = np.full_like(Y, np.nan)
    Q = {}
    P = plan.spairs
    if mode in ("split", "split_eager"):
        items = _split_order(plan.stask, plan.ssucc, rng, late_of, eager=mode == "split_eager")
    else:
        items = [(t, None) for t in _order(plan.stask, plan.ssucc, mode, rng)]
    held = {}
    for t, stage in items:
        w = plan.stask[t]
        typ = w[0] & 0xff
        m = w[1]
        if stage is not None:
            # a two-stage diagonal step: stage 0 takes its right-hand side
            # block and the first fused product, stage 1 the second product
            # and the inverse diagonal tile
            assert typ in (FDIAG, BDIAG) and w[3] - w[2] == 2
            p = w[2] + stage
            if typ == FDIAG:
                if stage == 0:
                    held[t] = Y[m].copy() - tiles[P[p, 0]] @ Y[P[p, 1]]
                else:
                    Y[m] = linv[m] @ (held.pop(t) - tiles[P[p, 0]] @ Y[P[p, 1]])
            else:
                if stage == 0:
                    base = Y[m] if w[0] & TF_FIRST else Z[m]
                    held[t] = base.copy() - tiles[P[p, 0]].T @ Z[P[p, 1]]
                else:
                    Z[m] = linv[m].T @ (held.pop(t) - tiles[P[p, 0]].T @ Z[P[p, 1]])
            continue
        if typ == FUPD:
            for p in range(w[2], w[3]):
                Y[m] -= tiles[P[p, 0]] @ Y[P[p, 1]]
        elif typ == FPART:
            q = np.zeros_like(Y[m])
            for p in range(w[2], w[3]):
                q += tiles[P[p, 0]] @ Y[P[p, 1]]
            Q[w[4]] = q
        elif typ == FSUM:
            for s in range(w[2], w[3]):
                Y[m] -= Q.pop(s)
        elif typ == FDIAG:
            v = Y[m].copy()
            for p in range(w[2], w[3]):
                v -= tiles[P[p, 0]] @ Y[P[p, 1]]
            Y[m] = linv[m] @ v
        elif typ == BUPD:
            v = (Y[m] if w[0] & TF_FIRST else Z[m]).copy()
            for p in range(w[2], w[3]):
                v -= tiles[P[p, 0]].T @ Z[P[p, 1]]
            Z[m] = v
        elif typ == BDIAG:
            v = (Y[m] if w[0] & TF_FIRST else Z[m]).copy()
            for p in range(w[2], w[3]):
                v -= tiles[P[p, 0]].T @ Z[P[p, 1]]
            Z[m] = linv[m].T @ v
        else:
            raise AssertionError("unknown solve task type %d" % typ)
    X = np.zeros_like(B)
    Xp = np.zeros_like(B)
    for m in range(ntr):
        rb, rc = plan.row_base[m], plan.row_cnt[m]
        Xp[rb:rb + rc] = Z[m, :rc]
    X[plan.perm] = Xp
    return X


def selinv(plan, tiles, linv, mode="ticket", seed=0):
    """Selected inversion (Sigma = A^{-1} on the tile pattern) by the plan's
    SWE / SW / SDIAG tasks; returns the Sigma tiles."""
    rng = np.random.default_rng(seed)
    itask, isucc, lst = plan.selinv_tables()
    sigma = np.full_like(tiles, np.nan)
    dpart, qpart = {}, {}

    def sig(code):
        x = sigma[code & ~SIG_TRANS]
        assert not np.isnan(x).any(), "Sigma tile read before it was written"
        return x.T if code & SIG_TRANS else x

    for t in _order(itask, isucc, mode, rng):
        w = itask[t]
        typ = w[0] & 0xff
        if typ == SWE:
            acc = sum(sig(lst[w[2] + 2 * q]) @ tiles[lst[w[2] + 2 * q + 1]] for q in range(w[3]))
            sigma[w[1]] = sigma[w[1]] + acc if w[0] & TF_ACC else acc
        elif typ == SW:
            o = w[3]
            nsum, npush, nprod = w[4] & 0xff, (w[4] >> 8) & 0xff, w[4] >> 16
            prod = lst[o:o + 2 * nprod]
            sums = lst[o + 2 * nprod:o + 2 * nprod + nsum]
            push = lst[o + 2 * nprod + nsum:o + 2 * nprod + nsum + npush]
            W = sigma[w[1]].copy() if w[0] & TF_ACC else np.zeros_like(tiles[0])
            for q in sums:
                W += qpart.pop(q)
            for q in range(nprod):
                W += sig(prod[2 * q]) @ tiles[prod[2 * q + 1]]
            Sg = -W @ linv[w[2]]
            sigma[w[1]] = Sg
            dpart[w[1]] = tiles[w[1]].T @ Sg
            for u in push:
                assert u not in qpart
                qpart[u] = Sg.T @ tiles[u]
        elif typ == TSUM:
            src = qpart if w[4] == 1 else dpart
            acc = np.zeros_like(tiles[0])
            for q in lst[w[2]:w[2] + w[3]]:
                acc += src.pop(q)
            assert w[1] not in src
            src[w[1]] = acc
        elif typ == SDIAG:
            o = w[3]
            Z = linv[w[2]].copy()
            for q in lst[o:o + w[4]]:
                Z -= dpart.pop(q)
            R = linv[w[2]].T @ Z
            sigma[w[1]] = np.tril(R) + np.tril(R, -1).T
        else:
            raise AssertionError("unknown selected-inversion task type %d" % typ)
    assert not qpart and not dpart, "partials produced but never consumed"
    return sigma


def factor_solve(plan, Aperm, B, mode="ticket", seed=0):
    """The merged factorization + solve DAG (one ticket order for both task
    kinds); returns (tiles, linv, X) like factor() and solve()."""
    rng = np.random.default_rng(seed)
    ex = lambda k: S.stiles_symbolic_export(plan._sym.handle, k)
    tasks, succ, P = ex("mtask").reshape(-1, 8), ex("msucc"), ex("mpairs").reshape(-1, 2)
    T, ntr = plan.T, plan.ntr
    tiles = scatter(plan, Aperm)
    linv = np.zeros((ntr, T, T))
    part = np.zeros((max(plan.npart, 1), T, T))
    done_tile = np.zeros(len(plan.tcol), dtype=bool)   # final value written
    nrhs = B.shape[1]
    Y = np.zeros((ntr, T, nrhs))
    Bp = B[plan.perm]
    for m in range(ntr):
        rb, rc = plan.row_base[m], plan.row_cnt[m]
        Y[m, :rc] = Bp[rb:rb + rc]
    Z = np.zeros_like(Y)
    Q = {}

    def tile(t):
        assert done_tile[t], "solve task read a factor tile before it was final"
        return tiles[t]

    for t in _order(tasks, succ, mode, rng):
        w = tasks[t]
        typ = w[0] & 0xff
        m = w[1]
        if typ in (UPD, PART):
            acc = sum(tiles[P[p, 0]] @ tiles[P[p, 1]].T for p in range(w[2], w[3]))
            if typ == UPD:
                tiles[w[1]] -= np.tril(acc) if w[0] & TF_DIAG else acc
            elif w[0] & TF_ACC:
                part[w[4]] += acc
            else:
                part[w[4]] = acc
        elif typ == UPDB:
            update_block(w, P, tiles, done_tile)
        elif typ == TREE:
            s_ = part[w[2]] + (part[w[3]] if w[3] >= 0 else 0.0)
            if w[4] >= 0:
                part[w[4]] = s_
            else:
                tiles[w[1]] -= s_
        elif typ == POTRF:
            C = tiles[w[1]].copy()
            for p in range(w[3], w[4]):
                C -= tiles[P[p, 0]] @ tiles[P[p, 1]].T
            L = np.linalg.cholesky(np.tril(C) + np.tril(C, -1).T)
            tiles[w[1]] = L
            linv[w[2]] = np.linalg.inv(L)
            done_tile[w[1]] = True
        elif typ == TRSM:
            C = tiles[w[1]].copy()
            for p in range(w[3], w[4]):
                C -= tiles[P[p, 0]] @ tiles[P[p, 1]].T
            tiles[w[1]] = C @ linv[w[2]].T
            done_tile[w[1]] = True
        elif typ == FUPD:
            for p in range(w[2], w[3]):
                Y[m] -= tile(P[p, 0]) @ Y[P[p, 1]]
        elif typ == FPART:
            q = np.zeros_like(Y[m])
            for p in range(w[2], w[3]):
                q += tile(P[p, 0]) @ Y[P[p, 1]]
            Q[w[4]] = q
        elif typ == FSUM:
            for s_ in range(w[2], w[3]):
                Y[m] -= Q.pop(s_)
        elif typ == FDIAG:
            v = Y[m].copy()
            for p in range(w[2], w[3]):
                v -= tile(P[p, 0]) @ Y[P[p, 1]]
            Y[m] = linv[m] @ v
        elif typ == BUPD:
            v = (Y[m] if w[0] & TF_FIRST else Z[m]).copy()
            for p in range(w[2], w[3]):
                v -= tile(P[p, 0]).T @ Z[P[p, 1]]
            Z[m] = v
        elif typ == BDIAG:
            v = (Y[m] if w[0] & TF_FIRST else Z[m]).copy()
            for p in range(w[2], w[3]):
                v -= tile(P[p, 0]).T @ Z[P[p, 1]]
            Z[m] = linv[m].T @ v
        else:
            raise AssertionError("unknown task type %d" % typ)
    X = np.zeros_like(B)
    Xp = np.zeros_like(B)
    for m in range(ntr):
        rb, rc = plan.row_base[m], plan.row_cnt[m]
        Xp[rb:rb + rc] = Z[m, :rc]
    X[plan.perm] = Xp
    return tiles, linv, X
