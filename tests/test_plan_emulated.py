"""CPU checks of the host planner through the C ABI (no GPU): the factor and
solve DAGs, executed by the host emulator in ticket order and in random
topological orders, reproduce the oracle's factor and solution."""
import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

import dag_emulator as E

SHAPES = [
    # n, a, widths, seg, tile, tree ratio
    (300, 5, 7, None, 32, 2),
    (700, 40, 60, None, 64, 2),
    (700, 40, 60, None, 64, 0),
    (1000, 0, 30, None, 32, 2),
    (400, 70, 0, None, 32, 2),
    (2000, 100, [10, 130, 40, 90], 500, 32, 2),
]


def _oracle_dense_L(p, vals):
    L, info = oracle.factor(p.f, vals)
    assert info == 0
    D = np.zeros((p.N, p.N))
    rp = p.row_ptr()
    for i in range(p.N):
        D[i, p.f[i]:i + 1] = L[rp[i]:rp[i + 1]]
    return D, L


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%d_a%d_T%d_r%d" % (s[0], s[1], s[4], s[5]))
@pytest.mark.parametrize("mode", ["ticket", "random"])
def test_emulated_factor_and_solve_match_oracle(shape, mode):
    n, a, w, seg, T, ratio = shape
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + a)
    sym = S.Symbolic.from_pattern(p, tile=T, tree_min_ratio=ratio)
    plan = E.Plan(sym)
    A = I.to_dense(p, vals)
    tiles, linv = E.factor(plan, A, mode=mode, seed=n)
    Ld = E.dense_factor(plan, tiles)
    Lo, Lv = _oracle_dense_L(p, vals)
    assert np.linalg.norm(Ld - Lo) / np.linalg.norm(Lo) <= 1e-12
    B = I.rhs(p.N, 3, seed=9)
    X = E.solve(plan, tiles, linv, B, mode=mode, seed=n + 1)
    Xo = oracle.solve(p.f, Lv, B)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-12


def test_tree_shape_and_corner_count():
    """With the tree, every arrow-corner tile sums one partial per chunk of
    band columns through a binary GEADD tree; without it, one chain."""
    p = I.make_pattern(3000, 50, 40)
    on = S.Symbolic.from_pattern(p, tile=32, tree_min_ratio=2)
    off = S.Symbolic.from_pattern(p, tile=32, tree_min_ratio=0)
    assert on.info.tree_used == 1 and off.info.tree_used == 0
    # about one corner accumulation per band tile row
    assert on.info.corner_accumulations == on.info.band_tile_rows
    ft = S.stiles_symbolic_export(on.handle, "ftask").reshape(-1, 8)
    types = ft[:, 0] & 0xff
    nparts = int((types == E.PART).sum())
    ntree = int((types == E.TREE).sum())
    ncorner = 3          # lower tiles of the 2 x 2 arrow-corner tile block (a = 50, T = 32)
    # a binary tree over G partials takes G - 1 additions (the last one subtracts
    # into the corner tile) and G - 2 intermediate slots
    assert ntree == nparts - ncorner
    npart_slots = int(S.stiles_symbolic_export(on.handle, "npart")[0])
    assert npart_slots == nparts + (nparts - 2 * ncorner)
    ft_off = S.stiles_symbolic_export(off.handle, "ftask").reshape(-1, 8)
    assert int(((ft_off[:, 0] & 0xff) == E.PART).sum()) == 0


def test_csc_input_with_rcm_permutation():
    """A randomly relabelled band: partial RCM is kept by the fill check and
    the emulated factor is the Cholesky factor of P A P^T."""
    rng = np.random.default_rng(3)
    p = I.make_pattern(600, 8, 12)
    vals = I.make_values(p, seed=5)
    A = I.to_dense(p, vals)
    shuf = np.concatenate([rng.permutation(p.n), np.arange(p.n, p.N)])
    As = A[np.ix_(shuf, shuf)]
    Ls = np.tril(As)
    colptr = np.zeros(p.N + 1, dtype=np.int64)
    rows = []
    for j in range(p.N):
        r = np.nonzero(Ls[:, j])[0]
        r = r[r >= j]
        if r[0] != j:
            r = np.concatenate([[j], r])
        rows.append(r)
        colptr[j + 1] = colptr[j] + len(r)
    rowind = np.concatenate(rows)
    auto = S.Symbolic.from_csc(p.N, p.a, colptr, rowind, tile=32)
    none = S.Symbolic.from_csc(p.N, p.a, colptr, rowind, tile=32, ordering=S.STILES_ORDER_NONE)
    assert auto.info.ordering_used == S.STILES_ORDER_PARTIAL_RCM
    assert auto.info.tiles < none.info.tiles
    perm = auto.perm()
    assert np.array_equal(np.sort(perm), np.arange(p.N))
    assert np.array_equal(perm[p.n:], np.arange(p.n, p.N))   # the arrow stays last
    plan = E.Plan(auto)
    Ap = As[np.ix_(perm, perm)]
    tiles, linv = E.factor(plan, Ap, mode="random", seed=1)
    Ld = E.dense_factor(plan, tiles)
    Lref = np.linalg.cholesky(Ap)
    assert np.linalg.norm(Ld - Lref) / np.linalg.norm(Lref) <= 1e-12
    B = I.rhs(p.N, 2, seed=4)
    X = E.solve(plan, tiles, linv, B)
    assert np.linalg.norm(X - np.linalg.solve(As, B)) / np.linalg.norm(X) <= 1e-12


@pytest.mark.parametrize("mode", ["ticket", "random"])
@pytest.mark.parametrize("n,a,w,seg,T,parts", [
    (2400, 30, [10, 60, 25], 400, 32, 3),
    (3000, 20, 24, None, 32, 0),
    (1500, 70, [20, 50], 300, 64, 2),
])
def test_emulated_nd_plan(n, a, w, seg, T, parts, mode):
    """Adaptable ND plans (partitions, separators in bisection order, long
    forward rows summed from partial products) reproduce the oracle."""
    from permute_util import permute_profile
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + T)
    sym = S.Symbolic.from_pattern(p, tile=T, ordering=S.STILES_ORDER_ADAPTABLE_ND, nd_parts=parts)
    assert sym.info.nd_parts >= 2
    plan = E.Plan(sym)
    perm = plan.perm
    A = I.to_dense(p, vals)
    tiles, linv = E.factor(plan, A[np.ix_(perm, perm)], mode=mode, seed=n)
    Ld = E.dense_factor(plan, tiles)
    f2, v2 = permute_profile(p.f, vals, perm)
    L2, info = oracle.factor(f2, v2)
    assert info == 0
    D2 = np.zeros((p.N, p.N))
    rp2 = np.concatenate([[0], np.cumsum(np.arange(p.N) - f2 + 1)])
    for i in range(p.N):
        D2[i, f2[i]:i + 1] = L2[rp2[i]:rp2[i + 1]]
    assert np.linalg.norm(Ld - D2) / np.linalg.norm(D2) <= 1e-12
    B = I.rhs(p.N, 2, seed=4)
    X = E.solve(plan, tiles, linv, B, mode=mode, seed=n + 1)
    Lo, Lv = _oracle_dense_L(p, vals)
    Xo = oracle.solve(p.f, Lv, B)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-12


def test_long_forward_rows_use_partials():
    """An arrow row spanning many band tiles is summed from parallel partial
    products (FPART tasks and one FSUM) instead of one sequential chain."""
    p = I.make_pattern(3000, 20, 24)
    sym = S.Symbolic.from_pattern(p, tile=32)
    plan = E.Plan(sym)
    types = plan.stask[:, 0] & 0xff
    assert (types == E.FPART).sum() >= 2 and (types == E.FSUM).sum() >= 1


@pytest.mark.parametrize("shape", SHAPES[:4] + SHAPES[5:], ids=lambda s: "n%d_a%d_T%d" % (s[0], s[1], s[4]))
@pytest.mark.parametrize("mode", ["ticket", "random"])
def test_emulated_merged_factor_solve(shape, mode):
    """The merged factorization + solve DAG: every solve task runs only after
    the factor tiles it reads are final, and the result is the oracle's."""
    n, a, w, seg, T, ratio = shape
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + a)
    sym = S.Symbolic.from_pattern(p, tile=T, tree_min_ratio=ratio)
    plan = E.Plan(sym)
    B = I.rhs(p.N, 3, seed=9)
    tiles, linv, X = E.factor_solve(plan, I.to_dense(p, vals), B, mode=mode, seed=n + 3)
    Lo, Lv = _oracle_dense_L(p, vals)
    assert np.linalg.norm(E.dense_factor(plan, tiles) - Lo) / np.linalg.norm(Lo) <= 1e-12
    Xo = oracle.solve(p.f, Lv, B)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-12


@pytest.mark.parametrize("parts", [2, 0])
def test_emulated_merged_factor_solve_nd(parts):
    p = I.make_pattern(3000, 24, [20, 90, 45], seg=600)
    vals = I.make_values(p, seed=31)
    sym = S.Symbolic.from_pattern(p, tile=32, ordering=S.STILES_ORDER_ADAPTABLE_ND, nd_parts=parts)
    plan = E.Plan(sym)
    A = I.to_dense(p, vals)
    B = I.rhs(p.N, 2, seed=4)
    _, _, X = E.factor_solve(plan, A[np.ix_(plan.perm, plan.perm)], B, mode="random", seed=parts)
    L, info = oracle.factor(p.f, vals)
    Xo = oracle.solve(p.f, L, B)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-12


@pytest.mark.parametrize("parts", [None, 3])
def test_merged_counters_split_factor_and_solve_predecessors(parts):
    """Merged DAG counters: a solve task counts each factorization predecessor
    as MERGED_FDEP and each solve predecessor as 1 -- a two-stage diagonal
    step each early solve predecessor as SPLIT_W and its one late
    predecessor as 1 --, the MERGED_FDEP entries are exactly the
    factorization -> solve edges, and the factorization predecessors of a
    solve task include the final task of every factor tile it reads and, for
    a diagonal step, the POTRF of its row -- so its tiles may be staged once
    the counter is below MERGED_FDEP."""
    p = I.make_pattern(2500, 18, [16, 70, 30], seg=500)
    kw = dict(ordering=S.STILES_ORDER_ADAPTABLE_ND, nd_parts=parts) if parts else {}
    sym = S.Symbolic.from_pattern(p, tile=32, **kw)
    ex = lambda k: S.stiles_symbolic_export(sym.handle, k)
    tasks, succ, P = ex("mtask").reshape(-1, 8), ex("msucc"), ex("mpairs").reshape(-1, 2)
    typ = tasks[:, 0] & 0xff
    is_fac = typ < E.FUPD
    n = len(tasks)
    fpred = [set() for _ in range(n)]
    fweight = [0] * n      # factorization tasks: counter weight of their predecessors
    spred = [0] * n
    split_steps = 0
    final_of, potrf_of = {}, {}
    for t in range(n):
        if typ[t] in (E.POTRF, E.TRSM):
            final_of[int(tasks[t, 1])] = t
        if typ[t] == E.POTRF:
            potrf_of[int(tasks[t, 2])] = t
        for q in range(tasks[t, 5], tasks[t, 6]):
            x, dec = E.succ_edge(succ[q])
            assert x > t
            if not is_fac[t] or not is_fac[x]:
                # factorization -> solve edges weigh MERGED_FDEP, solve -> solve 1,
                # or SPLIT_W from an early predecessor of a two-stage diagonal step
                assert (dec == E.MERGED_FDEP) == (is_fac[t] and not is_fac[x])
                if dec == E.SPLIT_W:
                    assert not is_fac[t] and tasks[x, 0] & E.TF_SPLIT and typ[x] in (E.FDIAG, E.BDIAG)
            else:
                # factorization -> factorization: MERGED_FDEP only into a
                # two-stage POTRF/TRSM, from one of its early predecessors
                assert dec == 1 or tasks[x, 0] & E.TF_SPLIT
                fweight[x] += dec
            if is_fac[t]:
                fpred[x].add(t)
            else:
                spred[x] += dec
    for t in range(n):
        if is_fac[t]:
            assert tasks[t, 7] == fweight[t] and spred[t] == 0
            if tasks[t, 0] & E.TF_SPLIT:
                # exactly one late predecessor (weight 1)
                assert fweight[t] % E.MERGED_FDEP == 1
            continue
        assert tasks[t, 7] == spred[t] + E.MERGED_FDEP * len(fpred[t])
        if tasks[t, 0] & E.TF_SPLIT:
            # exactly one late solve predecessor (weight 1), the others SPLIT_W
            assert typ[t] in (E.FDIAG, E.BDIAG) and spred[t] % E.SPLIT_W == 1
            split_steps += 1
        if typ[t] == E.FSUM:
            continue
        for q in range(tasks[t, 2], tasks[t, 3]):
            assert final_of[int(P[q, 0])] in fpred[t]
        if typ[t] in (E.FDIAG, E.BDIAG):
            assert potrf_of[int(tasks[t, 1])] in fpred[t]
    assert split_steps > 0          # the two-stage diagonal steps are exercised


@pytest.mark.parametrize("sched_workers", [-1, 0, 16])
def test_ticket_orders_emulate_to_the_oracle(sched_workers):
    """Every ticket order (earliest start, list schedules on 512 or 16
    workgroups) is topological and gives the oracle's factor and solution."""
    p = I.make_pattern(2500, 18, [16, 70, 30], seg=500)
    vals = I.make_values(p, seed=8)
    sym = S.Symbolic.from_pattern(p, tile=32, ordering=S.STILES_ORDER_ADAPTABLE_ND, nd_parts=3,
                                  sched_workers=sched_workers)
    plan = E.Plan(sym)
    A = I.to_dense(p, vals)
    B = I.rhs(p.N, 2, seed=3)
    _, _, X = E.factor_solve(plan, A[np.ix_(plan.perm, plan.perm)], B, mode="ticket")
    L, info = oracle.factor(p.f, vals)
    Xo = oracle.solve(p.f, L, B)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-12


@pytest.mark.parametrize("ordering,parts", [(S.STILES_ORDER_ADAPTABLE_ND, 3), (S.STILES_ORDER_ADAPTABLE_ND, 0),
                                            (S.STILES_ORDER_NONE, 0)])
def test_tiles_with_entries_match_the_permuted_matrix(ordering, parts):
    """Export 17 (tiles that receive entries of A; the residual of the mixed
    mode skips the others) against the tiles of the permuted dense matrix:
    exactly the tiles with a nonzero entry, plus the diagonal tiles."""
    p = I.make_pattern(3000, 24, [20, 90, 45], seg=600)
    vals = I.make_values(p, seed=31)
    sym = S.Symbolic.from_pattern(p, tile=32, ordering=ordering, nd_parts=parts)
    plan = E.Plan(sym)
    A = I.to_dense(p, vals)
    tiles = E.scatter(plan, A[np.ix_(plan.perm, plan.perm)])
    ref = np.array([np.any(tiles[t] != 0) or plan.trow[t] == plan.tcol[t] for t in range(len(plan.tcol))])
    has = S.stiles_symbolic_export(sym.handle, "tile_has_a").astype(bool)
    assert np.array_equal(has, ref)
    if ordering == S.STILES_ORDER_ADAPTABLE_ND:
        assert (~has).sum() > 0   # nested dissection leaves tiles of fill only


def test_tiles_with_entries_csc_input():
    from permute_util import profile_entries
    p = I.make_pattern(2500, 16, [12, 60], seg=500)
    vals = I.make_values(p, seed=12)
    rng = np.random.default_rng(5)
    q = np.arange(p.N)
    q[:p.n] = rng.permutation(p.n)
    r, c, v = profile_entries(p.f, vals)
    rr, cc = q[r], q[c]
    hi, lo = np.maximum(rr, cc), np.minimum(rr, cc)
    order = np.lexsort((hi, lo))
    colptr = np.zeros(p.N + 1, dtype=np.int64)
    np.cumsum(np.bincount(lo, minlength=p.N), out=colptr[1:])
    sym = S.Symbolic.from_csc(p.N, p.a, colptr, hi[order].astype(np.int64), tile=32,
                              ordering=S.STILES_ORDER_ADAPTABLE_ND, nd_parts=3)
    plan = E.Plan(sym)
    A = np.zeros((p.N, p.N))
    A[hi, lo] = v
    A[lo, hi] = v
    tiles = E.scatter(plan, A[np.ix_(plan.perm, plan.perm)])
    ref = np.array([np.any(tiles[t] != 0) or plan.trow[t] == plan.tcol[t] for t in range(len(plan.tcol))])
    has = S.stiles_symbolic_export(sym.handle, "tile_has_a").astype(bool)
    assert np.array_equal(has, ref)


@pytest.mark.parametrize("ublock", [1, 3, 6])
@pytest.mark.parametrize("mode", ["ticket", "random"])
@pytest.mark.parametrize("ordering,parts", [(S.STILES_ORDER_NONE, 0), (S.STILES_ORDER_ADAPTABLE_ND, 3)],
                         ids=["natural", "nd3"])
def test_emulated_block_updates(ublock, mode, ordering, parts):
    """2 x 2 block update tasks (two tile rows of two adjacent band columns
    sharing their operand tiles, absent operands skipped per target) in the
    factorization and the merged DAG: the emulated factor and solution match
    the oracle."""
    p = I.make_pattern(2500, 40, [20, 150, 70, 110], seg=600)
    vals = I.make_values(p, seed=31)
    sym = S.Symbolic.from_pattern(p, tile=32, ordering=ordering, nd_parts=parts, ublock=ublock)
    assert sym.info.update_blocks > 0
    plan = E.Plan(sym)
    A = I.to_dense(p, vals)[np.ix_(plan.perm, plan.perm)]
    L, info = oracle.factor(p.f, vals)
    assert info == 0
    if ordering == S.STILES_ORDER_NONE:
        tiles, linv = E.factor(plan, A, mode=mode, seed=ublock)
        Lo, _ = _oracle_dense_L(p, vals)
        assert np.linalg.norm(E.dense_factor(plan, tiles) - Lo) / np.linalg.norm(Lo) <= 1e-12
    B = I.rhs(p.N, 2, seed=5)
    _, _, X = E.factor_solve(plan, A, B, mode=mode, seed=ublock + 1)
    Xo = oracle.solve(p.f, L, B)
    assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-12


@pytest.mark.parametrize("parts", [0, 3])
def test_two_stage_solve_steps_read_only_final_blocks(parts):
    """Two-stage diagonal solve steps (TF_SPLIT) run as two sub-tasks in
    random orders: the first stage (right-hand side block and first fused
    product) after the early predecessors only, the second after the late
    one.  Every order reproduces the oracle's solution, with backward blocks
    not yet written reading as NaN; and declaring another predecessor late
    (the step's update chain, so that its first stage may read an
    unfinished block) is caught when the first stages run as early as
    their predecessors allow."""
    p = I.make_pattern(2500, 18, [16, 70, 30], seg=500)
    vals = I.make_values(p, seed=21)
    kw = dict(ordering=S.STILES_ORDER_ADAPTABLE_ND, nd_parts=parts) if parts else {}
    sym = S.Symbolic.from_pattern(p, tile=32, **kw)
    plan = E.Plan(sym)
    A = I.to_dense(p, vals)
    tiles, linv = E.factor(plan, A[np.ix_(plan.perm, plan.perm)])
    B = I.rhs(p.N, 2, seed=6)
    L, info = oracle.factor(p.f, vals)
    Xo = oracle.solve(p.f, L, B)
    typ = plan.stask[:, 0] & 0xff
    split = np.nonzero(plan.stask[:, 0] & E.TF_SPLIT)[0]
    assert set(typ[split]) == {E.FDIAG, E.BDIAG}
    for mode, seed in [("split", 0), ("split", 1), ("split", 2), ("split_eager", 3)]:
        X = E.solve(plan, tiles, linv, B, mode=mode, seed=seed)
        assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-12
    # planted: the late predecessor of every split backward step that has an
    # update chain becomes that chain's last task
    preds = {}
    for t in range(len(plan.stask)):
        for q in range(plan.stask[t, 5], plan.stask[t, 6]):
            preds.setdefault(E.succ_edge(plan.ssucc[q])[0], []).append(t)
    late_of = {}
    for t in split:
        if typ[t] == E.BDIAG and not plan.stask[t, 0] & E.TF_FIRST:
            late_of[int(t)] = max(x for x in preds[t] if typ[x] == E.BUPD)
    assert late_of
    X = E.solve(plan, tiles, linv, B, mode="split_eager", seed=0, late_of=late_of)
    assert not np.all(np.isfinite(X)) or np.linalg.norm(X - Xo) / np.linalg.norm(Xo) > 1e-6
