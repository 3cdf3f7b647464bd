"""The executor's counter protocol under ThreadSanitizer (host, no GPU).

tests/race/exec_race.cpp runs an exported factorization DAG on worker
threads with the device executor's protocol: tickets in the static order,
per-task counters, two-stage waits for TF_SPLIT tasks (the early
predecessors first, then the late one), notifications that subtract the
edge's weight; acquire/release atomics order the tile accesses.  Under
ThreadSanitizer a task that reads a tile before the task that writes it is
ordered before it (a missing edge in the plan, or a read placed before the
wait that covers it) is reported as a data race.  Each plan runs with 8
threads and random delays under three seeds; the factor must match the
oracle's (1e-12).  A planted missing edge (POTRF -> TRSM) must be caught.
The merged factorization + solve DAG (the launch the bench times) runs the
same way with its three counter weights (factorization predecessors of a
solve task, early solve predecessors of a two-stage diagonal step, the rest):
no race, and both the factor and the solution match the oracle."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import paper_2501_02483_amd as S
from paper_2501_02483_amd import inputs as I

import dag_emulator as E
from permute_util import permute_profile

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "race", "exec_race.cpp")
TSAN_OPTIONS = "halt_on_error=1 exitcode=66 history_size=4"


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("race") / "exec_race")
    r = subprocess.run(["g++", "-O1", "-g", "-fsanitize=thread", "-std=c++17", "-pthread", SRC, "-o", out],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("cannot build with -fsanitize=thread: " + r.stderr[-300:])
    return out


def _export(plan, Aperm, path, drop=None):
    ex = lambda k: S.stiles_symbolic_export(plan._sym.handle, k)
    tasks, succ, pairs = ex("ftask"), ex("fsucc"), ex("fpairs")
    tiles = E.scatter(plan, Aperm)
    T = plan.T
    hdr = np.array([T, len(plan.tcol), plan.ntr, len(tasks) // 8, len(succ), len(pairs), plan.npart],
                   dtype=np.int32)
    with open(path, "wb") as f:
        f.write(hdr.tobytes())
        f.write(np.ascontiguousarray(tasks, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(succ, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(pairs, dtype=np.int32).tobytes())
        # column-major T x T tiles
        f.write(np.ascontiguousarray(tiles.transpose(0, 2, 1)).tobytes())
    return tasks.reshape(-1, 8), succ


def _run(exe, inp, out, seed, drop=None):
    cmd = [exe, inp, out, "8", str(seed)] + ([str(drop)] if drop is not None else [])
    env = dict(os.environ, TSAN_OPTIONS=TSAN_OPTIONS)
    env.pop("LD_PRELOAD", None)   # a preloaded ASan runtime (host sanitizer run) cannot share with TSan
    return subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=600)


def _oracle_factor_permuted(p, vals, perm):
    f2, v2 = permute_profile(p.f, vals, perm)
    L, info = oracle.factor(f2, v2)
    assert info == 0
    N = len(f2)
    D = np.zeros((N, N))
    rp = np.concatenate([[0], np.cumsum(np.arange(N) - f2 + 1)])
    for i in range(N):
        D[i, f2[i]:i + 1] = L[rp[i]:rp[i + 1]]
    return D


CASES = [
    # n, arrow, widths, segment, tile, ordering, parts, ublock
    (900, 40, [15, 70, 30], 300, 32, S.STILES_ORDER_NONE, 0, 0),
    (1500, 24, [20, 60, 35], 300, 32, S.STILES_ORDER_ADAPTABLE_ND, 3, 0),
    (1200, 30, [30, 90], 400, 32, S.STILES_ORDER_NONE, 0, 3),
]


@pytest.mark.parametrize("case", CASES, ids=["natural_tree", "nd3", "blocks"])
def test_protocol_has_no_races(exe, tmp_path, case):
    n, a, w, seg, T, ordering, parts, ub = case
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + a)
    sym = S.Symbolic.from_pattern(p, tile=T, ordering=ordering, nd_parts=parts, ublock=ub)
    plan = E.Plan(sym)
    Aperm = I.to_dense(p, vals)[np.ix_(plan.perm, plan.perm)]
    tasks, _ = _export(plan, Aperm, str(tmp_path / "plan.bin"))
    assert (tasks[:, 0] & E.TF_SPLIT).any()          # two-stage waits are exercised
    Lo = _oracle_factor_permuted(p, vals, plan.perm)
    for seed in (1, 2, 3):
        r = _run(exe, str(tmp_path / "plan.bin"), str(tmp_path / "out.bin"), seed)
        assert r.returncode == 0, r.stderr[-3000:]
        assert "ThreadSanitizer" not in r.stderr
        t = np.fromfile(str(tmp_path / "out.bin"), dtype=np.float64).reshape(-1, T, T).transpose(0, 2, 1)
        Ld = E.dense_factor(plan, t)
        assert np.linalg.norm(Ld - Lo) / np.linalg.norm(Lo) <= 1e-12


def test_planted_missing_edge_is_reported(exe, tmp_path):
    """A POTRF -> TRSM edge removed from the plan (the TRSM no longer waits
    for the inverse diagonal tile it reads): ThreadSanitizer reports the
    race (or the factor is wrong) in every seeded run."""
    p = I.make_pattern(600, 10, 40)
    vals = I.make_values(p, seed=5)
    sym = S.Symbolic.from_pattern(p, tile=32)
    plan = E.Plan(sym)
    Aperm = I.to_dense(p, vals)
    tasks, succ = _export(plan, Aperm, str(tmp_path / "plan.bin"))
    typ = tasks[:, 0] & 0xff
    drop = None
    for t in np.nonzero(typ == E.POTRF)[0][2:]:
        for q in range(tasks[t, 5], tasks[t, 6]):
            x = int(succ[q]) & ~E.SUCC_FDEP
            if typ[x] == E.TRSM:
                drop = q
                break
        if drop is not None:
            break
    assert drop is not None
    Lo = _oracle_factor_permuted(p, vals, plan.perm)
    # the POTRF that lost the edge starts late, so the TRSM reads first
    caught = 0
    for seed in (1, 2):
        r = _run(exe, str(tmp_path / "plan.bin"), str(tmp_path / "out.bin"), seed, drop=drop)
        if r.returncode == 66 or "ThreadSanitizer: data race" in r.stderr:
            caught += 1
            continue
        t = np.fromfile(str(tmp_path / "out.bin"), dtype=np.float64).reshape(-1, 32, 32).transpose(0, 2, 1)
        if np.linalg.norm(E.dense_factor(plan, t) - Lo) / np.linalg.norm(Lo) > 1e-12:
            caught += 1
    assert caught == 2


def _export_merged(plan, Aperm, B, path):
    ex = lambda k: S.stiles_symbolic_export(plan._sym.handle, k)
    tasks, succ, pairs = ex("mtask"), ex("msucc"), ex("mpairs")
    tiles = E.scatter(plan, Aperm)
    T, ntr, nrhs = plan.T, plan.ntr, B.shape[1]
    Bp = B[plan.perm]
    Yb = np.zeros((ntr, nrhs, T))
    for m in range(ntr):
        rb, rc = plan.row_base[m], plan.row_cnt[m]
        Yb[m, :, :rc] = Bp[rb:rb + rc].T
    hdr = np.array([T, len(plan.tcol), ntr, len(tasks) // 8, len(succ), len(pairs), plan.npart], dtype=np.int32)
    with open(path, "wb") as f:
        f.write(hdr.tobytes())
        for a in (tasks, succ, pairs):
            f.write(np.ascontiguousarray(a, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(tiles.transpose(0, 2, 1)).tobytes())
        f.write(np.array([nrhs], dtype=np.int32).tobytes())
        f.write(Yb.tobytes())
    return tasks.reshape(-1, 8)


MERGED_CASES = [
    # n, arrow, widths, segment, tile, ordering, parts
    (900, 40, [15, 70, 30], 300, 32, S.STILES_ORDER_NONE, 0),
    (1500, 24, [20, 60, 35], 300, 32, S.STILES_ORDER_ADAPTABLE_ND, 3),
]


@pytest.mark.parametrize("case", MERGED_CASES, ids=["natural", "nd3"])
def test_merged_protocol_has_no_races(exe, tmp_path, case):
    n, a, w, seg, T, ordering, parts = case
    p = I.make_pattern(n, a, w, seg=seg)
    vals = I.make_values(p, seed=n + a + 1)
    sym = S.Symbolic.from_pattern(p, tile=T, ordering=ordering, nd_parts=parts)
    plan = E.Plan(sym)
    Aperm = I.to_dense(p, vals)[np.ix_(plan.perm, plan.perm)]
    B = I.rhs(p.N, 3, seed=n)
    tasks = _export_merged(plan, Aperm, B, str(tmp_path / "plan.bin"))
    typ = tasks[:, 0] & 0xff
    assert ((tasks[:, 0] & E.TF_SPLIT) != 0)[(typ == E.FDIAG) | (typ == E.BDIAG)].any()
    Lo = _oracle_factor_permuted(p, vals, plan.perm)
    L, info = oracle.factor(p.f, vals)
    Xo = oracle.solve(p.f, L, B)
    ntiles, ntr = len(plan.tcol), plan.ntr
    for seed in (1, 2, 3):
        r = _run(exe, str(tmp_path / "plan.bin"), str(tmp_path / "out.bin"), seed)
        assert r.returncode == 0, r.stderr[-3000:]
        assert "ThreadSanitizer" not in r.stderr
        out = np.fromfile(str(tmp_path / "out.bin"), dtype=np.float64)
        t = out[:ntiles * T * T].reshape(-1, T, T).transpose(0, 2, 1)
        assert np.linalg.norm(E.dense_factor(plan, t) - Lo) / np.linalg.norm(Lo) <= 1e-12
        Z = out[ntiles * T * T:].reshape(ntr, B.shape[1], T)
        Xp = np.zeros_like(B)
        for m in range(ntr):
            rb, rc = plan.row_base[m], plan.row_cnt[m]
            Xp[rb:rb + rc] = Z[m, :, :rc].T
        X = np.zeros_like(B)
        X[plan.perm] = Xp
        assert np.linalg.norm(X - Xo) / np.linalg.norm(Xo) <= 1e-12


def test_merged_planted_missing_edge_is_reported(exe, tmp_path):
    """An early solve edge into a two-stage backward diagonal step (weight
    2^8) removed from the merged DAG: the step's first stage may read a
    block before it is written, which ThreadSanitizer reports in every
    seeded run."""
    p = I.make_pattern(900, 40, [15, 70, 30], seg=300)
    vals = I.make_values(p, seed=941)
    sym = S.Symbolic.from_pattern(p, tile=32)
    plan = E.Plan(sym)
    Aperm = I.to_dense(p, vals)[np.ix_(plan.perm, plan.perm)]
    B = I.rhs(p.N, 3, seed=900)
    tasks = _export_merged(plan, Aperm, B, str(tmp_path / "plan.bin"))
    succ = S.stiles_symbolic_export(sym.handle, "msucc")
    typ = tasks[:, 0] & 0xff
    drop = None
    for t in np.nonzero(typ == E.BDIAG)[0][3:]:
        for q in range(tasks[t, 5], tasks[t, 6]):
            v = int(succ[q])
            if v & E.SUCC_MID and typ[v & ~E.SUCC_MID] == E.BDIAG:
                drop = q
                break
        if drop is not None:
            break
    assert drop is not None
    caught = 0
    for seed in (1, 2):
        r = _run(exe, str(tmp_path / "plan.bin"), str(tmp_path / "out.bin"), seed, drop=drop)
        caught += r.returncode == 66 or "ThreadSanitizer: data race" in r.stderr
    assert caught == 2
