"""Serving on the GPU (continuous batching over resident patterns).

Requests that arrive together overlap on the device (several persistent
launches on different streams, sharing the workgroups).  Each result must be
the same in the mix as when the request runs alone: the per-tile
accumulation order is fixed by the task DAG, so the comparison is bit for
bit.  The values the device generator drew are read back and checked against
the oracle, so the served results are also correct, not only reproducible."""
import numpy as np
import pytest

from paper_2501_02483_amd import inputs as I

from gpu_util import oracle_reference, rel, say

pytestmark = pytest.mark.gpu


def _patterns():
    return [I.make_pattern(3000, 16, 64, name="s0"), I.make_pattern(9000, 40, 150, name="s1"),
            I.make_pattern(20000, 8, 100, name="s2")]


def test_serve_mix_equals_alone_and_oracle():
    import torch

    from paper_2501_02483_amd.serve import OP_LOGDET, OP_SOLVE, GpuExecutor, Request, Server

    pats = _patterns()
    budget = 8 << 30
    ex = GpuExecutor(pats, tile=64, slots=4)
    reqs = [Request(rid=i, arrival=0.0, pattern=i % 3, op=(i // 3) % 3, seed=700 + i) for i in range(18)]
    say("[gpu serve] mix of %d requests on 4 slots, shortest first" % len(reqs))
    srv = Server(ex, budget, 4, policy="sjf")
    done = srv.run(reqs)
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    # all arrived at once: the four slots start with the cheapest pattern's requests
    assert [reqs[rid].pattern for rid in srv.admit_order[:4]] == [0, 0, 0, 0]
    assert all(r.result["info"] == 0 for r in done)
    # the mix really overlapped: some request was admitted before another finished
    overlap = sum(1 for r in done for q in done if q.rid != r.rid and q.t_admit < r.t_done and r.t_admit < q.t_done)
    assert overlap > 0

    ex1 = GpuExecutor(pats, tile=64, slots=1)
    for r in sorted(done, key=lambda r: r.rid):
        alone = Server(ex1, budget, 1).run([Request(rid=r.rid, arrival=0.0, pattern=r.pattern, op=r.op,
                                                    seed=r.seed)])[0]
        assert alone.result["info"] == 0
        assert torch.equal(alone.result["values"], r.result["values"])
        if r.op == OP_SOLVE:
            assert torch.equal(alone.result["x"], r.result["x"]), "request %d: x differs alone vs mix" % r.rid
        elif r.op == OP_LOGDET:
            assert torch.equal(alone.result["logdet"], r.result["logdet"]), "request %d: logdet differs" % r.rid

    # oracle on the device-drawn values, one solve and one logdet per pattern
    checked = set()
    for r in done:
        key = (r.pattern, r.op)
        if r.op not in (OP_SOLVE, OP_LOGDET) or key in checked:
            continue
        checked.add(key)
        p = pats[r.pattern]
        vals = r.result["values"].cpu().numpy()
        B = np.ones((p.N, 1))
        ref = oracle_reference(p, vals, B)
        assert ref["info"] == 0
        if r.op == OP_SOLVE:
            x = r.result["x"].cpu().numpy().reshape(-1, 1)
            assert rel(x, ref["X"]) <= 1e-12
        else:
            ld = r.result["logdet"].item()
            assert abs(ld - ref["logdet"]) <= 1e-12 * abs(ref["logdet"])
    assert len(checked) == 6


def test_device_values_deterministic_and_spd():
    """The device generator is a pure function of (pattern, seed): two draws
    agree bit for bit on different streams, different seeds differ, and the
    diagonal dominance law holds (diagonal = absolute row sum + 1)."""
    import torch

    from paper_2501_02483_amd.devgen import DevicePattern

    p = I.make_pattern(5000, 30, 120)
    dp = DevicePattern(p)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    t1 = torch.empty(2 * p.N, dtype=torch.float64, device="cuda")
    t2 = torch.empty(2 * p.N, dtype=torch.float64, device="cuda")
    v1 = dp.values(11, stream=s1, tmp=t1)
    v2 = dp.values(11, stream=s2, tmp=t2)
    v3 = dp.values(12, stream=s2, tmp=t2)
    torch.cuda.synchronize()
    assert torch.equal(v1, v2)
    assert not torch.equal(v1, v3)
    v = v1.cpu().numpy()
    rp = p.row_ptr()
    N = p.N
    rowabs = np.zeros(N)
    for i in range(N):
        off = v[rp[i]:rp[i + 1] - 1]
        rowabs[i] += np.abs(off).sum()
        cols = np.arange(p.f[i], i)
        np.add.at(rowabs, cols, np.abs(off))
    diag = v[rp[1:] - 1]
    assert np.allclose(diag, rowabs + 1.0, rtol=1e-13, atol=0)
    off = np.delete(v, rp[1:] - 1)
    # off-diagonals look standard normal
    assert abs(off.mean()) < 0.01 and abs(off.std() - 1.0) < 0.01


def _mix_then_alone(pats, reqs, slots, precision=0, ordering=None):
    import torch

    from paper_2501_02483_amd.serve import OP_LOGDET, OP_SOLVE, GpuExecutor, Request, Server

    budget = 64 << 30
    ex = GpuExecutor(pats, tile=64, slots=slots, precision=precision, ordering=ordering)
    assert (ex.workers is not None) == (precision != 0)    # mixed: one issuing thread per slot
    done = Server(ex, budget, slots).run(reqs)
    ex.close()
    torch.cuda.synchronize()
    assert len(done) == len(reqs)
    assert all(r.result["info"] == 0 for r in done)
    ex1 = GpuExecutor(pats, tile=64, slots=1, precision=precision, ordering=ordering)
    for r in sorted(done, key=lambda r: r.rid):
        alone = Server(ex1, budget, 1).run([Request(rid=r.rid, arrival=0.0, pattern=r.pattern, op=r.op,
                                                    seed=r.seed)])[0]
        assert alone.result["info"] == 0
        assert torch.equal(alone.result["values"], r.result["values"])
        if r.op == OP_SOLVE:
            assert torch.equal(alone.result["x"], r.result["x"]), "request %d: x differs alone vs mix" % r.rid
        elif r.op == OP_LOGDET:
            assert torch.equal(alone.result["logdet"], r.result["logdet"]), "request %d: logdet differs" % r.rid
    ex1.close()
    return done


def test_serve_large_pattern_mix_equals_alone_and_oracle():
    """A pattern of the serving workload's size (n = 120,000, half-width 400,
    arrow 100; adaptable ND as the serving bench uses for long patterns)
    served together with a small one: bitwise the same alone and in the mix,
    and the solution and log-determinant of the large pattern match the
    oracle on the values the device drew."""
    import torch

    import paper_2501_02483_amd as S
    from paper_2501_02483_amd.serve import OP_LOGDET, OP_SOLVE, Request

    pats = [I.make_pattern(120_000, 100, 400, name="L0"), I.make_pattern(10_000, 16, 64, name="L1")]
    reqs = [Request(rid=i, arrival=0.0, pattern=(0 if i < 4 else 1), op=[1, 2, 1, 2, 1, 2][i], seed=900 + i)
            for i in range(6)]
    say("[gpu serve] large pattern (n=120,000) with a small one, 3 slots")
    done = _mix_then_alone(pats, reqs, 3, ordering=S.STILES_ORDER_ADAPTABLE_ND)
    p = pats[0]
    for op in (OP_SOLVE, OP_LOGDET):
        r = next(r for r in done if r.pattern == 0 and r.op == op)
        vals = r.result["values"].cpu().numpy()
        ref = oracle_reference(p, vals, np.ones((p.N, 1)))
        assert ref["info"] == 0
        if op == OP_SOLVE:
            e = rel(r.result["x"].cpu().numpy().reshape(-1, 1), ref["X"])
        else:
            e = abs(r.result["logdet"].item() - ref["logdet"]) / abs(ref["logdet"])
        say("   op %d error %.2e" % (op, e))
        assert e <= 1e-12


def test_serve_mixed_precision_mix_equals_alone():
    """Mixed-precision serving: FP32 updates with FP64 refinement per solve
    request; results bitwise the same alone and in the mix, solutions within
    1e-12 of the FP64 oracle after refinement, log-determinants within the
    mixed-mode bound."""
    from paper_2501_02483_amd.serve import OP_LOGDET, OP_SOLVE, Request

    pats = _patterns()
    reqs = [Request(rid=i, arrival=0.0, pattern=i % 3, op=(i // 3) % 3, seed=800 + i, precision=1)
            for i in range(9)]
    say("[gpu serve] mixed precision, 9 requests on 3 slots")
    done = _mix_then_alone(pats, reqs, 3, precision=1)
    for r in done:
        if r.op not in (OP_SOLVE, OP_LOGDET):
            continue
        p = pats[r.pattern]
        ref = oracle_reference(p, r.result["values"].cpu().numpy(), np.ones((p.N, 1)))
        if r.op == OP_SOLVE:
            assert rel(r.result["x"].cpu().numpy().reshape(-1, 1), ref["X"]) <= 1e-12
        else:
            assert abs(r.result["logdet"].item() - ref["logdet"]) <= 1e-6 * abs(ref["logdet"])
