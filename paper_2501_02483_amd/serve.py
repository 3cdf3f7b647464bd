"""Request serving over resident sparsity patterns (continuous batching).

INLA-style workloads refactorize the same sparsity pattern many times with
new values (the paper, Sections I and III-A, Appendix A).  The server keeps
one symbolic object per pattern and a pool of device workspaces (resident
task tables and factor storage), admits requests by their HBM footprint, and
launches every admitted request at once on a free stream slot: requests that
arrive while others run are started as soon as a slot and memory free up, and
their persistent kernels share the GPU (each launch is capped to its share of
the workgroups).  Latency is measured from the request's scheduled arrival.

Executors:
  GpuExecutor  -- the HIP library through the C ABI (values drawn on the device)
  FakeExecutor -- modeled durations and memory on a virtual clock, for CPU tests
"""
import heapq
import time
from dataclasses import dataclass, field

import numpy as np

OP_FACTORIZE, OP_SOLVE, OP_LOGDET = 0, 1, 2
OP_NAMES = {OP_FACTORIZE: "factorize", OP_SOLVE: "factorize+solve", OP_LOGDET: "factorize+logdet"}


@dataclass
class Request:
    rid: int
    arrival: float            # scheduled arrival, seconds from the start
    pattern: int
    op: int
    seed: int
    precision: int = 0
    t_admit: float = -1.0
    t_done: float = -1.0
    slot: int = -1
    bypassed: int = 0
    result: dict = field(default_factory=dict)

    @property
    def latency(self):
        return self.t_done - self.arrival


class Server:
    """Admission, slot assignment, completion.

    A request is admitted when a slot is free and the in-flight footprint plus
    its own stays within the HBM budget.  Two orders of admission:

    policy "fifo": arrival order.  When the queue head does not fit, later
    requests that fit may bypass it, but the head can be bypassed at most
    `max_bypass` times (no starvation).

    policy "sjf": the queued request with the least expected work first
    (executor.cost(req); ties by arrival), which shortens the waits of the
    many small requests behind a large one.  Every admission ahead of an
    older queued request counts as one bypass of it; a request bypassed
    `max_overtake` times goes next (the oldest such first) and nothing else is
    admitted until it fits, so no request starves."""

    def __init__(self, executor, budget_bytes, slots, max_bypass=4, policy="fifo", max_overtake=16):
        if policy not in ("fifo", "sjf"):
            raise ValueError("policy must be 'fifo' or 'sjf'")
        self.ex = executor
        self.budget = budget_bytes
        self.slots = slots
        self.max_bypass = max_bypass
        self.policy = policy
        self.max_overtake = max_overtake
        self.inflight = {}        # slot -> request
        self.used = 0
        self.max_used = 0
        self.admit_order = []

    def _free_slot(self):
        for s in range(self.slots):
            if s not in self.inflight:
                return s
        return -1

    def _admit(self, req, now):
        fp = self.ex.footprint(req)
        if fp > self.budget:
            raise ValueError("request %d needs %d bytes, more than the whole budget" % (req.rid, fp))
        slot = self._free_slot()
        req.slot = slot
        req.t_admit = now
        self.inflight[slot] = req
        self.used += fp
        self.max_used = max(self.max_used, self.used)
        self.admit_order.append(req.rid)
        self.ex.launch(req, slot)

    def _try_admit(self, queue, now):
        if self.policy == "sjf":
            return self._try_admit_sjf(queue, now)
        while queue and self._free_slot() >= 0:
            head = queue[0]
            if self.ex.footprint(head) > self.budget:
                raise ValueError("request %d needs more than the whole budget" % head.rid)
            if self.used + self.ex.footprint(head) <= self.budget:
                self._admit(queue.pop(0), now)
                continue
            if head.bypassed >= self.max_bypass:
                return
            for i in range(1, len(queue)):
                r = queue[i]
                if self.used + self.ex.footprint(r) <= self.budget:
                    head.bypassed += 1
                    self._admit(queue.pop(i), now)
                    break
            else:
                return

    def _try_admit_sjf(self, queue, now):
        while queue and self._free_slot() >= 0:
            for r in queue:
                if self.ex.footprint(r) > self.budget:
                    raise ValueError("request %d needs more than the whole budget" % r.rid)
            starving = [r for r in queue if r.bypassed >= self.max_overtake]
            if starving:
                cands = [min(starving, key=lambda r: (r.arrival, r.rid))]
            else:
                cands = sorted(queue, key=lambda r: (self.ex.cost(r), r.arrival, r.rid))
            pick = next((r for r in cands if self.used + self.ex.footprint(r) <= self.budget), None)
            if pick is None:
                return
            for r in queue:
                if r is not pick and (r.arrival, r.rid) < (pick.arrival, pick.rid):
                    r.bypassed += 1
            queue.remove(pick)
            self._admit(pick, now)

    def run(self, requests):
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        queue = []
        i = 0
        done = []
        self.ex.start()
        while i < len(reqs) or queue or self.inflight:
            now = self.ex.now()
            while i < len(reqs) and reqs[i].arrival <= now:
                queue.append(reqs[i])
                i += 1
            self._try_admit(queue, now)
            for slot, req in list(self.inflight.items()):
                if self.ex.poll(req):
                    req.t_done = self.ex.now()
                    self.used -= self.ex.footprint(req)
                    del self.inflight[slot]
                    done.append(req)
            nxt = reqs[i].arrival if i < len(reqs) else None
            self.ex.idle(nxt, bool(self.inflight))
        return done


def summarize(done, flops_of=None):
    lat = np.array([r.latency for r in done])
    span = max(r.t_done for r in done) - min(r.arrival for r in done)
    out = {"requests": len(done), "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
           "achieved_rps": len(done) / span if span > 0 else float("nan")}
    if flops_of is not None:
        out["tflops"] = sum(flops_of(r) for r in done) / span / 1e12
    per, by_op = {}, {}
    for r in done:
        per.setdefault(r.pattern, []).append(r.latency)
        by_op.setdefault(r.op, []).append(r.latency)
    out["per_pattern_count"] = {int(k): len(v) for k, v in sorted(per.items())}
    out["per_pattern_p50_ms"] = {int(k): float(np.percentile(v, 50) * 1e3) for k, v in sorted(per.items())}
    out["per_pattern_p99_ms"] = {int(k): float(np.percentile(v, 99) * 1e3) for k, v in sorted(per.items())}
    out["per_op_p50_ms"] = {OP_NAMES[k]: float(np.percentile(v, 50) * 1e3) for k, v in sorted(by_op.items())}
    out["per_op_p99_ms"] = {OP_NAMES[k]: float(np.percentile(v, 99) * 1e3) for k, v in sorted(by_op.items())}
    return out


# ------------------------------------------------------------------ executors

class FakeExecutor:
    """Virtual-clock executor: a request takes flops / rate + overhead seconds,
    slowed by the number of requests sharing the device (processor sharing)."""

    def __init__(self, flops, ws_bytes, rate=1e12, overhead=1e-4, values_bytes=None):
        self.flops = flops
        self.ws = ws_bytes
        self.vb = values_bytes or [0] * len(flops)
        self.rate = rate
        self.overhead = overhead
        self.t = 0.0
        self.active = {}          # rid -> remaining work (seconds at full rate)

    def start(self):
        self.t = 0.0

    def now(self):
        return self.t

    def footprint(self, req):
        return self.ws[req.pattern] + self.vb[req.pattern]

    def cost(self, req):
        return self.flops[req.pattern] / self.rate + self.overhead

    def launch(self, req, slot):
        self.active[req.rid] = self.flops[req.pattern] / self.rate + self.overhead
        req.result["launched_at"] = self.t

    def poll(self, req):
        return req.rid not in self.active

    def idle(self, next_arrival, busy):
        # advance to the next event: an arrival or the first completion
        n = len(self.active)
        t_next = next_arrival if next_arrival is not None else float("inf")
        if n:
            kmin = min(self.active, key=lambda k: (self.active[k], k))
            rem = self.active[kmin]
            t_done = self.t + rem * n
            if t_done <= t_next:
                for k in list(self.active):
                    if k == kmin or self.active[k] <= rem:
                        del self.active[k]
                    else:
                        self.active[k] -= rem
                self.t = t_done
                return
        if t_next < float("inf"):
            if n:
                dt = t_next - self.t
                for k in self.active:
                    self.active[k] -= dt / n
            self.t = max(self.t, t_next)


class GpuExecutor:
    """Runs requests through the C ABI on a pool of streams.

    Per pattern: a Symbolic object, device row pointers for the value
    generator, and a pool of workspaces (Factor objects) reused across
    requests.  A request draws its values on the device (seeded), then
    factorizes, and solves one right-hand side or takes the log-determinant.

    In mixed precision a solve refines in FP64, and each refinement step
    reads its residual norms back to the host (a stream synchronization).
    So that one refining request does not hold up admissions and the other
    slots, requests are then issued from one host thread per slot (the C
    calls release the interpreter lock); completion is still observed by the
    serving loop.  host_threads=None picks threads for mixed precision only."""

    def __init__(self, patterns, tile=64, precision=0, slots=4, nrhs=1, ordering=None, nd_min_rows=512,
                 host_threads=None, keep_results=True):
        """ordering: None/STILES_ORDER_NONE keeps the natural order; with
        STILES_ORDER_ADAPTABLE_ND, patterns with at least nd_min_rows band
        tile rows (long pivot chains) are partitioned, the others not.
        keep_results=False frees a request's values and solution on
        completion (long runs; only info and the log-determinant stay)."""
        import threading
        from concurrent.futures import ThreadPoolExecutor
        import torch
        import paper_2501_02483_amd as S
        from paper_2501_02483_amd.devgen import DevicePattern
        self.S = S
        self.torch = torch
        self.patterns = patterns
        self.precision = precision
        self.nrhs = nrhs
        nd = ordering == S.STILES_ORDER_ADAPTABLE_ND

        def analyze(p):
            if nd and (p.n + tile - 1) // tile >= nd_min_rows:
                return S.Symbolic.from_pattern(p, tile=tile, ordering=S.STILES_ORDER_ADAPTABLE_ND)
            return S.Symbolic.from_pattern(p, tile=tile, ordering=S.STILES_ORDER_NONE)

        self.syms = [analyze(p) for p in patterns]
        self.devpat = [DevicePattern(p) for p in patterns]
        self.ws_bytes = [s.workspace_size(precision, nrhs) for s in self.syms]
        self.slots = slots
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        # per-slot generator scratch: requests in flight on different slots
        # must not share it
        nmax = max(p.N for p in patterns)
        self.gtmp = [torch.empty(2 * nmax, dtype=torch.float64, device="cuda") for _ in range(slots)]
        self.pool = {i: [] for i in range(len(patterns))}
        self.pool_lock = threading.Lock()
        self.vals = {}            # slot -> values tensor
        self.events = {}
        if host_threads is None:
            host_threads = precision != S.STILES_FP64
        self.workers = ThreadPoolExecutor(max_workers=slots) if host_threads else None
        self.futures = {}
        self.keep_results = keep_results
        self.cap_wg = None
        self.t0 = 0.0

    def flops(self, pattern):
        return self.syms[pattern].info.flops_alg

    def cost(self, req):
        """Expected work of a request (for shortest-first admission): the
        flops its factorization executes."""
        return self.syms[req.pattern].info.flops_exec

    def footprint(self, req):
        p = self.patterns[req.pattern]
        return self.ws_bytes[req.pattern] + 8 * p.nnz + 8 * p.N * self.nrhs

    def start(self):
        self.torch.cuda.synchronize()
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def _factor(self, pi, stream):
        with self.pool_lock:
            if self.pool[pi]:
                return self.pool[pi].pop()
        f = self.S.Factor(self.syms[pi], self.precision, nrhs_max=self.nrhs, stream=stream)
        return f

    def launch(self, req, slot):
        if self.workers is None:
            self._issue(req, slot)
        else:
            self.futures[req.rid] = self.workers.submit(self._issue, req, slot)

    def _issue(self, req, slot):
        torch = self.torch
        st = self.streams[slot]
        with torch.cuda.stream(st):
            fac = self._factor(req.pattern, st)
            fac.set_max_workgroups(max(64, 512 // self.slots))
            v = self.devpat[req.pattern].values(req.seed, stream=st, tmp=self.gtmp[slot])
            fac.factorize(v, stream=st)
            if req.op == OP_SOLVE:
                b = torch.ones(self.patterns[req.pattern].N, dtype=torch.float64, device="cuda")
                fac.solve(b, stream=st)
                req.result["x"] = b
            elif req.op == OP_LOGDET:
                req.result["logdet"] = fac.logdet(stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        req.result["factor"] = fac
        req.result["values"] = v
        self.events[req.rid] = ev

    def poll(self, req):
        fut = self.futures.get(req.rid)
        if fut is not None:
            if not fut.done():
                return False
            del self.futures[req.rid]
            fut.result()              # re-raises an error of the issuing thread
        ev = self.events.get(req.rid)
        if ev is None or not ev.query():
            return False
        fac = req.result.pop("factor")
        req.result["info"] = fac.info(stream=self.streams[req.slot])
        with self.pool_lock:
            self.pool[req.pattern].append(fac)
        del self.events[req.rid]
        if not self.keep_results:
            req.result.pop("values", None)
            req.result.pop("x", None)
        return True

    def close(self):
        if self.workers is not None:
            self.workers.shutdown(wait=True)
            self.workers = None

    def idle(self, next_arrival, busy):
        if busy:
            time.sleep(20e-6)
        elif next_arrival is not None:
            dt = next_arrival - self.now()
            if dt > 0:
                time.sleep(min(dt, 0.01))
