"""Tile-size, ordering and occupancy autotuner.

The paper tunes its tile size by sweeping (Section IV-B: larger tiles on the
GPU; Appendix B: 40 to 400 on the CPU) and picks an ordering per matrix
structure (Section III-A).  Here the candidates are the tile sizes the
kernels support (32, 64), the natural order or adaptable nested dissection
with several partition counts (single matrices), and caps on the number of
persistent workgroups; each candidate is timed on the device with the
library's own event pair around the factorization kernel, and the fastest is
kept.  A choice is made per pattern (single matrices) or per batch (one tile
size per launch), and cached by pattern signature.
"""
import hashlib
import json
import os

import numpy as np

TILES = (32, 64)


def signature(pattern):
    h = hashlib.sha1(np.ascontiguousarray(pattern.f).tobytes()).hexdigest()[:16]
    return "n%d_a%d_%s" % (pattern.n, pattern.a, h)


def _time_factor(fac, dv, reps):
    import paper_2501_02483_amd as S
    S.stiles_factor_set_timing(fac.handle, True)
    ts = []
    for _ in range(reps + 1):
        fac.factorize(dv)
        ts.append(S.stiles_factor_kernel_ms(fac.handle, 0))
    S.stiles_factor_set_timing(fac.handle, False)
    return float(np.median(ts[1:]))


# orderings tried for one matrix: the natural order, and adaptable nested
# dissection with the analysis' own partition count and a few fixed ones
# (0 = chosen by the analysis); the schedule is the one the analysis derives
# for each choice
ORDERINGS = (("none", 0), ("nd", 0), ("nd", 4), ("nd", 8), ("nd", 16), ("nd", 32))


def tune_single(pattern, values, tiles=TILES, wg_caps=(0,), reps=3, precision=0, orderings=ORDERINGS):
    """Time factorizations of one matrix for each candidate (tile size x
    ordering x workgroup cap); returns (best dict, all results).  values: a
    host array or a device tensor in the pattern's row-profile order."""
    import torch

    import paper_2501_02483_amd as S
    dv = values if hasattr(values, "data_ptr") else torch.from_numpy(values).cuda()
    results = []
    seen = set()
    for T in tiles:
        for oname, parts in orderings:
            ordv = S.STILES_ORDER_ADAPTABLE_ND if oname == "nd" else S.STILES_ORDER_NONE
            sym = S.Symbolic.from_pattern(pattern, tile=T, ordering=ordv, nd_parts=parts)
            key = (T, sym.info.ordering_used, sym.info.nd_parts)
            if key in seen:          # e.g. ND infeasible (falls back) or the same P twice
                continue
            seen.add(key)
            fac = S.Factor(sym, precision)
            for cap in wg_caps:
                fac.set_max_workgroups(cap)
                ms = _time_factor(fac, dv, reps)
                results.append({"tile": T, "ordering": oname if sym.info.nd_parts > 1 else "none",
                                "nd_parts": sym.info.nd_parts, "max_wg": cap, "ms": ms,
                                "tflops": sym.info.flops_alg / ms / 1e9,
                                "exec_over_alg": sym.info.flops_exec / sym.info.flops_alg})
            del fac
    best = min(results, key=lambda r: r["ms"])
    return best, results


def batch_symbolics(patterns, tile, nd_min_rows=0, nd_parts=2):
    """Symbolic objects for a batch: matrices with at least nd_min_rows band
    tile rows (0: none) are cut into nd_parts partitions by adaptable nested
    dissection, so that the longest pivot chains of the batch shrink (two
    partitions add no fill: both have their separator at their end); the
    others keep their order."""
    import paper_2501_02483_amd as S
    out = []
    for p in patterns:
        long_chain = nd_min_rows > 0 and (p.n + tile - 1) // tile >= nd_min_rows
        if long_chain:
            out.append(S.Symbolic.from_pattern(p, tile=tile, ordering=S.STILES_ORDER_ADAPTABLE_ND, nd_parts=nd_parts))
        else:
            out.append(S.Symbolic.from_pattern(p, tile=tile, ordering=S.STILES_ORDER_NONE))
    return out


def tune_batch(patterns, values, tiles=TILES, reps=2, nd_thresholds=(0, 240, 160, 120)):
    """Time one batched launch of all matrices for each tile size and
    nested-dissection threshold (values: host arrays or device tensors)."""
    import torch

    import paper_2501_02483_amd as S
    dvals = [v if hasattr(v, "data_ptr") else torch.from_numpy(v).cuda() for v in values]
    results = []
    for T, thr in [(T, thr) for T in tiles for thr in nd_thresholds]:
        syms = batch_symbolics(patterns, T, thr)
        facs = [S.Factor(s) for s in syms]
        batch = S.Batch(facs)
        batch.factorize(dvals)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            batch.factorize(dvals)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        F = sum(s.info.flops_alg for s in syms)
        results.append({"tile": T, "nd_min_rows": thr, "nd_matrices": sum(1 for s in syms if s.info.nd_parts > 1),
                        "ms": float(np.median(ts)), "tflops": F / float(np.median(ts)) / 1e9})
        del batch, facs, syms
    best = min(results, key=lambda r: r["ms"])
    return best, results


class Cache:
    """JSON cache of tuning decisions keyed by pattern signature."""

    def __init__(self, path):
        self.path = path
        self.data = json.load(open(path)) if os.path.exists(path) else {}

    def get(self, pattern):
        return self.data.get(signature(pattern))

    def put(self, pattern, choice):
        self.data[signature(pattern)] = choice
        with open(self.path, "w") as fh:
            json.dump(self.data, fh, indent=1, sort_keys=True)
