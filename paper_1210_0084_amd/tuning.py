"""Work-item autotuner and HIP-graph capture for batched sliCQ calls.

The plan's tuning options choose how the kernels cut the work: whether each
slice runs in one workgroup (``fused``: half spectrum and band transforms in
LDS, where they fit) or through the multi-kernel pipeline, and for the
pipeline the number of coefficients per analysis work item (``group_cap``),
the target complex values per synthesis work item (``lds_cap``) and the values
per slice-FFT work item (``pass_cap``), which set the block sizes and the
radix schedules of the band and slice transforms. ``autotune`` times every
candidate on the caller's batch shape with HIP events (content does not
change the time of the transform) and returns the fastest, cached on disk
per (plan parameters, dtype, batch shape, device).
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Optional, Sequence

CANDIDATES = [dict(fused=True, layout="band")] + [
    dict(fused=False, group_cap=g, pass_cap=p, lds_cap=l, layout="band")
    for g in (1024, 2048, 4096)
    for p in (2048, 4096)
    for l in (2048, 4096, 8192)
]


def _key(params: dict, dtype: str, lengths: Sequence[int], device_name: str) -> str:
    sig = json.dumps([params, dtype, sorted(int(t) for t in lengths), device_name], sort_keys=True)
    return hashlib.sha256(sig.encode()).hexdigest()[:24]


def autotune(params: dict, lengths: Sequence[int], dtype: str = "f32", cache: Optional[str] = None,
             reps: int = 5, candidates=None) -> Dict:
    """Fastest tuning options for analysis + synthesis of a batch of `lengths`.

    `params` holds fs, fmin, fmax, bins_per_octave, slice_len, transition (and
    optionally min_win, dual_slice). Returns a dict with the chosen options and
    the measured milliseconds of every candidate.
    """
    import torch
    from . import Plan, SlicqError

    dev = torch.device("cuda", torch.cuda.current_device())
    name = torch.cuda.get_device_name(dev)
    key = _key(params, dtype, lengths, name)
    db = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            db = json.load(fh)
        if key in db:
            return db[key]
    tdt = torch.float32 if dtype == "f32" else torch.float64
    ctype = torch.complex64 if dtype == "f32" else torch.complex128
    total = int(sum(lengths))
    x = torch.randn(total, dtype=tdt, device=dev)
    y = torch.empty_like(x)
    results = []
    for cand in (candidates or CANDIDATES):
        try:
            plan = Plan(**params, **cand)
        except SlicqError:
            continue
        if cand.get("fused") and (0 if dtype == "f32" else 1) not in plan.fused_dtypes:
            continue                          # the slice does not fit one workgroup: same as a pipeline candidate
        lay = plan.batch_layout(lengths)
        coef = torch.empty(max(lay.coef_len, 1), dtype=ctype, device=dev)
        for _ in range(2):
            plan.analyze_batched(x, out=coef, layout=lay)
            plan.synthesize_batched(coef, out=y, layout=lay)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize(dev)
        e0.record()
        for _ in range(reps):
            plan.analyze_batched(x, out=coef, layout=lay)
            plan.synthesize_batched(coef, out=y, layout=lay)
        e1.record()
        torch.cuda.synchronize(dev)
        results.append((e0.elapsed_time(e1) / reps, cand))
        del plan, coef
    if not results:
        raise SlicqError("no tuning candidate is valid for these parameters")
    results.sort(key=lambda r: r[0])
    best = {"options": results[0][1], "ms": results[0][0],
            "all": [{"ms": round(ms, 4), **c} for ms, c in results]}
    if cache:
        db[key] = best
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as fh:
            json.dump(db, fh, indent=1)
    return best


class BatchGraph:
    """Analysis + synthesis of one batch shape captured in a HIP graph.

    Every kernel of both calls (task builder, slice FFTs, band transforms,
    overlap-adds) is recorded once; ``replay()`` relaunches the whole
    sequence with a single graph launch on the current stream. Inputs and
    outputs are the fixed tensors given here (fill ``x`` before replaying).
    """

    def __init__(self, plan, x, coef, y, layout, adjoint: bool = False):
        import torch
        self.plan, self.x, self.coef, self.y, self.layout = plan, x, coef, y, layout
        dt = 0 if x.dtype == torch.float32 else 1
        plan._ensure_tables(dt, x.device)
        # the graph records this workspace's address: it is owned here, so no
        # later call on the plan (which may replace the plan's own workspace)
        # can free it while the graph may still be replayed
        self.work = torch.empty(plan.workspace_bytes(dt, layout.total_slices), dtype=torch.uint8, device=x.device)
        layout.device(x.device)
        # warm up outside the capture (first-use attribute settings, allocations)
        self._run(adjoint)
        torch.cuda.synchronize(x.device)
        self.graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream(device=x.device)
        s.wait_stream(torch.cuda.current_stream(x.device))
        with torch.cuda.stream(s):
            with torch.cuda.graph(self.graph, stream=s):
                self._run(adjoint)
        torch.cuda.current_stream(x.device).wait_stream(s)
        torch.cuda.synchronize(x.device)

    def _run(self, adjoint):
        self.plan.analyze_batched(self.x, out=self.coef, layout=self.layout, work=self.work)
        self.plan.synthesize_batched(self.coef, out=self.y, layout=self.layout, adjoint=adjoint, work=self.work)

    def replay(self):
        self.graph.replay()
