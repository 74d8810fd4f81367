"""sliCQ analysis + synthesis throughput on one MI355X.

Workload (default): 60 s of stereo audio at 44.1 kHz (2 x 2,646,000 samples of
seeded pink noise plus harmonic tones), 48 bins per octave from 32.7 Hz to
22.05 kHz, slice length 2N = 65536, Tukey transition 8192, FP32. One step is
the analysis of both channels followed by their synthesis (one batched launch
sequence each); inputs are resident in HBM before the timed region.

Prints one JSON line: Msamples/s of audio (padding excluded); the roofline
of the dominant kernel, whose achieved rate counts only its share of the
path's algorithmic bytes (the signal read once, the coefficients written once
and read once, the output written once; every intermediate it moves is
overhead and appears in `traffic`), against the 8 TB/s HBM peak and against a
device copy timed in the same run; per-stage timings; sub-records for the
batched (ragged batch in one HIP graph), differentiable (loss forward +
adjoint backward) and streaming (p50/p99 slice latency) forms; and the FP64
CPU oracle timed on the host: the 2^16-sample FP64 workload in CPU seconds,
and a 10 s excerpt of the benchmark signal single-process and with a process
pool over slices (median of 5 after a warm-up, core count and CPU model).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "sliCQ analysis+synthesis Msamples/s at 1 GPU, % HBM roofline; p99 slice latency"
STAGES = ["fwd_pass1", "fwd_pass2", "band_ana", "band_syn", "inv_passA", "inv_passB"]


def stage_bytes(plan, n_slices: int, b: int) -> dict:
    """Bytes each kernel's interface reads and writes once per launch (b =
    bytes per real value): algorithmic bytes plus the intermediates the
    pipeline passes between kernels."""
    N, M, cps = plan.N, plan.transition, plan.coefs_per_slice
    cb = 2 * b
    win = N + M - 1                         # non-zero samples of one slice window
    per = {
        "fwd_pass1": b * win + cb * N,      # windowed samples in, packed column FFTs out
        "fwd_pass2": cb * N + cb * (N + 1),  # column FFTs in, half spectrum out
        "band_ana": cb * (N + 1) + cb * cps,  # half spectrum in, coefficients out
        "band_syn": cb * cps + cb * (N + 1),  # coefficients in, half spectrum out
        "inv_passA": cb * (N + 1) + cb * N,
        "inv_passB": cb * N + b * win,
    }
    return {k: v * n_slices for k, v in per.items()}


def algorithmic_share(plan, n_slices: int, samples: int, b: int) -> dict:
    """Each kernel's share of the path's algorithmic bytes: the signal read
    once (slice pass 1), the coefficients written once (band analysis) and
    read once (band synthesis), the output written once (inverse pass B with
    its overlap fix-up). Intermediates (column FFTs, half spectra) count
    nothing."""
    c = 2 * b * n_slices * plan.coefs_per_slice
    return {"fwd_pass1": b * samples, "fwd_pass2": 0, "band_ana": c, "band_syn": c, "inv_passA": 0,
            "inv_passB": b * samples}


def copy_rate(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Device-to-device copy of nbytes (read + write counted), GB/s: the
    practical HBM ceiling measured in the same run."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "fused.hpp", "bandmix.hpp", "coefops.hpp", "fft_device.hpp", "pipeline.hpp", "common.hpp",
              "plan.hpp", "plan.cpp"):
        with open(os.path.join(ROOT, "paper_1210_0084_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str = "c2"):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or
    None when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.loads(fh.readline())
    if rec.get("kernels_sha256") != kernel_sources_hash() or kernel not in rec.get("kernels", {}):
        return None
    return int(rec["kernels"][kernel]["traffic_bytes"])


def time_stages(plan, n_slices, x, coef, y, reps=20, layout=None):
    import torch
    out = {}
    for s, name in enumerate(STAGES):
        plan.profile_stage(s, n_slices, x, coef, y, layout=layout)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.profile_stage(s, n_slices, x, coef, y, layout=layout)
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    return out


def _stage_report(plan, n_slices, x, coef, y, reps, layout=None):
    ms = time_stages(plan, n_slices, x, coef, y, reps, layout)
    sb = stage_bytes(plan, n_slices, 4)
    return {k: {"ms": round(ms[k], 4), "GBs": round(sb[k] / (ms[k] * 1e-3) / 1e9, 1)} for k in STAGES}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_POOL_STATE = {}


def _pool_init(opl, x):
    _POOL_STATE["opl"], _POOL_STATE["x"] = opl, x


def _pool_slices(rng):
    from oracle import analyze_slices, synthesize_slices
    opl, x = _POOL_STATE["opl"], _POOL_STATE["x"]
    c = analyze_slices(opl, x, rng[0], rng[1])
    return synthesize_slices(opl, c, len(x), rng[0], rng[1])


def _median_time(fn, runs=5):
    fn()                                    # warm-up
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def cpu_baseline(xs):
    """The FP64 oracle (unchanged) on the host cores: the 2^16-sample FP64
    workload (analysis then synthesis, CPU seconds), and a 10 s excerpt of
    the benchmark's left channel single-process and with a pool of processes
    over its slices. Median of 5 runs after one warm-up each."""
    import multiprocessing as mp
    from oracle import OraclePlan, analyze, synthesize, num_slices
    from workloads import make_c1
    p1 = _preset("c1")
    opl1 = OraclePlan(**p1)
    x1 = make_c1()
    t_c1 = _median_time(lambda: synthesize(opl1, analyze(opl1, x1), len(x1)))
    prm = _preset("c2")
    opl = OraclePlan(**prm)
    T = int(10 * prm["fs"])                 # a 10 s excerpt
    x = xs[0][:T].astype(np.float64)
    t_one = _median_time(lambda: synthesize(opl, analyze(opl, x), T))
    err = float(np.abs(synthesize(opl, analyze(opl, x), T) - x).max())
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    procs = max(1, min(16, avail))          # the host's share for one GPU
    S = num_slices(T, opl.two_n)
    cuts = np.linspace(0, S, min(procs, S) + 1).astype(int)
    ranges = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    ctx = mp.get_context("fork")
    with ctx.Pool(len(ranges), initializer=_pool_init, initargs=(opl, x)) as pool:
        def pooled():
            return sum(pool.map(_pool_slices, ranges))[:T]
        t_pool = _median_time(pooled)
        perr = float(np.abs(pooled() - x).max())
    rate = lambda n, t: n / t / 1e6
    # the other FP32 configurations' plans, single process, on one signal each
    from workloads import noise_plus_sines
    side = {}
    for name, T_s in (("c3", int(10 * 44100)), ("c4", 264600), ("c5", int(10 * 48000))):
        pk = _preset(name)
        ok = OraclePlan(**pk)
        xk = noise_plus_sines(T_s, pk["fs"], 7)
        tk = _median_time(lambda: synthesize(ok, analyze(ok, xk), T_s))
        side[name] = {"Msamples_per_s": round(rate(T_s, tk), 3), "seconds": round(tk, 4), "samples": T_s}
    return {"value": round(rate(T, t_pool), 3), "unit": "Msamples/s", "cores": len(ranges), "kind": "oracle",
            "sample": f"FP64 numpy oracle, analysis+synthesis of a 10 s excerpt ({T} samples, {S} slices) of the "
                      f"benchmark's left channel, slices split over a pool of {len(ranges)} processes; median of 5 "
                      f"after a warm-up; reconstruction max error {max(err, perr):.1e}",
            "single_process": {"value": round(rate(T, t_one), 3), "unit": "Msamples/s", "cores": 1,
                               "seconds": round(t_one, 4)},
            "fp64_2p16_workload": {"seconds": round(t_c1, 4), "Msamples_per_s": round(rate(len(x1), t_c1), 3),
                                   "cores": 1, "sample": "2^16 samples, B=12, 110-11025 Hz, 2N=8192, M=1024, "
                                                         "analysis then synthesis"},
            "side_by_side_single_process": side,
            "nproc": os.cpu_count(), "cpu_affinity": avail, "cpu_model": _cpu_model()}


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _time(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0, e1 = _events()
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _preset(name):
    from workloads import PRESETS
    p = PRESETS[name]
    return dict(fs=p.fs, fmin=p.fmin, fmax=p.fmax, bins_per_octave=p.bins_per_octave, slice_len=p.slice_len,
                transition=p.transition)


def _frac(nbytes, ms, copy_gbs=None):
    gbs = nbytes / (ms * 1e-3) / 1e9
    out = {"GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    if copy_gbs:
        out["frac_of_copy"] = round(gbs / copy_gbs, 4)
    return out


def bench_batched(args, copy_gbs=None):
    """Ragged batch of 256 signals (5-30 s): one graph launch of the batched
    calls, the same calls eagerly, and a loop of single-signal calls."""
    import torch
    import paper_1210_0084_amd as sq
    from paper_1210_0084_amd.tuning import BatchGraph, autotune
    from workloads import make_c3_cut
    dev = torch.device("cuda:0")
    prm = _preset("c3")
    lens, offs0, base = make_c3_cut(args.c3_signals)
    base = base.astype(np.float32)
    tuned = None
    opts = {}
    if args.c3_tune:
        tuned = autotune(prm, lens, "f32", cache=args.tune_cache, reps=3)
        opts = dict(tuned["options"])
    if args.fused:
        opts.setdefault("fused", True)
    plan = sq.Plan(**prm, **opts)
    lay = plan.batch_layout(lens)
    x = torch.tensor(np.concatenate([base[o:o + t] for o, t in zip(offs0, lens)]), device=dev)
    coef = torch.empty(lay.coef_len, dtype=torch.complex64, device=dev)
    y = torch.empty_like(x)
    graph = BatchGraph(plan, x, coef, y, lay)
    ms_graph = _time(graph.replay, args.steps, args.warmup)
    err = float((y - x).abs().max())
    ms_eager = _time(lambda: (plan.analyze_batched(x, out=coef, layout=lay),
                              plan.synthesize_batched(coef, out=y, layout=lay)), args.steps, args.warmup)
    stages = _stage_report(plan, lay.total_slices, x, coef, y, args.stage_reps, lay)
    offs = lay.x_off
    cofs = lay.coef_off
    views = [(x[offs[i]:offs[i + 1]], coef[cofs[i]:cofs[i] + lay.slices[i] * plan.coefs_per_slice],
              y[offs[i]:offs[i + 1]]) for i in range(len(lens))]

    def loop():
        for xi, ci, yi in views:
            plan.analyze(xi, out=ci)
            plan.synthesize(ci, xi.numel(), out=yi)
    ms_loop = _time(loop, max(1, args.steps // 5), 1)
    samples = int(sum(lens))
    path_bytes = 2 * 4 * samples + 2 * 8 * lay.total_slices * plan.coefs_per_slice
    rate = lambda ms: round(samples / (ms * 1e-3) / 1e6, 1)
    return {"metric": METRIC, "value": rate(ms_graph), "unit": "Msamples/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_graph, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"ragged batch of {len(lens)} signals of 5-30 s (44.1 kHz), B=24, "
                                   "41.2-22050 Hz, 2N=32768, M=4096; analysis+synthesis in one HIP graph",
                       "samples": samples, "slices": lay.total_slices, "options": opts or "defaults"},
            "path": dict(_frac(path_bytes, ms_graph, copy_gbs), algorithmic_bytes=path_bytes,
                         reconstruction_max_abs_err=err),
            "stages": stages,
            "tuning": ({"chosen": tuned["options"], "ms": round(tuned["ms"], 4), "candidates": len(tuned["all"])}
                       if tuned else None),
            "compare": {"graph_ms": round(ms_graph, 3), "eager_batched_ms": round(ms_eager, 3),
                        "per_signal_loop_ms": round(ms_loop, 3), "graph_Msps": rate(ms_graph),
                        "eager_Msps": rate(ms_eager), "loop_Msps": rate(ms_loop)}}


def bench_differentiable(args, copy_gbs=None):
    """Batch of 32 x 6 s: loss of the log-magnitude coefficients against a
    second batch, forward through SliCQFunction and backward through the
    adjoint kernel, beside the plain analysis + synthesis of the same batch."""
    import torch
    import paper_1210_0084_amd as sq
    from workloads import make_c4
    dev = torch.device("cuda:0")
    plan = sq.Plan(**_preset("c4"), fused=args.fused)
    xb = make_c4(args.c4_batch)
    yb = make_c4(args.c4_batch, target=True)
    B, T = xb.shape
    x = torch.tensor(xb, dtype=torch.float32, device=dev, requires_grad=True)
    with torch.no_grad():
        cy = sq.slicq(torch.tensor(yb, dtype=torch.float32, device=dev), plan)
        ly = torch.log1p(cy.real ** 2 + cy.imag ** 2)

    def fwd_bwd():
        # analysis kernels, the fused loss-and-gradient kernel, adjoint kernels
        x.grad = None
        loss = sq.logmag_loss(sq.slicq(x, plan), ly)
        loss.backward()

    def fwd_bwd_torch_loss():
        x.grad = None
        c = sq.slicq(x, plan)
        loss = ((torch.log1p(c.real ** 2 + c.imag ** 2) - ly) ** 2).sum()
        loss.backward()
    ms_fb = _time(fwd_bwd, args.steps, args.warmup)
    ms_fb_torch = _time(fwd_bwd_torch_loss, args.steps, args.warmup)
    lay = plan.batch_layout([T] * B)
    xf = x.detach().reshape(-1).contiguous()
    coef = torch.empty(lay.coef_len, dtype=torch.complex64, device=dev)
    yy = torch.empty_like(xf)
    ms_plain = _time(lambda: (plan.analyze_batched(xf, out=coef, layout=lay),
                              plan.synthesize_batched(coef, out=yy, layout=lay)), args.steps, args.warmup)
    ms_ana = _time(lambda: plan.analyze_batched(xf, out=coef, layout=lay), args.steps, args.warmup)
    ms_adj = _time(lambda: plan.synthesize_batched(coef, out=yy, layout=lay, adjoint=True), args.steps, args.warmup)
    plan.analyze_batched(xf, out=coef, layout=lay)
    plan.synthesize_batched(coef, out=yy, layout=lay)
    stages = _stage_report(plan, lay.total_slices, xf, coef, yy, args.stage_reps, lay)
    samples = B * T
    cbytes = 8 * lay.total_slices * plan.coefs_per_slice
    # forward (x read, c written) + backward through the adjoint (grad c read,
    # grad x written): the same algorithmic bytes as analysis + synthesis
    path_bytes = 2 * 4 * samples + 2 * cbytes
    rate = lambda ms: round(samples / (ms * 1e-3) / 1e6, 1)
    return {"metric": METRIC, "value": rate(ms_fb), "unit": "Msamples/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms_fb, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{B} x 6 s (264600 samples) at 44.1 kHz, B=36, 65.4-16000 Hz, 2N=16384, "
                                   "M=2048; log-magnitude loss forward + adjoint backward", "slices": lay.total_slices,
                       "fused": 0 in plan.fused_dtypes},
            "stages": stages,
            "hbm": {"forward_backward": _frac(path_bytes, ms_fb, copy_gbs),
                    "plain_analysis_synthesis": _frac(path_bytes, ms_plain, copy_gbs),
                    "analysis_only": _frac(4 * samples + cbytes, ms_ana, copy_gbs),
                    "adjoint_only": _frac(cbytes + 4 * samples, ms_adj, copy_gbs),
                    "algorithmic_bytes": path_bytes},
            "compare": {"forward_backward_ms": round(ms_fb, 3), "plain_analysis_synthesis_ms": round(ms_plain, 3),
                        "analysis_only_ms": round(ms_ana, 3), "adjoint_only_ms": round(ms_adj, 3),
                        "loss_kernel_ms": round(ms_fb - ms_ana - ms_adj, 3),
                        "forward_backward_torch_loss_ms": round(ms_fb_torch, 3),
                        "forward_backward_Msps": rate(ms_fb), "plain_Msps": rate(ms_plain)}}


def bench_stream(args):
    """Streaming service: 512 streams of 48 kHz audio delivering 4096-sample
    hops. Paced: hops arrive at real-time rate with Poisson stream arrivals
    and exponential lifetimes (mean 60 s), one tick thread batches whatever
    is ready; reports p50/p99 slice latency. Unpaced: every stream pushes as
    fast as the server drains (one push_packed, tick and poll_many call per
    round), for the sustainable throughput."""
    import threading
    import torch
    import paper_1210_0084_amd as sq
    from workloads import make_c5_stream
    torch.cuda.init()
    plan = sq.Plan(**_preset("c5"), layout="slice", fused=args.fused)
    fs, hop, n_streams = 48000.0, 4096, args.c5_streams
    pool = [make_c5_stream(i, int(fs * 10)).astype(np.float32) for i in range(16)]
    srv = sq.StreamServer(plan, "f32", max_streams=n_streams + 64, max_batch=2 * n_streams)
    rng = np.random.default_rng(5)
    stop = threading.Event()

    def ticker():
        while not stop.is_set():
            if srv.tick() == 0:
                time.sleep(2e-4)

    active = {}
    def open_stream(k):
        sid = srv.open()
        active[sid] = {"src": k % len(pool), "pos": 0, "end": time.perf_counter() + rng.exponential(60.0)}
    for k in range(n_streams):
        open_stream(k)
    th = threading.Thread(target=ticker, daemon=True)
    th.start()
    hop_s = hop / fs
    t0 = time.perf_counter()
    next_arrival = t0 + rng.exponential(60.0 / n_streams)
    nxt = t0
    k_new = n_streams
    while time.perf_counter() - t0 < args.c5_seconds:
        now = time.perf_counter()
        if now < nxt:
            time.sleep(min(nxt - now, 0.005))
            continue
        for sid in list(active):
            st = active[sid]
            if now > st["end"]:
                srv.close(sid)
                del active[sid]
                continue
            src = pool[st["src"]]
            a = st["pos"] % (len(src) - hop)
            srv.push(sid, src[a:a + hop])
            st["pos"] += hop
            srv.poll(sid)
        while next_arrival <= now:
            try:
                open_stream(k_new)
            except sq.SlicqBusy:
                pass
            k_new += 1
            next_arrival += rng.exponential(60.0 / n_streams)
        nxt += hop_s
    stop.set()
    th.join()
    paced = srv.stats()
    wall = time.perf_counter() - t0
    # unpaced: push one hop per stream per round as fast as ticks drain
    srv.reset_stats()
    ids = list(active)
    packed = np.concatenate([pool[active[i]["src"]][:hop] for i in ids]).astype(np.float32)
    counts = np.full(len(ids), hop, dtype=np.int64)
    t1 = time.perf_counter()
    rounds = 0
    while time.perf_counter() - t1 < args.c5_seconds / 2:
        srv.push_packed(ids, packed, counts)   # one call per round for all streams
        srv.tick()
        srv.poll_many(ids)
        rounds += 1
    un = srv.stats()
    t_un = time.perf_counter() - t1
    return {"metric": METRIC, "value": round(paced["samples_in"] / wall / 1e6, 2), "unit": "Msamples/s",
            "n_gpus": 1, "steps": paced["ticks"], "warmup": 0, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f32", "data": "synthetic",
            "config": {"workload": f"{n_streams} real-time streams at 48 kHz, 4096-sample hops, Poisson "
                                   "arrivals, mean lifetime 60 s; B=96, 27.5-20000 Hz, 2N=16384, M=2048",
                       "seconds": round(wall, 1)},
            "latency_ms": {"p50": round(paced["latency_p50_s"] * 1e3, 3), "p99": round(paced["latency_p99_s"] * 1e3, 3),
                           "max": round(paced["latency_max_s"] * 1e3, 3), "slices": paced["latency_count"]},
            "paced": {k: paced[k] for k in ("ticks", "slices", "samples_in", "samples_out", "admitted", "rejected",
                                            "closed")},
            "unpaced": {"Msamples_per_s": round(un["samples_in"] / t_un / 1e6, 2), "slices_per_s":
                        round(un["slices"] / t_un, 1), "streams": len(ids), "rounds": rounds,
                        "latency_p50_ms": round(un["latency_p50_s"] * 1e3, 3),
                        "latency_p99_ms": round(un["latency_p99_s"] * 1e3, 3)},
            "device_bytes": {"per_stream": un["bytes_per_stream"], "fixed": un["fixed_bytes"]}}


def bench_approx(args):
    """Section 5.3's approximation study, all on the GPU: SNR of the sliCQ
    layer sum s^0 + s^1 (FP32: complex analysis onto all bands, then the
    layer kernel) against the full-length CQ-NSGT on the same
    Blackman-Harris band windows (FP64, sliCQ lattice, rescaled by
    sqrt(2N / L)), for slice lengths 4096, 16384 and 65536, transitions 1/4
    and 1/128 of the slice, minimal filter lengths 4, 8, 16 and 32 bins;
    seeded random complex signals of 2^20 samples (a stand-in for the paper's
    Set 1). Mean and spread over the signals, and the full-length
    transform's own speed (FP32, the 2N = 4096 plan)."""
    import torch
    import paper_1210_0084_amd as sq
    dev = torch.device("cuda:0")
    L = 1 << args.approx_log2_len
    sigs = []
    for s in range(args.approx_signals):
        g = np.random.default_rng(100 + s)
        sigs.append(torch.tensor(g.standard_normal(L) + 1j * g.standard_normal(L), dtype=torch.complex128,
                                 device=dev))
    table = []
    full_cache = {}
    timing = None
    t0 = time.perf_counter()
    for two_n in (4096, 16384, 65536):
        for frac in (4, 128):
            for mw in (4, 8, 16, 32):
                kw = dict(fs=44100.0, fmin=200.0, fmax=22000.0, bins_per_octave=48, slice_len=two_n,
                          transition=two_n // frac, window="blackman_harris", min_win=float(mw))
                plan = sq.Plan(**kw)
                S = plan.num_slices(L)
                r = math.sqrt(two_n / L)
                stored = (S // 2) * plan.coefs_per_slice
                snrs = []
                for si, f in enumerate(sigs):
                    key = (two_n, mw, si)
                    if key not in full_cache:         # the full-length transform does not depend on M
                        fp = sq.FullPlan(plan, L, "slicq")
                        full_cache[key] = fp.analyze(f)[:stored] * r
                        if timing is None and two_n == 4096:
                            timing = _full_timing(fp, f.to(torch.complex64), args)
                    full = full_cache[key]
                    c = plan.analyze_complex(f.to(torch.complex64))
                    ls = plan.layers(c[:S * plan.coefs_per_slice], S).to(torch.complex128)
                    snrs.append(20.0 * math.log10(float(torch.linalg.vector_norm(full)) /
                                                  float(torch.linalg.vector_norm(full - ls))))
                table.append({"slice_len": two_n, "transition": two_n // frac, "min_win": mw,
                              "snr_db_mean": round(float(np.mean(snrs)), 2),
                              "snr_db_spread": round(float(np.max(snrs) - np.min(snrs)), 3)})
                print(json.dumps(table[-1]), file=sys.stderr, flush=True)
        full_cache.clear()
    return {"workload": "approximation study (Section 5.3): sliCQ s^0+s^1 (FP32) vs full-length CQ-NSGT (FP64), "
                        "both on the GPU",
            "signals": args.approx_signals, "length": L, "bins_per_octave": 48, "fmin": 200.0,
            "window": "blackman_harris", "seconds": round(time.perf_counter() - t0, 1), "table": table,
            "full_length_fp32": timing}


def _full_timing(fp, x, args):
    """Speed of the full-length transform (FP32) on one signal: analysis
    (algorithmic bytes: the signal read once, the coefficients written once)
    and, on the painless lattice of the same plan, analysis + synthesis."""
    import torch
    import paper_1210_0084_amd as sq
    out = {}
    c = fp.analyze(x)
    ms = _time(lambda: fp.analyze(x, out=c), 10, 3)
    nbytes = 8 * (fp.L + fp.coef_count)
    out["analysis_slicq_lattice"] = {"ms": round(ms, 4), "Msamples_per_s": round(fp.L / ms / 1e3, 1),
                                     "GBs": round(nbytes / ms / 1e6, 1), "coef_count": int(fp.coef_count)}
    pp = sq.FullPlan(fp.plan, fp.L, "painless")
    cp = pp.analyze(x)
    y = pp.synthesize(cp)
    ms = _time(lambda: (pp.analyze(x, out=cp), pp.synthesize(cp, out=y)), 10, 3)
    nbytes = 16 * (pp.L + pp.coef_count)
    out["analysis_synthesis_painless"] = {"ms": round(ms, 4), "Msamples_per_s": round(pp.L / ms / 1e3, 1),
                                          "GBs": round(nbytes / ms / 1e6, 1), "coef_count": int(pp.coef_count),
                                          "reconstruction_rel_err": float(torch.linalg.vector_norm(y - x) /
                                                                          torch.linalg.vector_norm(x))}
    return out


def _bench_smooth(prm, x, y, T, args, copy_gbs):
    """The same c2 step with the smooth-number policy (M_k the smallest even
    2^a, 3 2^a or 5 2^a >= |J_k|): fewer coefficients, mixed-radix band
    kernels. Its own algorithmic bytes (smaller: fewer coefficients)."""
    import torch
    import paper_1210_0084_amd as sq
    plan = sq.Plan(**prm, m_policy="smooth")
    lay = plan.batch_layout([T, T])
    coef = torch.empty(lay.coef_len, dtype=torch.complex64, device=x.device)

    def step():
        plan.analyze_batched(x, out=coef, layout=lay)
        plan.synthesize_batched(coef, out=y, layout=lay)
    ms = _time(step, args.steps, args.warmup)
    err = float((y - x).abs().max().item())
    S = lay.total_slices
    stage_ms = time_stages(plan, S, x, coef, y, args.stage_reps, lay)
    share = algorithmic_share(plan, S, 2 * T, 4)
    path_bytes = 2 * 4 * 2 * T + 2 * 8 * S * plan.coefs_per_slice
    return {"value": round(2 * T / (ms * 1e-3) / 1e6, 1), "unit": "Msamples/s", "ms_per_step": round(ms, 4),
            "coefs_per_slice": plan.coefs_per_slice, "algorithmic_bytes_per_step": path_bytes,
            "path": _frac(path_bytes, ms, copy_gbs), "reconstruction_max_abs_err": err,
            "band_ana": {"ms": round(stage_ms["band_ana"], 4),
                         "algorithmic_GBs": round(share["band_ana"] / (stage_ms["band_ana"] * 1e-3) / 1e9, 1)},
            "band_syn": {"ms": round(stage_ms["band_syn"], 4),
                         "algorithmic_GBs": round(share["band_syn"] / (stage_ms["band_syn"] * 1e-3) / 1e9, 1)}}


def _bench_fp64(args, copy_gbs):
    """The FP64 path on the GPU: the 2^16-sample workload of the CPU baseline
    (B=12, 2N=8192; 16 slices, launch-bound) and the benchmark's 60 s stereo
    in FP64, analysis + synthesis per step, with their FP64 algorithmic bytes."""
    import torch
    import paper_1210_0084_amd as sq
    from workloads import make_c1, make_c2
    dev = torch.device("cuda:0")
    out = {}
    for name, sig in (("c1_2p16", make_c1()[None, :]), ("c2_60s_stereo", make_c2())):
        plan = sq.Plan(**_preset("c1" if name.startswith("c1") else "c2"))
        T = sig.shape[1]
        lay = plan.batch_layout([T] * sig.shape[0])
        x = torch.tensor(sig.reshape(-1), dtype=torch.float64, device=dev)
        coef = torch.empty(lay.coef_len, dtype=torch.complex128, device=dev)
        y = torch.empty_like(x)

        def step():
            plan.analyze_batched(x, out=coef, layout=lay)
            plan.synthesize_batched(coef, out=y, layout=lay)
        ms = _time(step, args.steps, args.warmup)
        nbytes = 2 * 8 * x.numel() + 2 * 16 * lay.total_slices * plan.coefs_per_slice
        out[name] = {"Msamples_per_s": round(x.numel() / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 4),
                     "algorithmic_bytes": nbytes, **_frac(nbytes, ms, copy_gbs),
                     "reconstruction_max_abs_err": float((y - x).abs().max())}
        del x, coef, y
        torch.cuda.empty_cache()
    return out


def _form_summary(rec):
    """The key figures of a form's record, for the default line."""
    keep = {k: rec[k] for k in ("value", "unit", "ms_per_step") if k in rec}
    keep["workload"] = rec["config"]["workload"]
    for k in ("path", "hbm", "compare", "latency_ms", "unpaced", "tuning"):
        if rec.get(k) is not None:
            keep[k] = rec[k]
    return keep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the batched, differentiable and streaming sub-records of the default line")
    ap.add_argument("--graph", action="store_true", help="replay the step's launches as one HIP graph (same speed on c2)")
    ap.add_argument("--stage-reps", type=int, default=20)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (scale for HBM byte counters)")
    ap.add_argument("--workload", choices=["c2", "c3", "c4", "c5", "approx"], default="c2",
                    help="c2 (default): 60 s stereo; c3: ragged batch in a HIP graph; c4: differentiable; "
                         "c5: streaming service; approx: the Section 5.3 approximation study")
    ap.add_argument("--approx-signals", type=int, default=3)
    ap.add_argument("--approx-log2-len", type=int, default=20)
    ap.add_argument("--c3-signals", type=int, default=256)
    ap.add_argument("--no-c3-tune", dest="c3_tune", action="store_false",
                    help="skip the autotuner for the ragged batch (default: tune, cached per batch shape)")
    ap.add_argument("--tune-cache", default=os.path.join(tempfile.gettempdir(), "slicq_tune_cache.json"))
    ap.add_argument("--c4-batch", type=int, default=32)
    ap.add_argument("--fused", action="store_true",
                    help="batched, differentiable and streaming forms with one workgroup per slice where "
                         "the half spectrum fits in LDS (default: the multi-kernel pipeline)")
    ap.add_argument("--c5-streams", type=int, default=512)
    ap.add_argument("--c5-seconds", type=float, default=10.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (slices would shard with a "
              "one-time overlap halo exchange). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    if args.workload != "c2":
        fn = {"c3": bench_batched, "c4": bench_differentiable, "c5": bench_stream, "approx": bench_approx}[args.workload]
        print(json.dumps(fn(args)), flush=True)
        return

    from workloads import PRESETS, make_c2
    xs = make_c2()
    # the oracle's process pool forks before anything touches the GPU
    cpu = None if args.no_cpu_baseline else cpu_baseline(xs)

    import torch
    import paper_1210_0084_amd as sq

    p = PRESETS["c2"]
    prm = dict(fs=p.fs, fmin=p.fmin, fmax=p.fmax, bins_per_octave=p.bins_per_octave, slice_len=p.slice_len,
               transition=p.transition)
    dev = torch.device("cuda:0")
    T = xs.shape[1]
    plan = sq.Plan(**prm)
    lay = plan.batch_layout([T, T])
    x = torch.tensor(xs.reshape(-1), dtype=torch.float32, device=dev)
    coef = torch.empty(lay.coef_len, dtype=torch.complex64, device=dev)
    y = torch.empty(2 * T, dtype=torch.float32, device=dev)

    def eager():
        plan.analyze_batched(x, out=coef, layout=lay)
        plan.synthesize_batched(coef, out=y, layout=lay)

    step = eager
    if args.graph:
        # the step's 12 launches (analysis + synthesis) captured once, replayed as one graph launch
        from paper_1210_0084_amd.tuning import BatchGraph
        step = BatchGraph(plan, x, coef, y, lay).replay

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    err = float((y - x).abs().max().item())
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_host = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host
    ms = e0.elapsed_time(e1) / args.steps
    samples = 2 * T
    value = samples / (ms * 1e-3) / 1e6
    # each step timed on its own (median), and analysis and synthesis apart
    per_step = []
    for _ in range(max(args.steps, 20)):
        a0, a1 = _events()
        a0.record()
        step()
        a1.record()
        torch.cuda.synchronize()
        per_step.append(a0.elapsed_time(a1))
    ms_ana = _time(lambda: plan.analyze_batched(x, out=coef, layout=lay), args.steps, 2)
    ms_syn = _time(lambda: plan.synthesize_batched(coef, out=y, layout=lay), args.steps, 2)
    step()
    torch.cuda.synchronize()

    # per-kernel timing of the pipeline the last step launched (HIP events on the same stream)
    S = lay.total_slices
    if args.graph:
        eager()                             # the stage hooks read the plan's own workspace
        torch.cuda.synchronize()
    stage_ms = time_stages(plan, S, x, coef, y, args.stage_reps, lay)
    sbytes = stage_bytes(plan, S, 4)
    share = algorithmic_share(plan, S, samples, 4)
    copy_gbs = copy_rate()
    stages = {k: {"ms": round(stage_ms[k], 4), "interface_GBs": round(sbytes[k] / (stage_ms[k] * 1e-3) / 1e9, 1),
                  "algorithmic_GBs": round(share[k] / (stage_ms[k] * 1e-3) / 1e9, 1)} for k in STAGES}
    dom = max(STAGES, key=lambda k: stage_ms[k])
    achieved = share[dom] / (stage_ms[dom] * 1e-3) / 1e9
    path_bytes = 2 * 4 * samples + 2 * 8 * S * plan.coefs_per_slice
    rec = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Msamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "60 s stereo 44.1 kHz pink noise + harmonic tones; B=48, 32.7-22050 Hz, "
                               "2N=65536, M=8192; analysis+synthesis" + (" (one HIP graph)" if args.graph else ""),
                   "signals": 2, "samples_per_signal": T, "slices": S, "coefs_per_slice": plan.coefs_per_slice},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
                     "algorithmic_bytes": share[dom], "interface_bytes": sbytes[dom],
                     "kernel_ms": round(stage_ms[dom], 4), "copy_GBs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
        "path": {"algorithmic_bytes_per_step": path_bytes,
                 "GBs": round(path_bytes / (ms * 1e-3) / 1e9, 1),
                 "frac": round(path_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "frac_of_copy": round(path_bytes / (ms * 1e-3) / 1e9 / copy_gbs, 4),
                 "host_wall_ms_per_step": round(t_host * 1e3 / args.steps, 4),
                 "median_ms_per_step": round(float(np.median(per_step)), 4),
                 "analysis_ms": round(ms_ana, 4), "synthesis_ms": round(ms_syn, 4),
                 "reconstruction_max_abs_err": err},
        "stages": stages,
    }
    if not args.no_forms:
        rec["smooth_M"] = _bench_smooth(prm, x, y, T, args, copy_gbs)
        rec["fp64"] = _bench_fp64(args, copy_gbs)
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = 4 * n
        del src, dst
    del x, coef, y
    torch.cuda.empty_cache()
    if not args.no_forms:
        sub = argparse.Namespace(**vars(args))
        sub.steps, sub.warmup, sub.stage_reps = 10, 3, 5
        sub.c5_seconds = min(args.c5_seconds, 6.0)
        forms = {}
        for name, fn in (("batched", bench_batched), ("differentiable", bench_differentiable)):
            forms[name] = _form_summary(fn(sub, copy_gbs))
            torch.cuda.empty_cache()
        forms["streaming"] = _form_summary(bench_stream(sub))
        rec["forms"] = forms
    if cpu is not None:
        rec["cpu_baseline"] = cpu
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
