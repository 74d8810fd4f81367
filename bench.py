"""sliCQ analysis + synthesis throughput on one MI355X.

Workload (default): 60 s of stereo audio at 44.1 kHz (2 x 2,646,000 samples of
seeded pink noise plus harmonic tones), 48 bins per octave from 32.7 Hz to
22.05 kHz, slice length 2N = 65536, Tukey transition 8192, FP32. One step is
the analysis of both channels followed by their synthesis (one batched launch
sequence each); inputs are resident in HBM before the timed region.

Prints one JSON line: Msamples/s of audio (padding excluded), the roofline of
the dominant kernel (algorithmic bytes per launch / HIP-event launch time
against the 8 TB/s HBM peak), per-stage timings, and the FP64 CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
STAGES = ["fwd_pass1", "fwd_pass2", "band_ana", "band_syn", "inv_passA", "inv_passB"]


def stage_bytes(plan, n_slices: int, b: int) -> dict:
    """Algorithmic HBM bytes per launch of each kernel: what its interface must
    read and write once (b = bytes per real value)."""
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


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hpp", "fft_device.hpp", "pipeline.hpp", "common.hpp"):
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


def time_stages(plan, n_slices, x, coef, y, reps=20):
    import torch
    out = {}
    for s, name in enumerate(STAGES):
        plan.profile_stage(s, n_slices, x, coef, y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.profile_stage(s, n_slices, x, coef, y)
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / reps
    return out


def cpu_baseline(prm, xs, seconds_target=15.0):
    """The FP64 oracle (unchanged) on the first slices of the left channel."""
    from oracle import OraclePlan, analyze, synthesize
    opl = OraclePlan(prm["fs"], prm["fmin"], prm["fmax"], prm["bins_per_octave"], prm["slice_len"],
                     prm["transition"])
    T = int(10 * prm["fs"])                 # a 10 s excerpt
    x = xs[0][:T].astype(np.float64)
    t0 = time.perf_counter()
    c = analyze(opl, x)
    y = synthesize(opl, c, T)
    dt = time.perf_counter() - t0
    reps = 1
    while dt * reps < seconds_target and reps < 8:
        t0 = time.perf_counter()
        c = analyze(opl, x)
        y = synthesize(opl, c, T)
        dt = min(dt, time.perf_counter() - t0)
        reps += 1
    err = float(np.abs(y - x).max())
    return {"value": T / dt / 1e6, "unit": "Msamples/s", "cores": 1, "kind": "oracle",
            "sample": f"analysis+synthesis of 10 s ({T} samples) of the left channel, FP64 numpy, "
                      f"best of {reps}; reconstruction max error {err:.1e}"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--stage-reps", type=int, default=20)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (slices would shard with a "
              "one-time overlap halo exchange; see DESIGN.md). Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1210_0084_amd as sq
    from workloads import PRESETS, make_c2

    p = PRESETS["c2"]
    prm = dict(fs=p.fs, fmin=p.fmin, fmax=p.fmax, bins_per_octave=p.bins_per_octave, slice_len=p.slice_len,
               transition=p.transition)
    dev = torch.device("cuda:0")
    xs = make_c2()
    T = xs.shape[1]
    plan = sq.Plan(**prm)
    lay = plan.batch_layout([T, T])
    x = torch.tensor(xs.reshape(-1), dtype=torch.float32, device=dev)
    coef = torch.empty(lay.coef_len, dtype=torch.complex64, device=dev)
    y = torch.empty(2 * T, dtype=torch.float32, device=dev)

    def step():
        plan.analyze_batched(x, out=coef, layout=lay)
        plan.synthesize_batched(coef, out=y, layout=lay)

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

    # per-kernel timing of the pipeline the last step launched (HIP events on the same stream)
    S = lay.total_slices
    stage_ms = time_stages(plan, S, x, coef, y, args.stage_reps)
    sbytes = stage_bytes(plan, S, 4)
    stages = {k: {"ms": round(stage_ms[k], 4), "GBs": round(sbytes[k] / (stage_ms[k] * 1e-3) / 1e9, 1)}
              for k in STAGES}
    dom = max(STAGES, key=lambda k: stage_ms[k])
    achieved = sbytes[dom] / (stage_ms[dom] * 1e-3) / 1e9
    path_bytes = 2 * 4 * samples + 2 * 8 * S * plan.coefs_per_slice
    rec = {
        "metric": "sliCQ analysis+synthesis Msamples/s at 1 GPU, % HBM roofline; p99 slice latency",
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
                               "2N=65536, M=8192; analysis+synthesis",
                   "signals": 2, "samples_per_signal": T, "slices": S, "coefs_per_slice": plan.coefs_per_slice},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(dom), "algorithmic_bytes": sbytes[dom]},
        "path": {"algorithmic_bytes_per_step": path_bytes,
                 "GBs": round(path_bytes / (ms * 1e-3) / 1e9, 1),
                 "frac": round(path_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                 "host_wall_ms_per_step": round(t_host * 1e3 / args.steps, 4),
                 "reconstruction_max_abs_err": err},
        "stages": stages,
    }
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = 4 * n
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(prm, xs)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
