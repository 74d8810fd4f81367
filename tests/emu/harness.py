"""Builds and drives the CPU emulation runner of the library's kernels.

Test infrastructure only: the runner compiles the library's own kernel,
pipeline and plan sources with g++ against a thread-per-lane stand-in for the
HIP runtime (AddressSanitizer and UBSan on), and runs one transform on host
memory.
"""
from __future__ import annotations

import os
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1210_0084_amd", "csrc")
BUILD = os.path.join(HERE, "_build")
EXE = os.path.join(BUILD, "emu_runner")
SOURCES = [os.path.join(HERE, "emu_runner.cpp"), os.path.join(CSRC, "plan.cpp")]
HEADERS = [os.path.join(CSRC, f) for f in ("kernels.hpp", "fft_device.hpp", "fused.hpp", "pipeline.hpp", "plan.hpp",
                                            "common.hpp", "stream_server.hpp", "fullnsgt.hpp", "bandmix.hpp", "coefops.hpp")]
STREAM_EXE = os.path.join(BUILD, "stream_runner")
FULL_EXE = os.path.join(BUILD, "full_runner")


def _stale(exe: str, main_src: str) -> bool:
    deps = [main_src, os.path.join(CSRC, "plan.cpp")] + HEADERS + [os.path.join(HERE, "include", "hip", "hip_runtime.h")]
    return not (os.path.exists(exe) and os.path.getmtime(exe) > max(os.path.getmtime(d) for d in deps))


def _command(exe: str, main_src: str, opt: str):
    tmp = f"{exe}.{os.getpid()}.tmp"       # parallel test workers may build at once
    cmd = ["g++", "-std=c++20", opt, "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
           "-pthread", f"-I{os.path.join(HERE, 'include')}", f"-I{CSRC}", main_src, os.path.join(CSRC, "plan.cpp"),
           "-o", tmp]
    return cmd, tmp


def _build(exe: str, main_src: str, opt: str = "-O1") -> str:
    os.makedirs(BUILD, exist_ok=True)
    if not _stale(exe, main_src):
        return exe
    cmd, tmp = _command(exe, main_src, opt)
    subprocess.check_call(cmd)
    os.replace(tmp, exe)
    return exe


def build_all() -> None:
    """Builds the stale runners side by side (a serial test run then waits for
    the slowest compile only)."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for exe, src, opt in ((EXE, "emu_runner.cpp", "-O1"), (STREAM_EXE, "stream_runner.cpp", "-O0"),
                          (FULL_EXE, "full_runner.cpp", "-O1")):
        src = os.path.join(HERE, src)
        if _stale(exe, src):
            cmd, tmp = _command(exe, src, opt)
            jobs.append((subprocess.Popen(cmd), tmp, exe))
    for proc, tmp, exe in jobs:
        if proc.wait() != 0:
            raise RuntimeError(f"building {exe} failed")
        os.replace(tmp, exe)


def build() -> str:
    return _build(EXE, os.path.join(HERE, "emu_runner.cpp"))


def stream(plan: dict, signals, hop: int, dtype: int = 1, mode: int = 0, max_streams: int = 8,
           max_batch: int = 16, budget: int = 0):
    """Runs the streaming scenario of stream_runner.cpp; returns (outputs, stats)."""
    # the streaming scenarios are tiny: an unoptimised build compiles several times faster
    exe = _build(STREAM_EXE, os.path.join(HERE, "stream_runner.cpp"), "-O0")
    lens = [len(s) for s in signals]
    payload = np.concatenate([[len(signals)], lens] + [np.asarray(s, dtype=np.float64) for s in signals])
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in.bin"), os.path.join(td, "out.bin")
        payload.tofile(fin)
        args = [exe, str(dtype), repr(float(plan["fs"])), repr(float(plan["fmin"])), repr(float(plan["fmax"])),
                str(plan["bins_per_octave"]), str(plan["slice_len"]), str(plan["transition"]),
                repr(float(plan.get("min_win", 16.0))), str(max_streams), str(max_batch), str(budget), str(hop),
                str(mode), fin, fout]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")
        r = subprocess.run(args, capture_output=True, text=True, env=env, timeout=900)
        if r.returncode != 0:
            raise RuntimeError(f"stream_runner failed ({r.returncode}): {r.stderr[-3000:]}")
        out = np.fromfile(fout, dtype=np.float64)
    sel = range(len(signals)) if mode == 0 else [mode - 1]
    ys, pos = [], 0
    for i in sel:
        ys.append(out[pos:pos + lens[i]])
        pos += lens[i]
    return ys, out[pos:pos + 5]


def run(op: str, dtype: int, plan: dict, payload: np.ndarray, chunk: int = 0,
        group_cap: int = 0, lds_cap: int = 0, pass_cap: int = 0, layout: int = 0, fused: int = 0) -> np.ndarray:
    """fused = 1 asks for the one-workgroup-per-slice kernels (the runner fails
    if they do not fit the plan), 0 for the multi-kernel pipeline."""
    exe = build()
    with tempfile.TemporaryDirectory() as td:
        fin = os.path.join(td, "in.bin")
        fout = os.path.join(td, "out.bin")
        np.asarray(payload, dtype=np.float64).tofile(fin)
        args = [exe, op, str(dtype), repr(float(plan["fs"])), repr(float(plan["fmin"])), repr(float(plan["fmax"])),
                str(plan["bins_per_octave"]), str(plan["slice_len"]), str(plan["transition"]),
                repr(float(plan.get("min_win", 16.0))), str(plan.get("dual", 0)), str(group_cap), str(lds_cap),
                str(pass_cap), str(chunk), str(layout), str(int(fused)),
                str({"pow2": 0, "rect": 1, "smooth": 2}[plan.get("m_policy", "pow2")]), fin, fout]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")
        r = subprocess.run(args, capture_output=True, text=True, env=env, timeout=900)
        if r.returncode != 0:
            raise RuntimeError(f"emu_runner failed ({r.returncode}): {r.stderr[-3000:]}")
        return np.fromfile(fout, dtype=np.float64)


def analyze(plan: dict, x: np.ndarray, dtype: int = 1, **kw) -> np.ndarray:
    out = run("ana", dtype, plan, np.concatenate([[len(x)], x]), **kw)
    return out[0::2] + 1j * out[1::2]


def synthesize(plan: dict, coef: np.ndarray, T: int, dtype: int = 1, adjoint: bool = False, **kw) -> np.ndarray:
    c = np.asarray(coef, dtype=np.complex128)
    payload = np.concatenate([[T], np.stack([c.real, c.imag], axis=1).reshape(-1)])
    return run("adj" if adjoint else "syn", dtype, plan, payload, **kw)


def analyze_batched(plan: dict, xs, dtype: int = 1, **kw) -> np.ndarray:
    lens = [len(x) for x in xs]
    payload = np.concatenate([[len(xs)], lens] + [np.asarray(x, dtype=np.float64) for x in xs])
    out = run("bana", dtype, plan, payload, **kw)
    return out[0::2] + 1j * out[1::2]


def synthesize_batched(plan: dict, coef: np.ndarray, lens, dtype: int = 1, adjoint: bool = False, **kw):
    c = np.asarray(coef, dtype=np.complex128)
    payload = np.concatenate([[len(lens)], lens, np.stack([c.real, c.imag], axis=1).reshape(-1)])
    return run("badj" if adjoint else "bsyn", dtype, plan, payload, **kw)


def full(op: str, plan: dict, L: int, lattice: int, data, dtype: int = 1, window: int = 0):
    """Full-length analysis (op "ana", data: L complex values) or synthesis
    (op "syn", data: the coefficients) through full_runner.cpp."""
    exe = _build(FULL_EXE, os.path.join(HERE, "full_runner.cpp"))
    data = np.asarray(data, dtype=np.complex128)
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in.bin"), os.path.join(td, "out.bin")
        data.view(np.float64).tofile(fin)
        args = [exe, op, str(dtype), repr(float(plan["fs"])), repr(float(plan["fmin"])), repr(float(plan["fmax"])),
                str(plan["bins_per_octave"]), str(plan["slice_len"]), str(plan["transition"]),
                repr(float(plan.get("min_win", 16.0))), str(window), str(L), str(lattice), fin, fout]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")
        r = subprocess.run(args, capture_output=True, text=True, env=env, timeout=900)
        if r.returncode != 0:
            raise RuntimeError(f"full_runner failed ({r.returncode}): {r.stderr[-3000:]}")
        return np.fromfile(fout, dtype=np.float64).view(np.complex128)
