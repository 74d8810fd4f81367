"""MI355X sliCQ: Python binding of ``libslicq.so`` (include/slicq.h).

Argument marshalling only: every step of the transform runs in the HIP
kernels of the library. PyTorch provides device memory and the HIP stream
(``torch.cuda.current_stream().cuda_stream``). The binding fails loudly when
the library is missing; there is no other implementation behind it.

    plan = Plan(44100, 32.7, 22050, 48, 65536, 8192)
    c = plan.analyze(x)                 # x: (T,) float32/float64 on cuda
    y = plan.synthesize(c, T)           # perfect reconstruction
    cb = plan.band(c, k, plan.num_slices(T))   # (S, M_k) view of band k
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

__all__ = ["Plan", "SliCQFunction", "SliCQSynthesisFunction", "slicq", "islicq", "library_path", "SlicqError",
           "SlicqBusy", "StreamServer", "load_library"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libslicq.so")
_lib = None

F32, F64 = 0, 1


class SlicqError(RuntimeError):
    pass


class SlicqBusy(SlicqError):
    """Admission refused: no stream slot within the server's memory budget."""


class _StreamStats(ctypes.Structure):
    _fields_ = [("ticks", ctypes.c_int64), ("slices", ctypes.c_int64), ("samples_in", ctypes.c_int64),
                ("samples_out", ctypes.c_int64), ("admitted", ctypes.c_int64), ("rejected", ctypes.c_int64),
                ("closed", ctypes.c_int64), ("gap_samples", ctypes.c_int64), ("latency_p50_s", ctypes.c_double),
                ("latency_p99_s", ctypes.c_double), ("latency_max_s", ctypes.c_double),
                ("latency_count", ctypes.c_int64), ("busy_s", ctypes.c_double), ("slots", ctypes.c_int32),
                ("pad_", ctypes.c_int32), ("ring_len", ctypes.c_int64), ("bytes_per_stream", ctypes.c_int64),
                ("fixed_bytes", ctypes.c_int64)]


class _Opts(ctypes.Structure):
    _fields_ = [("fs", ctypes.c_double), ("fmin", ctypes.c_double), ("fmax", ctypes.c_double),
                ("bins_per_octave", ctypes.c_int32), ("slice_len", ctypes.c_int64),
                ("transition_len", ctypes.c_int64), ("min_win", ctypes.c_double),
                ("dual_slice", ctypes.c_int32), ("group_cap", ctypes.c_int32),
                ("lds_cap", ctypes.c_int32), ("pass_cap", ctypes.c_int32), ("coef_layout", ctypes.c_int32),
                ("window", ctypes.c_int32), ("scale", ctypes.c_int32), ("slicing", ctypes.c_int32),
                ("m_policy", ctypes.c_int32), ("fused", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("nbands", ctypes.c_int32), ("slice_len", ctypes.c_int64),
                ("transition_len", ctypes.c_int64), ("coefs_per_slice", ctypes.c_int64),
                ("Q", ctypes.c_double), ("max_M", ctypes.c_int32), ("n_ana_items", ctypes.c_int32),
                ("n_syn_items", ctypes.c_int32), ("coef_layout", ctypes.c_int32), ("fused", ctypes.c_int32),
                ("coefs_per_slice_all", ctypes.c_int64)]


class _FullInfo(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int64), ("nbands", ctypes.c_int32), ("lattice", ctypes.c_int32),
                ("painless", ctypes.c_int32), ("pad_", ctypes.c_int32), ("coef_count", ctypes.c_int64),
                ("max_M", ctypes.c_int64), ("entries", ctypes.c_int64)]


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Loads libslicq.so (built in-tree by ``python -m paper_1210_0084_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise SlicqError(f"{_LIB_PATH} is missing: build it with `python -m paper_1210_0084_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    P, I32, I64, D, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "nsgt_plan": (ctypes.c_int, [D, D, D, ctypes.c_int, I64, I64, ctypes.POINTER(P)]),
        "nsgt_plan_ex": (ctypes.c_int, [ctypes.POINTER(_Opts), ctypes.POINTER(P)]),
        "nsgt_plan_destroy": (None, [P]),
        "nsgt_plan_info": (ctypes.c_int, [P, ctypes.POINTER(_Info)]),
        "nsgt_plan_bands": (ctypes.c_int, [P, P, P, P, P, P, P]),
        "nsgt_plan_windows": (ctypes.c_int, [P, P, P, P, P, P]),
        "nsgt_plan_table_bytes": (ctypes.c_int, [P, ctypes.c_int, ctypes.POINTER(SZ)]),
        "nsgt_plan_upload": (ctypes.c_int, [P, ctypes.c_int, P, SZ, P]),
        "slicq_num_slices": (I64, [P, I64]),
        "slicq_workspace_size": (ctypes.c_int, [P, ctypes.c_int, I64, ctypes.POINTER(SZ)]),
        "slicq_analyze": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I64, P, SZ, P]),
        "slicq_analyze_static": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I64, P]),
        "slicq_static_scratch_bytes": (SZ, []),
        "slicq_synthesize": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I64, P, SZ, P]),
        "slicq_adjoint": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I64, P, SZ, P]),
        "slicq_analyze_batched": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I32, I64, P, I64, P, P, SZ, P]),
        "slicq_synthesize_batched": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, P, I64, P, I32, I64, P, SZ, P]),
        "slicq_adjoint_batched": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, P, I64, P, I32, I64, P, SZ, P]),
        "slicq_profile_stage": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, I64, P, P, P, P, SZ, P]),
        "slicq_synthesize_adjoint": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I64, P, SZ, P]),
        "slicq_complex_workspace_size": (ctypes.c_int, [P, ctypes.c_int, I64, ctypes.POINTER(SZ)]),
        "slicq_analyze_complex": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I64, P, SZ, P]),
        "slicq_synthesize_complex": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I64, P, SZ, P]),
        "slicq_layers": (ctypes.c_int, [P, ctypes.c_int, P, I64, ctypes.c_int, P, I64, P]),
        "slicq_mask_db": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I64, P]),
        "slicq_transpose": (ctypes.c_int, [P, ctypes.c_int, P, P, I64, I32, P]),
        "slicq_logmag_loss_partials": (I64, [I64]),
        "slicq_logmag_loss": (ctypes.c_int, [ctypes.c_int, P, P, I64, P, P, I64, P, P]),
        "slicq_batched_status": (ctypes.c_int, [P, ctypes.c_int, I64, P, SZ, ctypes.POINTER(I32),
                                                ctypes.POINTER(I64), P]),
        "slicq_batch_tasks_bytes": (SZ, [I64]),
        "slicq_profile_stage_batch": (ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, P, I64, P, I64, P, I64, P, SZ, P]),
        "slicq_batch_create": (ctypes.c_int, [P, P, P, I32, I64, I64, I64, P, SZ, P, ctypes.POINTER(P)]),
        "slicq_batch_destroy": (None, [P]),
        "slicq_analyze_batch": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I64, P, SZ, P]),
        "slicq_synthesize_batch": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I64, P, SZ, P]),
        "slicq_adjoint_batch": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, I64, P, SZ, P]),
        "slicq_stream_server_create": (ctypes.c_int, [P, ctypes.c_int, I32, I32, SZ, ctypes.POINTER(P)]),
        "slicq_stream_server_destroy": (None, [P]),
        "slicq_stream_open": (ctypes.c_int, [P, ctypes.POINTER(I32)]),
        "slicq_stream_push": (ctypes.c_int, [P, I32, P, I64]),
        "slicq_stream_push_gap": (ctypes.c_int, [P, I32, I64]),
        "slicq_stream_push_many": (ctypes.c_int, [P, I32, P, P, P]),
        "slicq_stream_poll_many": (ctypes.c_int, [P, I32, P, P, I64, P]),
        "slicq_stream_tick": (ctypes.c_int, [P, ctypes.POINTER(I64)]),
        "slicq_stream_poll": (ctypes.c_int, [P, I32, P, I64, ctypes.POINTER(I64)]),
        "slicq_stream_close": (ctypes.c_int, [P, I32]),
        "slicq_stream_coefs": (ctypes.c_int, [P, I32, P, I64, ctypes.POINTER(I64)]),
        "slicq_stream_stats_get": (ctypes.c_int, [P, ctypes.POINTER(_StreamStats)]),
        "slicq_stream_stats_reset": (ctypes.c_int, [P]),
        "slicq_stream_snapshot": (ctypes.c_int, [P, I32, P, SZ, ctypes.POINTER(SZ)]),
        "slicq_stream_restore": (ctypes.c_int, [P, I32, P, SZ]),
        "nsgt_full_plan": (ctypes.c_int, [P, I64, I32, ctypes.POINTER(P)]),
        "nsgt_full_destroy": (None, [P]),
        "nsgt_full_info": (ctypes.c_int, [P, ctypes.POINTER(_FullInfo)]),
        "nsgt_full_bands": (ctypes.c_int, [P, P, P, P, P]),
        "nsgt_full_windows": (ctypes.c_int, [P, P, P]),
        "nsgt_full_table_bytes": (ctypes.c_int, [P, ctypes.c_int, ctypes.POINTER(SZ)]),
        "nsgt_full_upload": (ctypes.c_int, [P, ctypes.c_int, P, SZ, P]),
        "nsgt_full_workspace_size": (ctypes.c_int, [P, ctypes.c_int, ctypes.POINTER(SZ)]),
        "nsgt_full_analyze": (ctypes.c_int, [P, ctypes.c_int, P, P, I64, P, SZ, P]),
        "nsgt_full_synthesize": (ctypes.c_int, [P, ctypes.c_int, P, I64, P, P, SZ, P]),
        "slicq_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        msg = load_library().slicq_last_error().decode(errors="replace")
        raise (SlicqBusy if rc == -5 else SlicqError)(f"slicq error {rc}: {msg}")


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype in (torch.float32, torch.complex64):
        return F32
    if t.dtype in (torch.float64, torch.complex128):
        return F64
    raise SlicqError(f"unsupported dtype {t.dtype}: use float32 or float64")


def _stream_ptr(dev) -> int:
    torch = _torch()
    return torch.cuda.current_stream(dev).cuda_stream


def _require_cuda(t, name):
    if not t.is_cuda:
        raise SlicqError(f"{name} must be a HIP device tensor (got {t.device})")
    if not t.is_contiguous():
        raise SlicqError(f"{name} must be contiguous")


class BatchLayout:
    """Offsets of a ragged batch packed back to back (host and cached device copies)."""

    def __init__(self, plan, lengths):
        lengths = np.asarray(lengths, dtype=np.int64)
        self.lengths = lengths
        self.x_off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
        S = np.array([plan.num_slices(int(t)) for t in lengths], dtype=np.int64)
        self.slices = S
        c_sz = S * plan.coefs_per_slice
        self.coef_off = (np.concatenate([[0], np.cumsum(c_sz)[:-1]]).astype(np.int64) if len(lengths)
                         else np.zeros(0, dtype=np.int64))
        self.total_slices = int(S.sum())
        self.coef_len = int(c_sz.sum())
        self._dev = {}
        self._plan = plan          # a prepared task table is only valid for this plan

    @property
    def nsig(self) -> int:
        return len(self.lengths)

    def device(self, dev):
        key = str(dev)
        if key not in self._dev:
            torch = _torch()
            self._dev[key] = (torch.as_tensor(self.x_off, device=dev), torch.as_tensor(self.coef_off, device=dev))
        return self._dev[key]

    def prepared(self, plan, dev):
        """Handle of this batch's slice task table on dev (built once, on the current stream)."""
        key = ("tasks", str(dev))
        if key not in self._dev:
            torch = _torch()
            lib = plan._lib
            d_xoff, d_coff = self.device(dev)
            nb = lib.slicq_batch_tasks_bytes(self.total_slices)
            tasks = torch.empty(max(int(nb), 1), dtype=torch.uint8, device=dev)
            h = ctypes.c_void_p()
            _check(lib.slicq_batch_create(plan._h, ctypes.c_void_p(d_xoff.data_ptr()),
                                          ctypes.c_void_p(d_coff.data_ptr()), self.nsig, self.total_slices,
                                          int(self.x_off[-1]), self.coef_len, ctypes.c_void_p(tasks.data_ptr()),
                                          tasks.numel(), ctypes.c_void_p(_stream_ptr(dev)), ctypes.byref(h)))
            self._dev[key] = (tasks, _BatchHandle(lib, h))
        return self._dev[key][1].h

    @property
    def is_preparable(self) -> bool:
        return self.nsig > 0 and self.total_slices > 0


class _BatchHandle:
    def __init__(self, lib, h):
        self.lib, self.h = lib, h

    def __del__(self):
        if self.h is not None and self.h.value:
            self.lib.slicq_batch_destroy(self.h)
            self.h = None


class Plan:
    """A sliCQ plan (Section 3, Table 1; Section 4.3) with its device tables.

    Parameters follow the paper: sampling rate ``fs`` (xi_s), ``fmin``/``fmax``
    (xi_min, xi_max), ``bins_per_octave`` (B), ``slice_len`` (2N) and
    ``transition`` (M of the Tukey slicing window).
    """

    def __init__(self, fs: float, fmin: float, fmax: float, bins_per_octave: int, slice_len: int,
                 transition: int, min_win: float = 16.0, dual_slice: str = "canonical",
                 group_cap: int = 0, lds_cap: int = 0, pass_cap: int = 0, layout: str = "band",
                 fused: bool = False, window: str = "hann", scale: str = "cq", slicing: str = "tukey",
                 m_policy: str = "pow2"):
        lib = load_library()
        o = _Opts(float(fs), float(fmin), float(fmax), int(bins_per_octave), int(slice_len), int(transition),
                  float(min_win), {"canonical": 0, "indicator": 1}[dual_slice], int(group_cap), int(lds_cap),
                  int(pass_cap), {"band": 0, "slice": 1}[layout],
                  {"hann": 0, "blackman_harris": 1}[window], {"cq": 0, "mel": 1, "bark": 2}[scale],
                  {"tukey": 0, "sqrt_tukey": 1}[slicing], {"pow2": 0, "rect": 1, "smooth": 2}[m_policy], 1 if fused else 0)
        h = ctypes.c_void_p()
        _check(lib.nsgt_plan_ex(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._lib = lib
        info = _Info()
        _check(lib.nsgt_plan_info(h, ctypes.byref(info)))
        self.K = info.K
        self.nbands = info.nbands
        self.slice_len = info.slice_len
        self.N = info.slice_len // 2
        self.transition = info.transition_len
        self.coefs_per_slice = info.coefs_per_slice
        self.Q = info.Q
        self.max_M = info.max_M
        self.n_ana_items = info.n_ana_items
        self.n_syn_items = info.n_syn_items
        self.layout = "slice" if info.coef_layout == 1 else "band"
        self.fused_dtypes = {d for d, bit in ((F32, 1), (F64, 2)) if info.fused & bit}
        self.coefs_per_slice_all = info.coefs_per_slice_all
        self.fs, self.fmin, self.fmax, self.bins_per_octave = float(fs), float(fmin), float(fmax), int(bins_per_octave)
        nb = self.nbands
        self.M = np.zeros(nb, dtype=np.int32)
        self.offsets = np.zeros(nb, dtype=np.int64)
        self.starts = np.zeros(nb, dtype=np.int64)
        self.lengths = np.zeros(nb, dtype=np.int32)
        self.fc = np.zeros(nb)
        self.bw = np.zeros(nb)
        _check(lib.nsgt_plan_bands(h, self.M.ctypes.data, self.offsets.ctypes.data, self.starts.ctypes.data,
                                   self.lengths.ctypes.data, self.fc.ctypes.data, self.bw.ctypes.data))
        self._tables = {}
        self._work = {}
        self._tasks_in = {}       # (dtype, device) -> slices whose task table the internal workspace holds

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.nsgt_plan_destroy(h)
            self._h = None

    # -- host tables -------------------------------------------------------
    def windows(self):
        """FP64 host tables: (g, gd, h0, hd, D) as numpy arrays."""
        tot = int(self.lengths.sum())
        g, gd = np.zeros(tot), np.zeros(tot)
        h0, hd, D = np.zeros(self.slice_len), np.zeros(self.slice_len), np.zeros(self.slice_len)
        _check(self._lib.nsgt_plan_windows(self._h, g.ctypes.data, gd.ctypes.data, h0.ctypes.data,
                                           hd.ctypes.data, D.ctypes.data))
        return g, gd, h0, hd, D

    # -- device state --------------------------------------------------------
    def _ensure_tables(self, dt: int, device):
        torch = _torch()
        key = (dt, str(device))
        if key in self._tables:
            return
        nbytes = ctypes.c_size_t()
        _check(self._lib.nsgt_plan_table_bytes(self._h, dt, ctypes.byref(nbytes)))
        buf = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        off = (-buf.data_ptr()) % 256
        _check(self._lib.nsgt_plan_upload(self._h, dt, ctypes.c_void_p(buf.data_ptr() + off), nbytes.value,
                                          ctypes.c_void_p(_stream_ptr(device))))
        self._tables[key] = buf

    def workspace_bytes(self, dt: int, n_slices: int) -> int:
        b = ctypes.c_size_t()
        _check(self._lib.slicq_workspace_size(self._h, dt, int(n_slices), ctypes.byref(b)))
        return b.value

    def _workspace(self, dt: int, n_slices: int, device, work=None):
        torch = _torch()
        need = self.workspace_bytes(dt, n_slices)
        if work is not None:
            return work, work.numel() * work.element_size()
        key = (dt, str(device))
        w = self._work.get(key)
        if w is None or w.numel() < need:
            w = torch.empty(need, dtype=torch.uint8, device=device)
            self._work[key] = w
            self._tasks_in.pop(key, None)
        return w, w.numel()

    # -- shapes -------------------------------------------------------------
    def num_slices(self, T: int) -> int:
        return int(self._lib.slicq_num_slices(self._h, int(T)))

    def coef_count(self, T: int) -> int:
        return self.num_slices(T) * self.coefs_per_slice

    def band(self, coef, k: int, S: int):
        """Band k of one signal's coefficient vector as an (S, M_k) view."""
        Mk, off = int(self.M[k]), int(self.offsets[k])
        if self.layout == "slice":
            return coef[:S * self.coefs_per_slice].view(S, self.coefs_per_slice)[:, off:off + Mk]
        return coef[off * S:off * S + S * Mk].view(S, Mk)

    def to_band_major(self, coef, S: int):
        """Band-major copy of one signal's coefficients (identity for band-major plans)."""
        if self.layout == "band":
            return coef
        import torch
        return torch.cat([self.band(coef, k, S).reshape(-1) for k in range(self.nbands)])

    # -- transforms ---------------------------------------------------------
    def analyze(self, x, out=None, work=None):
        """Coefficients of the real signal x (Algorithm 3), band-major complex vector."""
        torch = _torch()
        _require_cuda(x, "x")
        if x.dim() != 1:
            raise SlicqError("x must be 1-D; use analyze_batched for several signals")
        dt = _dtype_code(x)
        T = x.numel()
        S = self.num_slices(T)
        ctype = torch.complex64 if dt == F32 else torch.complex128
        if out is None:
            out = torch.empty(S * self.coefs_per_slice, dtype=ctype, device=x.device)
        _require_cuda(out, "out")
        self._ensure_tables(dt, x.device)
        w, wb = self._workspace(dt, S, x.device, work)
        _check(self._lib.slicq_analyze(self._h, dt, ctypes.c_void_p(x.data_ptr()), T,
                                       ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.c_void_p(w.data_ptr()),
                                       wb, ctypes.c_void_p(_stream_ptr(x.device))))
        self._note_tasks(dt, x.device, S, work)
        return out

    def analyze_static(self, x, out):
        """``analyze`` into the caller's ``out`` with the library's fixed device
        scratch instead of a workspace: the call allocates nothing (for graph
        capture and serving loops). Calls on one device must not overlap."""
        _require_cuda(x, "x")
        _require_cuda(out, "out")
        if x.dim() != 1:
            raise SlicqError("x must be 1-D")
        dt = _dtype_code(x)
        if _dtype_code(out) != dt or not out.is_complex():
            raise SlicqError("out must be the complex dtype matching x")
        if (dt, str(x.device)) not in self._tables:
            raise SlicqError("upload the plan's tables first (one analyze call, or _ensure_tables)")
        _check(self._lib.slicq_analyze_static(self._h, dt, ctypes.c_void_p(x.data_ptr()), x.numel(),
                                              ctypes.c_void_p(out.data_ptr()), out.numel(),
                                              ctypes.c_void_p(_stream_ptr(x.device))))
        return out

    def _note_tasks(self, dt, device, n, work):
        if work is None:
            self._tasks_in[(dt, str(device))] = int(n)

    def _synth(self, coef, T, adjoint, out, work):
        torch = _torch()
        _require_cuda(coef, "coef")
        dt = _dtype_code(coef)
        rtype = torch.float32 if dt == F32 else torch.float64
        S = self.num_slices(T)
        if out is None:
            out = torch.empty(int(T), dtype=rtype, device=coef.device)
        _require_cuda(out, "out")
        self._ensure_tables(dt, coef.device)
        w, wb = self._workspace(dt, S, coef.device, work)
        fn = self._lib.slicq_adjoint if adjoint else self._lib.slicq_synthesize
        _check(fn(self._h, dt, ctypes.c_void_p(coef.data_ptr()), coef.numel(), ctypes.c_void_p(out.data_ptr()),
                  int(T), ctypes.c_void_p(w.data_ptr()), wb, ctypes.c_void_p(_stream_ptr(coef.device))))
        self._note_tasks(dt, coef.device, S, work)
        return out

    def synthesize(self, coef, T: int, out=None, work=None):
        """Reconstruction from band-major coefficients (Algorithm 4, canonical duals)."""
        return self._synth(coef, T, False, out, work)

    def adjoint(self, coef, T: int, out=None, work=None):
        """Re(A^H coef): the transpose of ``analyze`` for the real inner product."""
        return self._synth(coef, T, True, out, work)

    def synthesize_adjoint(self, y, out=None, work=None):
        """Adjoint of ``synthesize`` (coefficient gradient of a loss of the
        synthesised signal): the analysis of y with the dual windows."""
        torch = _torch()
        _require_cuda(y, "y")
        dt = _dtype_code(y)
        T = y.numel()
        S = self.num_slices(T)
        if out is None:
            out = torch.empty(S * self.coefs_per_slice, dtype=torch.complex64 if dt == F32 else torch.complex128,
                              device=y.device)
        _require_cuda(out, "out")
        self._ensure_tables(dt, y.device)
        w, wb = self._workspace(dt, S, y.device, work)
        _check(self._lib.slicq_synthesize_adjoint(self._h, dt, ctypes.c_void_p(y.data_ptr()), T,
                                                  ctypes.c_void_p(out.data_ptr()), out.numel(),
                                                  ctypes.c_void_p(w.data_ptr()), wb,
                                                  ctypes.c_void_p(_stream_ptr(y.device))))
        self._note_tasks(dt, y.device, S, work)
        return out

    # -- complex signals ------------------------------------------------------
    def _complex_work(self, dt, T, device):
        torch = _torch()
        b = ctypes.c_size_t()
        _check(self._lib.slicq_complex_workspace_size(self._h, dt, int(T), ctypes.byref(b)))
        key = ("complex", dt, str(device))
        w = self._work.get(key)
        if w is None or w.numel() < b.value:
            w = torch.empty(max(b.value, 1), dtype=torch.uint8, device=device)
            self._work[key] = w
        return w

    def analyze_complex(self, x, out=None):
        """Coefficients of a complex signal on all 2K+2 bands (stored bands,
        then the mirrors K+2..2K+1), band-major."""
        torch = _torch()
        _require_cuda(x, "x")
        if not x.is_complex():
            raise SlicqError("x must be complex")
        dt = _dtype_code(x)
        T = x.numel()
        S = self.num_slices(T)
        if out is None:
            out = torch.empty(S * self.coefs_per_slice_all, dtype=x.dtype, device=x.device)
        self._ensure_tables(dt, x.device)
        w = self._complex_work(dt, T, x.device)
        _check(self._lib.slicq_analyze_complex(self._h, dt, ctypes.c_void_p(x.data_ptr()), T,
                                               ctypes.c_void_p(out.data_ptr()), out.numel(),
                                               ctypes.c_void_p(w.data_ptr()), w.numel(),
                                               ctypes.c_void_p(_stream_ptr(x.device))))
        return out

    def synthesize_complex(self, coef, T: int, out=None):
        """Complex signal of T samples from coefficients on all 2K+2 bands."""
        torch = _torch()
        _require_cuda(coef, "coef")
        dt = _dtype_code(coef)
        if out is None:
            out = torch.empty(int(T), dtype=coef.dtype, device=coef.device)
        self._ensure_tables(dt, coef.device)
        w = self._complex_work(dt, T, coef.device)
        _check(self._lib.slicq_synthesize_complex(self._h, dt, ctypes.c_void_p(coef.data_ptr()), coef.numel(),
                                                  ctypes.c_void_p(out.data_ptr()), int(T),
                                                  ctypes.c_void_p(w.data_ptr()), w.numel(),
                                                  ctypes.c_void_p(_stream_ptr(coef.device))))
        return out

    # -- coefficient domain (2-layer array, spectrogram, masks, transposition) --
    def layer_views(self, coef, k: int, S: int):
        """Zero-copy (S/2, M_k) views of band k's even and odd slices (band-major
        plans): layer 1 is the odd slices in order; layer 0 is the even slices,
        whose flattened layer position is the view's flat index minus M_k / 2
        (circularly), as Algorithm 3 places them."""
        b = self.band(coef, k, S)
        return b[0::2], b[1::2]

    def layers(self, coef, S: int, spectrogram: bool = False, out=None):
        """s^0 + s^1 (complex) or the sliCQ spectrogram |s^0 + s^1|^2 (real)
        on the layer grid, band k's S M_k / 2 values at (S / 2) off_k."""
        torch = _torch()
        _require_cuda(coef, "coef")
        dt = _dtype_code(coef)
        n = (S // 2) * self.coefs_per_slice
        if out is None:
            rt = (torch.float32 if dt == F32 else torch.float64) if spectrogram else coef.dtype
            out = torch.empty(max(n, 1), dtype=rt, device=coef.device)
        self._ensure_tables(dt, coef.device)
        _check(self._lib.slicq_layers(self._h, dt, ctypes.c_void_p(coef.data_ptr()), int(S), 1 if spectrogram else 0,
                                      ctypes.c_void_p(out.data_ptr()), out.numel(),
                                      ctypes.c_void_p(_stream_ptr(coef.device))))
        return out

    def layer_band(self, grid, k: int, S: int):
        """Band k's S M_k / 2 values of a layer-grid array."""
        off, Mk = int(self.offsets[k]), int(self.M[k])
        return grid[(S // 2) * off:(S // 2) * (off + Mk)]

    def mask_db(self, coef, S: int, mask):
        """In place: coef scaled by 10^{5 (v - 1)} of the mask value v of its
        layer position (mask on the layer grid, values in [0, 1])."""
        _require_cuda(coef, "coef")
        _require_cuda(mask, "mask")
        dt = _dtype_code(coef)
        self._ensure_tables(dt, coef.device)
        _check(self._lib.slicq_mask_db(self._h, dt, ctypes.c_void_p(coef.data_ptr()), int(S),
                                       ctypes.c_void_p(mask.data_ptr()), mask.numel(),
                                       ctypes.c_void_p(_stream_ptr(coef.device))))
        return coef

    def transpose(self, coef, S: int, d: int, out=None):
        """Constant-Q bands moved up by d (8 bands = 2 semitones at 48 per octave)."""
        torch = _torch()
        _require_cuda(coef, "coef")
        dt = _dtype_code(coef)
        if out is None:
            out = torch.empty_like(coef)
        self._ensure_tables(dt, coef.device)
        _check(self._lib.slicq_transpose(self._h, dt, ctypes.c_void_p(coef.data_ptr()),
                                         ctypes.c_void_p(out.data_ptr()), int(S), int(d),
                                         ctypes.c_void_p(_stream_ptr(coef.device))))
        return out

    # -- ragged batches -----------------------------------------------------
    def batch_layout(self, lengths: Sequence[int]) -> BatchLayout:
        """Offsets for a ragged batch; pass it back to the batched calls to reuse it."""
        return BatchLayout(self, lengths)

    def _uniform_layout(self, B: int, T: int) -> BatchLayout:
        """Cached layout of B signals of T samples (the autograd path reuses it every step)."""
        cache = self.__dict__.setdefault("_layouts", {})
        lay = cache.get((B, T))
        if lay is None:
            if len(cache) >= 16:
                cache.clear()
            lay = cache[(B, T)] = BatchLayout(self, [T] * B)
        return lay

    def analyze_batched(self, x_packed, lengths=None, out=None, work=None, layout: Optional[BatchLayout] = None):
        """Analysis of a ragged batch packed back to back in x_packed; one launch per kernel."""
        torch = _torch()
        _require_cuda(x_packed, "x_packed")
        dt = _dtype_code(x_packed)
        lay = layout if layout is not None else self.batch_layout(lengths)
        ctype = torch.complex64 if dt == F32 else torch.complex128
        if out is None:
            out = torch.empty(max(lay.coef_len, 1), dtype=ctype, device=x_packed.device)
        _require_cuda(out, "out")
        self._ensure_tables(dt, x_packed.device)
        w, wb = self._workspace(dt, lay.total_slices, x_packed.device, work)
        if layout is not None and lay.is_preparable and lay._plan is self:
            # the task table of a reused layout is built once (slicq_batch_create)
            _check(self._lib.slicq_analyze_batch(
                lay.prepared(self, x_packed.device), dt, ctypes.c_void_p(x_packed.data_ptr()), x_packed.numel(),
                ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.c_void_p(w.data_ptr()), wb,
                ctypes.c_void_p(_stream_ptr(x_packed.device))))
            return out
        d_xoff, d_coff = lay.device(x_packed.device)
        _check(self._lib.slicq_analyze_batched(
            self._h, dt, ctypes.c_void_p(x_packed.data_ptr()), x_packed.numel(), ctypes.c_void_p(d_xoff.data_ptr()),
            lay.nsig, lay.total_slices, ctypes.c_void_p(out.data_ptr()), out.numel(),
            ctypes.c_void_p(d_coff.data_ptr()), ctypes.c_void_p(w.data_ptr()), wb,
            ctypes.c_void_p(_stream_ptr(x_packed.device))))
        self._note_tasks(dt, x_packed.device, lay.total_slices, work)
        return out

    def synthesize_batched(self, coef, lengths=None, out=None, work=None, layout: Optional[BatchLayout] = None,
                           adjoint: bool = False):
        """Synthesis (or adjoint) of a ragged batch; outputs packed like the inputs."""
        torch = _torch()
        _require_cuda(coef, "coef")
        dt = _dtype_code(coef)
        lay = layout if layout is not None else self.batch_layout(lengths)
        rtype = torch.float32 if dt == F32 else torch.float64
        if out is None:
            out = torch.empty(max(int(lay.x_off[-1]), 1), dtype=rtype, device=coef.device)
        _require_cuda(out, "out")
        self._ensure_tables(dt, coef.device)
        w, wb = self._workspace(dt, lay.total_slices, coef.device, work)
        if layout is not None and lay.is_preparable and lay._plan is self:
            fn = self._lib.slicq_adjoint_batch if adjoint else self._lib.slicq_synthesize_batch
            _check(fn(lay.prepared(self, coef.device), dt, ctypes.c_void_p(coef.data_ptr()), coef.numel(),
                      ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.c_void_p(w.data_ptr()), wb,
                      ctypes.c_void_p(_stream_ptr(coef.device))))
            return out
        d_xoff, d_coff = lay.device(coef.device)
        fn = self._lib.slicq_adjoint_batched if adjoint else self._lib.slicq_synthesize_batched
        _check(fn(self._h, dt, ctypes.c_void_p(coef.data_ptr()), coef.numel(), ctypes.c_void_p(d_coff.data_ptr()),
                  ctypes.c_void_p(out.data_ptr()), out.numel(), ctypes.c_void_p(d_xoff.data_ptr()), lay.nsig,
                  lay.total_slices, ctypes.c_void_p(w.data_ptr()), wb, ctypes.c_void_p(_stream_ptr(coef.device))))
        self._note_tasks(dt, coef.device, lay.total_slices, work)
        return out

    def batched_status(self, dt: int, n_slices: int, device, work=None) -> int:
        """Slice count the last batched call's task builder found in the
        workspace; raises SlicqError if that call skipped a signal whose
        ranges fell outside its buffers. Waits for the current stream."""
        w, wb = self._workspace(dt, n_slices, device, work)
        bad, n = ctypes.c_int32(), ctypes.c_int64()
        _check(self._lib.slicq_batched_status(self._h, dt, int(n_slices), ctypes.c_void_p(w.data_ptr()), wb,
                                              ctypes.byref(bad), ctypes.byref(n),
                                              ctypes.c_void_p(_stream_ptr(device))))
        return n.value

    def profile_stage(self, stage: int, n_slices: int, x, coef, y, work=None, layout: Optional[BatchLayout] = None):
        """Enqueues one kernel of the preceding call's pipeline (measurement hook). Pass the
        layout if the preceding call was a batched call with a reused layout."""
        dt = _dtype_code(x)
        w, wb = self._workspace(dt, n_slices, x.device, work)
        if layout is not None and layout.is_preparable and layout._plan is self:
            _check(self._lib.slicq_profile_stage_batch(
                layout.prepared(self, x.device), dt, int(stage), ctypes.c_void_p(x.data_ptr()), x.numel(),
                ctypes.c_void_p(coef.data_ptr()), coef.numel(), ctypes.c_void_p(y.data_ptr()), y.numel(),
                ctypes.c_void_p(w.data_ptr()), wb, ctypes.c_void_p(_stream_ptr(x.device))))
            return
        if work is None and self._tasks_in.get((dt, str(x.device)), -1) != int(n_slices):
            raise SlicqError("profile_stage: the workspace does not hold the task table of a preceding call over "
                             f"{n_slices} slices (pass the layout of a prepared batch)")
        _check(self._lib.slicq_profile_stage(self._h, dt, int(stage), int(n_slices), ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(coef.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                             ctypes.c_void_p(w.data_ptr()), wb,
                                             ctypes.c_void_p(_stream_ptr(x.device))))


class FullPlan:
    """The full-length CQ-NSGT of complex signals of length L (Algorithms 1
    and 2 at length L, Section 3) on the band windows of a sliCQ ``plan``
    sampled on the L-point grid, all 2K+2 bands (0..K+1, then the mirrors of
    K..1). ``lattice="slicq"`` keeps the sliCQ hops (M^L_k = M_k L / 2N: the
    lattice Proposition 4 compares s^0 + s^1 with); ``lattice="painless"``
    takes the smallest power of two >= |J^L_k|, for which synthesis is the
    exact inverse (Proposition 2)."""

    def __init__(self, plan: "Plan", L: int, lattice: str = "slicq"):
        lib = load_library()
        h = ctypes.c_void_p()
        _check(lib.nsgt_full_plan(plan._h, int(L), {"slicq": 0, "painless": 1}[lattice], ctypes.byref(h)))
        self._h, self._lib, self.plan = h, lib, plan
        info = _FullInfo()
        _check(lib.nsgt_full_info(h, ctypes.byref(info)))
        self.L, self.nbands, self.coef_count = info.L, info.nbands, info.coef_count
        self.painless, self.max_M, self.entries = bool(info.painless), info.max_M, info.entries
        self.lattice = lattice
        nb = self.nbands
        self.starts = np.zeros(nb, dtype=np.int64)
        self.lengths = np.zeros(nb, dtype=np.int32)
        self.M = np.zeros(nb, dtype=np.int32)
        self.offsets = np.zeros(nb, dtype=np.int64)
        _check(lib.nsgt_full_bands(h, self.starts.ctypes.data, self.lengths.ctypes.data, self.M.ctypes.data,
                                   self.offsets.ctypes.data))
        self._tables, self._work = {}, {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.nsgt_full_destroy(h)
            self._h = None

    def windows(self):
        """FP64 host tables (g^L, its canonical dual), concatenated over J^L_k."""
        tot = int(self.lengths.sum())
        g, gd = np.zeros(tot), np.zeros(tot)
        _check(self._lib.nsgt_full_windows(self._h, g.ctypes.data, gd.ctypes.data))
        return g, gd

    def band(self, coef, k: int):
        """View of band k's M^L_k coefficients."""
        o = int(self.offsets[k])
        return coef[o:o + int(self.M[k])]

    def _prepare(self, dt: int, device):
        torch = _torch()
        key = (dt, str(device))
        if key not in self._tables:
            nbytes = ctypes.c_size_t()
            _check(self._lib.nsgt_full_table_bytes(self._h, dt, ctypes.byref(nbytes)))
            buf = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
            off = (-buf.data_ptr()) % 256
            _check(self._lib.nsgt_full_upload(self._h, dt, ctypes.c_void_p(buf.data_ptr() + off), nbytes.value,
                                              ctypes.c_void_p(_stream_ptr(device))))
            self._tables[key] = buf
        if key not in self._work:
            b = ctypes.c_size_t()
            _check(self._lib.nsgt_full_workspace_size(self._h, dt, ctypes.byref(b)))
            self._work[key] = torch.empty(b.value, dtype=torch.uint8, device=device)
        return self._work[key]

    def analyze(self, x, out=None):
        """Coefficients (coef_count complex values, band k at offsets[k]) of the
        complex signal x (L values)."""
        torch = _torch()
        _require_cuda(x, "x")
        if not x.is_complex() or x.numel() != self.L:
            raise SlicqError(f"x must be a complex tensor of L = {self.L} values")
        dt = _dtype_code(x)
        if out is None:
            out = torch.empty(self.coef_count, dtype=x.dtype, device=x.device)
        _require_cuda(out, "out")
        w = self._prepare(dt, x.device)
        _check(self._lib.nsgt_full_analyze(self._h, dt, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                           out.numel(), ctypes.c_void_p(w.data_ptr()), w.numel(),
                                           ctypes.c_void_p(_stream_ptr(x.device))))
        return out

    def synthesize(self, coef, out=None):
        """The complex signal (L values) of coefficients on every band."""
        torch = _torch()
        _require_cuda(coef, "coef")
        if not coef.is_complex():
            raise SlicqError("coef must be complex")
        dt = _dtype_code(coef)
        if out is None:
            out = torch.empty(self.L, dtype=coef.dtype, device=coef.device)
        _require_cuda(out, "out")
        if out.numel() < self.L:
            raise SlicqError("out must hold L values")
        w = self._prepare(dt, coef.device)
        _check(self._lib.nsgt_full_synthesize(self._h, dt, ctypes.c_void_p(coef.data_ptr()), coef.numel(),
                                              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                              w.numel(), ctypes.c_void_p(_stream_ptr(coef.device))))
        return out


class StreamServer:
    """Real-time streaming sliCQ (continuous batching; see slicq.h).

    Streams are admitted with ``open()`` (SlicqBusy when the memory budget is
    full), fed with ``push(id, samples)`` from any thread, processed by
    ``tick()`` (every ready slice of every stream in one launch sequence) and
    drained with ``poll(id)``. Samples are host numpy arrays of the dtype.
    """

    def __init__(self, plan: Plan, dtype: str = "f32", max_streams: int = 512, max_batch: int = 1024,
                 hbm_budget_bytes: int = 0, device=None):
        torch = _torch()
        self.plan = plan
        self.dt = F32 if dtype == "f32" else F64
        self.np_dtype = np.float32 if self.dt == F32 else np.float64
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        plan._ensure_tables(self.dt, dev)
        torch.cuda.synchronize(dev)
        self._lib = plan._lib
        h = ctypes.c_void_p()
        _check(self._lib.slicq_stream_server_create(plan._h, self.dt, int(max_streams), int(max_batch),
                                                    int(hbm_budget_bytes), ctypes.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.slicq_stream_server_destroy(h)
            self._h = None

    def open(self) -> int:
        i = ctypes.c_int32()
        _check(self._lib.slicq_stream_open(self._h, ctypes.byref(i)))
        return i.value

    def push(self, sid: int, samples) -> None:
        a = np.ascontiguousarray(samples, dtype=self.np_dtype)
        _check(self._lib.slicq_stream_push(self._h, int(sid), a.ctypes.data, a.size))

    def push_many(self, ids, hops) -> None:
        """One hop (array) per stream id, in one call."""
        counts = np.array([len(h) for h in hops], dtype=np.int64)
        self.push_packed(ids, np.concatenate(hops) if len(hops) else np.zeros(0), counts)

    def push_packed(self, ids, packed, counts) -> None:
        """Hops packed back to back (counts[i] samples for ids[i]), in one call."""
        ids_a = np.ascontiguousarray(ids, dtype=np.int32)
        counts = np.ascontiguousarray(counts, dtype=np.int64)
        if ids_a.size != counts.size or int(counts.sum()) > np.size(packed):
            raise SlicqError("push_packed: ids, counts and samples do not match")
        packed = np.ascontiguousarray(packed, dtype=self.np_dtype)
        _check(self._lib.slicq_stream_push_many(self._h, ids_a.size, ids_a.ctypes.data, packed.ctypes.data,
                                                counts.ctypes.data))

    def poll_many(self, ids, cap: int = 1 << 22):
        """Final output of each stream id (a list of arrays, at most cap samples in all)."""
        ids_a = np.ascontiguousarray(ids, dtype=np.int32)
        counts = np.zeros(ids_a.size, dtype=np.int64)
        out = np.empty(int(cap), dtype=self.np_dtype)
        _check(self._lib.slicq_stream_poll_many(self._h, ids_a.size, ids_a.ctypes.data, out.ctypes.data, out.size,
                                                counts.ctypes.data))
        ends = np.cumsum(counts)
        return [out[e - c:e] for e, c in zip(ends, counts)]

    def push_gap(self, sid: int, n: int) -> None:
        _check(self._lib.slicq_stream_push_gap(self._h, int(sid), int(n)))

    def tick(self) -> int:
        n = ctypes.c_int64()
        _check(self._lib.slicq_stream_tick(self._h, ctypes.byref(n)))
        return n.value

    def poll(self, sid: int, max_samples: Optional[int] = None):
        """Final output samples of stream sid (all that are ready, or at most max_samples)."""
        parts = []
        left = int(max_samples) if max_samples is not None else -1
        n = ctypes.c_int64()
        while left != 0:
            out = np.empty(1 << 16 if left < 0 else min(left, 1 << 16), dtype=self.np_dtype)
            _check(self._lib.slicq_stream_poll(self._h, int(sid), out.ctypes.data, out.size, ctypes.byref(n)))
            parts.append(out[:n.value])
            if left > 0:
                left -= n.value
            if n.value < out.size:
                break
        return parts[0] if len(parts) == 1 else np.concatenate(parts)

    def close(self, sid: int) -> None:
        _check(self._lib.slicq_stream_close(self._h, int(sid)))

    def last_coefs(self, sid: int):
        """(m, c^m) of the stream's most recent slice, or (-1, None)."""
        ct = np.complex64 if self.dt == F32 else np.complex128
        out = np.empty(self.plan.coefs_per_slice, dtype=ct)
        m = ctypes.c_int64()
        _check(self._lib.slicq_stream_coefs(self._h, int(sid), out.ctypes.data, out.size, ctypes.byref(m)))
        return (m.value, out) if m.value >= 0 else (-1, None)

    def stats(self) -> dict:
        st = _StreamStats()
        _check(self._lib.slicq_stream_stats_get(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in _StreamStats._fields_ if name != "pad_"}

    def reset_stats(self) -> None:
        _check(self._lib.slicq_stream_stats_reset(self._h))

    def snapshot(self, sid: int) -> bytes:
        n = ctypes.c_size_t()
        _check(self._lib.slicq_stream_snapshot(self._h, int(sid), None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(self._lib.slicq_stream_snapshot(self._h, int(sid), buf, n.value, ctypes.byref(n)))
        return buf.raw[:n.value]

    def restore(self, sid: int, blob: bytes) -> None:
        _check(self._lib.slicq_stream_restore(self._h, int(sid), blob, len(blob)))


def _make_function():
    torch = _torch()

    class SliCQFunction(torch.autograd.Function):
        """Differentiable analysis: forward = slicq_analyze, backward = slicq_adjoint.

        x is a real (T,) signal or a (B, T) batch of equal-length signals; the
        output is the band-major coefficient vector (per signal for batches).
        The backward of a real-input, complex-output linear map is
        Re(A^H grad).
        """

        @staticmethod
        def forward(ctx, x, plan):
            ctx.plan = plan
            ctx.shape = x.shape
            if x.dim() == 1:
                return plan.analyze(x.contiguous())
            B, T = x.shape
            lay = plan._uniform_layout(B, T)
            ctx.layout = lay
            c = plan.analyze_batched(x.contiguous().view(-1), layout=lay)
            return c.view(B, -1)

        @staticmethod
        def backward(ctx, grad):
            plan = ctx.plan
            grad = grad.contiguous()
            if len(ctx.shape) == 1:
                return plan.adjoint(grad, ctx.shape[0]), None
            B, T = ctx.shape
            gx = plan.synthesize_batched(grad.view(-1), layout=ctx.layout, adjoint=True)
            return gx.view(B, T), None

    return SliCQFunction


def _make_loss_function():
    torch = _torch()

    class LogMagLoss(torch.autograd.Function):
        """sum (log(1 + |c|^2) - target)^2 by one HIP kernel that also writes
        the gradient (saved for backward)."""

        @staticmethod
        def forward(ctx, coef, target):
            lib = load_library()
            _require_cuda(coef, "coef")
            _require_cuda(target, "target")
            dt = _dtype_code(coef)
            c = coef.contiguous()
            t = target.contiguous()
            if t.numel() != c.numel():
                raise SlicqError("target must have one value per coefficient")
            rt = torch.float32 if dt == F32 else torch.float64
            grad = torch.empty_like(c)
            part = torch.empty(int(lib.slicq_logmag_loss_partials(c.numel())), dtype=rt, device=c.device)
            loss = torch.empty((), dtype=rt, device=c.device)
            _check(lib.slicq_logmag_loss(dt, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(t.data_ptr()), c.numel(),
                                         ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(part.data_ptr()),
                                         part.numel(), ctypes.c_void_p(loss.data_ptr()),
                                         ctypes.c_void_p(_stream_ptr(c.device))))
            ctx.save_for_backward(grad)
            return loss

        @staticmethod
        def backward(ctx, g):
            (grad,) = ctx.saved_tensors
            return grad * g, None

    return LogMagLoss


def _make_synthesis_function():
    torch = _torch()

    class SliCQSynthesisFunction(torch.autograd.Function):
        """Differentiable synthesis: forward = slicq_synthesize (coefficients to
        a real signal of T samples), backward = slicq_synthesize_adjoint (the
        dual-window analysis), for losses on the synthesised audio."""

        @staticmethod
        def forward(ctx, coef, plan, T):
            ctx.plan, ctx.T = plan, int(T)
            return plan.synthesize(coef.contiguous(), int(T))

        @staticmethod
        def backward(ctx, grad):
            return ctx.plan.synthesize_adjoint(grad.contiguous()), None, None

    return SliCQSynthesisFunction


_FUNCS = {}


def __getattr__(name):
    makers = {"SliCQFunction": _make_function, "SliCQSynthesisFunction": _make_synthesis_function,
              "LogMagLoss": _make_loss_function}
    if name in makers:
        if name not in _FUNCS:
            _FUNCS[name] = makers[name]()
        return _FUNCS[name]
    raise AttributeError(name)


def slicq(x, plan: Plan):
    """Differentiable sliCQ analysis (see SliCQFunction)."""
    return __getattr__("SliCQFunction").apply(x, plan)


def logmag_loss(coef, target):
    """sum (log(1 + |coef|^2) - target)^2, differentiable (see LogMagLoss)."""
    return __getattr__("LogMagLoss").apply(coef, target)


def islicq(coef, plan: Plan, T: int):
    """Differentiable sliCQ synthesis of one signal (see SliCQSynthesisFunction)."""
    return __getattr__("SliCQSynthesisFunction").apply(coef, plan, T)
