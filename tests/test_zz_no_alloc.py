"""The allocation-free analysis entry point (slicq_analyze_static) against
slicq_analyze through the C ABI: bitwise equal coefficients on two calls in
a row (the second with a smaller input), in FP32 (the 60 s benchmark signal
length, processed in chunks of the fixed scratch) and FP64, and a clear
error for a signal whose task table does not fit the scratch."""
import ctypes

import numpy as np
import pytest

from workloads import PRESETS, pink_plus_tones, noise_plus_sines

pytestmark = pytest.mark.gpu


def kw_of(name):
    p = PRESETS[name]
    return dict(fs=p.fs, fmin=p.fmin, fmax=p.fmax, bins_per_octave=p.bins_per_octave, slice_len=p.slice_len,
                transition=p.transition)


def _static(plan, x, out, dev):
    import torch
    P = ctypes.c_void_p
    st = P(torch.cuda.current_stream(dev).cuda_stream)
    dt = 0 if x.dtype == torch.float32 else 1
    return plan._lib.slicq_analyze_static(plan._h, dt, P(x.data_ptr()), x.numel(), P(out.data_ptr()), out.numel(),
                                          st)


@pytest.mark.parametrize("name,dt,lens", [("c2", "f32", (2646000, 700001)), ("c1", "f64", (65536, 9000)),
                                          ("c4", "f32", (264600, 50000))])
def test_static_entry_matches_workspace_entry(dev, name, dt, lens):
    import torch
    import paper_1210_0084_amd as sq
    plan = sq.Plan(**kw_of(name))
    tdt = torch.float32 if dt == "f32" else torch.float64
    ctype = torch.complex64 if dt == "f32" else torch.complex128
    assert plan._lib.slicq_static_scratch_bytes() == 32 << 20
    for i, T in enumerate(lens):
        print(f"case {name} {dt} T={T}", flush=True)
        x = torch.tensor(pink_plus_tones(T, kw_of(name)["fs"], 300 + i), dtype=tdt, device=dev)
        ref = plan.analyze(x)                      # workspace entry point (also uploads the tables)
        out = torch.full((plan.coef_count(T),), float("nan"), dtype=ctype, device=dev)
        assert _static(plan, x, out, dev) == 0, plan._lib.slicq_last_error()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (name, T)


def test_static_entry_rejects_oversized_task_tables(dev):
    # 2N = 128: each slice needs 96 bytes of task table; 400,000 slices do not
    # fit the 32 MiB scratch beside one slice's workspace. The buffers are real
    # (and large enough), so nothing is read out of bounds either way.
    import torch
    import paper_1210_0084_amd as sq
    plan = sq.Plan(fs=100.0, fmin=6.0, fmax=40.0, bins_per_octave=4, slice_len=128, transition=16, min_win=4.0)
    T = 200000 * 128
    x = torch.zeros(T, dtype=torch.float32, device=dev)
    plan.analyze(x[:1000])                         # uploads the tables
    out = torch.empty(plan.coef_count(T), dtype=torch.complex64, device=dev)
    assert plan.num_slices(T) == 400000
    rc = _static(plan, x, out, dev)
    assert rc == -4, rc
    assert "static scratch" in plan._lib.slicq_last_error().decode()
    small = noise_plus_sines(3000, 100.0, 4)
    xs = torch.tensor(small, dtype=torch.float32, device=dev)
    o2 = torch.empty(plan.coef_count(3000), dtype=torch.complex64, device=dev)
    assert _static(plan, xs, o2, dev) == 0
    torch.cuda.synchronize()
    assert torch.equal(o2, plan.analyze(xs))
