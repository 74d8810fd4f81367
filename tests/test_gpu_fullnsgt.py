"""GPU parity of the full-length CQ-NSGT (Algorithms 1 and 2 at the signal
length L) against the FP64 oracle: analysis on both lattices, synthesis and
reconstruction on the painless one, one-block and four-step transform
lengths, the approximation study's shape (L = 2^20), and the sliCQ's
approximation of it (Proposition 4) with both sides on the GPU."""
import math

import numpy as np
import pytest

from oracle import OraclePlan, analyze_full
from oracle.fullnsgt import full_length_bands, nsgt_full, nsgt_full_synthesize, snr_db
from oracle.layers import layers

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}
BAND_TOL = {"f32": 1e-4, "f64": 1e-10}
SMALLP = dict(fs=800.0, fmin=30.0, fmax=380.0, bins_per_octave=6, slice_len=64, transition=16, min_win=4.0)
STUDY = dict(fs=44100.0, fmin=200.0, fmax=22000.0, bins_per_octave=48, slice_len=4096, transition=1024,
             min_win=16.0, window="blackman_harris")


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def sq():
    import paper_1210_0084_amd as m
    return m


@pytest.fixture(scope="module")
def dev():
    import torch
    return torch.device("cuda:0")


def cdt(dt):
    import torch
    return torch.complex64 if dt == "f32" else torch.complex128


def signal(L, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(L) + 1j * g.standard_normal(L)


def check_bands(fp, got, ref_parts, dt):
    ref = np.concatenate(ref_parts)
    assert rel(got, ref) <= TOL[dt]
    worst = max(rel(got[int(o):int(o) + int(m)], r) for o, m, r in zip(fp.offsets, fp.M, ref_parts)
                if np.linalg.norm(r) > 0)
    assert worst <= BAND_TOL[dt], worst


@pytest.mark.parametrize("dt", ["f32", "f64"])
@pytest.mark.parametrize("L,lattice", [(64, "slicq"), (256, "painless"), (8192, "slicq"), (16384, "painless"),
                                       (1 << 18, "painless")])
def test_small_plan(sq, dev, dt, L, lattice):
    import torch
    print(f"case full-length L={L} {lattice} {dt}", flush=True)
    plan = sq.Plan(**SMALLP)
    fp = sq.FullPlan(plan, L, lattice)
    bands = full_length_bands(OraclePlan(**SMALLP), L, True, lattice)
    assert [b.M for b in bands] == list(fp.M) and [b.start for b in bands] == list(fp.starts)
    f = signal(L, L + 3)
    x = torch.tensor(f, dtype=cdt(dt), device=dev)
    c = fp.analyze(x)
    ref = nsgt_full(bands, f)
    torch.cuda.synchronize()
    check_bands(fp, c.cpu().numpy(), ref, dt)
    assert fp.painless
    y = fp.synthesize(torch.tensor(np.concatenate(ref), dtype=cdt(dt), device=dev))
    yc = fp.synthesize(c)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), nsgt_full_synthesize(bands, ref, L)) <= TOL[dt]
    assert rel(yc.cpu().numpy(), f) <= TOL[dt]


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_study_shape_analysis(sq, dev, dt):
    # 2N = 4096, B = 48, Blackman-Harris, L = 2^20 on the sliCQ lattice:
    # band transforms of up to 2^15 points (four-step) and aliasing bands
    import torch
    print(f"case full-length study shape {dt}", flush=True)
    L = 1 << 20
    plan = sq.Plan(**STUDY)
    fp = sq.FullPlan(plan, L, "slicq")
    assert not fp.painless and fp.max_M > 4096
    f = signal(L, 20)
    c = fp.analyze(torch.tensor(f, dtype=cdt(dt), device=dev))
    ref = nsgt_full(full_length_bands(OraclePlan(**STUDY), L, True, "slicq"), f)
    torch.cuda.synchronize()
    check_bands(fp, c.cpu().numpy(), ref, dt)
    with pytest.raises(sq.SlicqError, match="painless"):
        fp.synthesize(c)


def test_painless_roundtrip_long(sq, dev):
    # L = 2^22 at 2N = 16384: every FFT of the path is a four-step one
    import torch
    print("case full-length painless 2^22 f32", flush=True)
    kw = dict(STUDY, slice_len=16384, transition=4096)
    L = 1 << 22
    fp = sq.FullPlan(sq.Plan(**kw), L, "painless")
    f = signal(L, 22)
    x = torch.tensor(f, dtype=torch.complex64, device=dev)
    y = fp.synthesize(fp.analyze(x))
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), f) <= TOL["f32"]


def test_slicq_approximates_full_length_on_gpu(sq, dev):
    # Section 5.3 / Proposition 4: s^0 + s^1 from the GPU sliCQ against the
    # GPU full-length transform rescaled by sqrt(2N / L) gives the oracle's SNR
    import torch
    print("case full-length approximation SNR", flush=True)
    kw = dict(STUDY, slice_len=16384, transition=4096)
    L = 1 << 17
    plan = sq.Plan(**kw)
    opl = OraclePlan(**kw)
    fp = sq.FullPlan(plan, L, "slicq")
    f = signal(L, 11)
    x = torch.tensor(f, dtype=torch.complex128, device=dev)
    S = plan.num_slices(L)
    ls = plan.layers(plan.analyze_complex(x)[:S * plan.coefs_per_slice], S).cpu().numpy()
    cf = fp.analyze(x).cpu().numpy()
    r = math.sqrt(opl.two_n / L)
    full = [r * cf[int(o):int(o) + int(m)] for o, m in zip(fp.offsets[:plan.nbands], fp.M[:plan.nbands])]
    approx = [ls[(S // 2) * int(off):(S // 2) * (int(off) + int(m))] for off, m in zip(plan.offsets, plan.M)]
    snr_gpu = snr_db(full, approx)
    ref_full = nsgt_full(full_length_bands(opl, L, all_bands=False), f)
    lay = layers(opl, analyze_full(opl, f)[:opl.K + 2])
    snr_ref = snr_db([r * v for v in ref_full], [a + b for a, b in lay])
    print(f"SNR GPU {snr_gpu:.3f} dB, oracle {snr_ref:.3f} dB", flush=True)
    assert abs(snr_gpu - snr_ref) < 0.01
