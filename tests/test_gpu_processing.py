"""GPU parity of the frame variants, the adjoint of synthesis, the complex
transform and the coefficient-domain kernels against the FP64 oracle, and one
point of the Section 5.3 approximation study computed on the GPU."""
import math

import numpy as np
import pytest

from oracle import (OraclePlan, analyze, synthesize, synthesize_adjoint, analyze_full, synthesize_full, pack,
                    pack_full, unpack, unpack_full, num_slices)
from oracle.layers import layers, spectrogram, apply_mask, transpose
from oracle.fullnsgt import full_length_bands, nsgt_full, snr_db
from workloads import pink_plus_tones, noise_plus_sines

pytestmark = pytest.mark.gpu

TOL = {"f32": 1e-5, "f64": 1e-12}


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def sq():
    import paper_1210_0084_amd as m
    return m


def tdt(dt):
    import torch
    return torch.float32 if dt == "f32" else torch.float64


def cdt(dt):
    import torch
    return torch.complex64 if dt == "f32" else torch.complex128


C4 = dict(fs=44100.0, fmin=65.4, fmax=16000.0, bins_per_octave=36, slice_len=16384, transition=2048)
VARIANTS = [
    (dict(C4, window="blackman_harris"), "bh"),
    (dict(C4, scale="mel"), "mel"),
    (dict(C4, scale="bark", bins_per_octave=12), "bark"),
    (dict(C4, slicing="sqrt_tukey"), "sqrt"),
    (dict(fs=8000.0, fmin=200.0, fmax=3000.0, bins_per_octave=48, slice_len=4096, transition=1024, min_win=4.0,
          m_policy="rect"), "rect"),
    (dict(C4, m_policy="smooth"), "smooth"),
    (dict(C4, m_policy="smooth", scale="mel", window="blackman_harris"), "smooth-mel-bh"),
]


@pytest.mark.parametrize("fused", [True, False], ids=["fused", "pipeline"])
@pytest.mark.parametrize("kw,name", VARIANTS, ids=[v[1] for v in VARIANTS])
def test_variant_plans(sq, dev, kw, name, fused):
    import torch
    print(f"case variant {name} fused={fused}", flush=True)
    plan = sq.Plan(**kw, fused=fused)
    opl = OraclePlan(**kw)
    T = 60000
    x = pink_plus_tones(T, kw["fs"], 17)
    ref = pack(opl, analyze(opl, x))
    xd = torch.tensor(x, dtype=torch.float32, device=dev)
    c = plan.analyze(xd)
    y = plan.synthesize(c, T)
    torch.cuda.synchronize()
    assert rel(c.cpu().numpy(), ref) <= 1e-5
    assert rel(y.cpu().numpy(), x) <= 1e-5


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_synthesis_adjoint(sq, dev, dt):
    # against the oracle's adjoint of synthesis, and the dot-product identity
    # <S c, y> = Re <c, S^T y> computed on the GPU
    import torch
    kw = dict(fs=44100.0, fmin=110.0, fmax=11025.0, bins_per_octave=12, slice_len=8192, transition=1024)
    for fused in (True, False):
        plan = sq.Plan(**kw, fused=fused)
        opl = OraclePlan(**kw)
        T = 40000
        y = noise_plus_sines(T, 44100.0, 21)
        ref = pack(opl, synthesize_adjoint(opl, y, T))
        got = plan.synthesize_adjoint(torch.tensor(y, dtype=tdt(dt), device=dev))
        torch.cuda.synchronize()
        assert rel(got.cpu().numpy(), ref) <= TOL[dt], (fused, rel(got.cpu().numpy(), ref))
        g = np.random.default_rng(3)
        cr = g.standard_normal(len(ref)) + 1j * g.standard_normal(len(ref))
        crd = torch.tensor(cr, dtype=cdt(dt), device=dev)
        yd = torch.tensor(y, dtype=tdt(dt), device=dev)
        lhs = float(torch.dot(plan.synthesize(crd, T), yd).item())
        rhs = float(torch.sum((crd.conj() * got).real).item())
        assert abs(lhs - rhs) <= (1e-4 if dt == "f32" else 1e-10) * abs(lhs)


def test_synthesis_autograd_gradient_fd(sq, dev):
    # islicq: gradient of a loss of the synthesised signal with respect to the
    # coefficients, against central differences in FP64 on a few coordinates
    import torch
    kw = dict(fs=100.0, fmin=6.0, fmax=40.0, bins_per_octave=4, slice_len=128, transition=16, min_win=4.0)
    plan = sq.Plan(**kw)
    T = 300
    S = plan.num_slices(T)
    g = np.random.default_rng(8)
    c0 = torch.tensor(g.standard_normal(S * plan.coefs_per_slice) + 1j * g.standard_normal(S * plan.coefs_per_slice),
                      dtype=torch.complex128, device=dev)
    target = torch.tensor(g.standard_normal(T), dtype=torch.float64, device=dev)

    def loss(c):
        y = sq.islicq(c, plan, T)
        return ((y - target) ** 2).sum() + (y ** 4).sum() * 1e-2

    c = c0.clone().requires_grad_(True)
    loss(c).backward()
    grad = c.grad.detach()
    h = 1e-5
    for i in g.integers(0, c0.numel(), 6):
        for part, unit in ((0, 1.0), (1, 1j)):
            e = torch.zeros_like(c0)
            e[i] = unit * h
            fd = (loss(c0 + e) - loss(c0 - e)).item() / (2 * h)
            an = grad[i].real.item() if part == 0 else grad[i].imag.item()
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (i, part, fd, an)


@pytest.mark.parametrize("dt", ["f32", "f64"])
def test_complex_transform(sq, dev, dt):
    import torch
    kw = dict(fs=44100.0, fmin=110.0, fmax=11025.0, bins_per_octave=12, slice_len=8192, transition=1024)
    plan = sq.Plan(**kw)
    opl = OraclePlan(**kw)
    T = 30000
    g = np.random.default_rng(9)
    f = g.standard_normal(T) + 1j * g.standard_normal(T)
    ref = pack_full(opl, analyze_full(opl, f))
    assert plan.coefs_per_slice_all * num_slices(T, opl.two_n) == len(ref)
    fd = torch.tensor(f, dtype=cdt(dt), device=dev)
    c = plan.analyze_complex(fd)
    y = plan.synthesize_complex(c, T)
    torch.cuda.synchronize()
    assert rel(c.cpu().numpy(), ref) <= TOL[dt]
    assert rel(y.cpu().numpy(), f) <= TOL[dt]
    # synthesis of arbitrary coefficients on all bands
    S = num_slices(T, opl.two_n)
    cr = g.standard_normal(len(ref)) + 1j * g.standard_normal(len(ref))
    ys = plan.synthesize_complex(torch.tensor(cr, dtype=cdt(dt), device=dev), T).cpu().numpy()
    assert rel(ys, synthesize_full(opl, unpack_full(opl, cr, S), T)) <= TOL[dt]


@pytest.mark.parametrize("layout", ["band", "slice"])
def test_layers_masks_transposition(sq, dev, layout):
    import torch
    kw = dict(fs=8000.0, fmin=200.0, fmax=3000.0, bins_per_octave=48, slice_len=4096, transition=1024, min_win=4.0,
              m_policy="rect")
    plan = sq.Plan(**kw, layout=layout)
    opl = OraclePlan(**kw)
    T = 40000
    x = pink_plus_tones(T, 8000.0, 5)
    c_ref = analyze(opl, x)
    S = num_slices(T, opl.two_n)
    c = plan.analyze(torch.tensor(x, dtype=torch.float64, device=dev))
    # layer sum and spectrogram on the layer grid, band-major
    ls = plan.layers(c, S).cpu().numpy()
    sp = plan.layers(c, S, spectrogram=True).cpu().numpy()
    lay = layers(opl, c_ref)
    assert rel(ls, np.concatenate([a + b for a, b in lay])) <= 1e-12
    assert rel(sp, np.concatenate(spectrogram(opl, c_ref))) <= 1e-12
    # dB mask
    g = np.random.default_rng(4)
    masks = [g.uniform(0, 1, S * b.M // 2) for b in opl.bands]
    cm = c.clone()
    plan.mask_db(cm, S, torch.tensor(np.concatenate(masks), dtype=torch.float64, device=dev))
    got = plan.to_band_major(cm, S).cpu().numpy()
    assert rel(got, pack(opl, apply_mask(opl, c_ref, masks))) <= 1e-12
    # transposition by 8 bands (2 semitones at 48 per octave)
    ct = plan.transpose(c, S, 8)
    assert rel(plan.to_band_major(ct, S).cpu().numpy(), pack(opl, transpose(opl, c_ref, 8))) <= 1e-12
    # a plan whose moved bands change M refuses
    p2 = sq.Plan(fs=8000.0, fmin=200.0, fmax=3000.0, bins_per_octave=48, slice_len=4096, transition=1024, min_win=4.0)
    c2 = p2.analyze(torch.tensor(x, dtype=torch.float64, device=dev))
    with pytest.raises(sq.SlicqError):
        p2.transpose(c2, S, 8)


@pytest.mark.parametrize("layout", ["band", "slice"])
def test_layers_and_masks_smooth_policy(sq, dev, layout):
    # layer sums, spectrogram and masks with M_k = 3 2^a and 5 2^a (layer
    # positions and slice indices by general division)
    import torch
    kw = dict(fs=8000.0, fmin=200.0, fmax=3000.0, bins_per_octave=24, slice_len=4096, transition=1024, min_win=4.0,
              m_policy="smooth")
    plan = sq.Plan(**kw, layout=layout)
    opl = OraclePlan(**kw)
    assert any(b.M % 3 == 0 for b in opl.bands) and any(b.M % 5 == 0 for b in opl.bands)
    T = 40000
    x = pink_plus_tones(T, 8000.0, 6)
    c_ref = analyze(opl, x)
    S = num_slices(T, opl.two_n)
    c = plan.analyze(torch.tensor(x, dtype=torch.float64, device=dev))
    assert rel(plan.to_band_major(c, S).cpu().numpy(), pack(opl, c_ref)) <= 1e-12
    ls = plan.layers(c, S).cpu().numpy()
    sp = plan.layers(c, S, spectrogram=True).cpu().numpy()
    lay = layers(opl, c_ref)
    assert rel(ls, np.concatenate([a + b for a, b in lay])) <= 1e-12
    assert rel(sp, np.concatenate(spectrogram(opl, c_ref))) <= 1e-12
    g = np.random.default_rng(5)
    masks = [g.uniform(0, 1, S * b.M // 2) for b in opl.bands]
    cm = c.clone()
    plan.mask_db(cm, S, torch.tensor(np.concatenate(masks), dtype=torch.float64, device=dev))
    assert rel(plan.to_band_major(cm, S).cpu().numpy(), pack(opl, apply_mask(opl, c_ref, masks))) <= 1e-12


def test_approximation_study_point(sq, dev):
    # Section 5.3 on the GPU: a random complex 2^17-sample signal, Blackman-
    # Harris bands, minimal filter length 16: s^0 + s^1 from the GPU sliCQ
    # against the full-length CQ-NSGT (FP64 oracle, rescaled by sqrt(2N / L))
    import torch
    kw = dict(fs=44100.0, fmin=50.0, fmax=22000.0, bins_per_octave=48, slice_len=16384, transition=4096,
              window="blackman_harris", min_win=16.0)
    plan = sq.Plan(**kw)
    opl = OraclePlan(**kw)
    L = 1 << 17
    g = np.random.default_rng(11)
    f = g.standard_normal(L) + 1j * g.standard_normal(L)
    c = plan.analyze_complex(torch.tensor(f, dtype=torch.complex64, device=dev))
    S = plan.num_slices(L)
    stored = c[:S * plan.coefs_per_slice]
    ls = plan.layers(stored, S).cpu().numpy().astype(np.complex128)
    cf = nsgt_full(full_length_bands(opl, L, all_bands=False), f)
    r = math.sqrt(opl.two_n / L)
    approx = [ls[(S // 2) * off:(S // 2) * (off + b.M)] for off, b in zip(opl.offsets, opl.bands)]
    snr_gpu = snr_db([r * x for x in cf], approx)
    lay = layers(opl, analyze_full(opl, f)[:opl.K + 2])
    snr_ref = snr_db([r * x for x in cf], [a + b for a, b in lay])
    print(f"SNR GPU {snr_gpu:.2f} dB, oracle {snr_ref:.2f} dB", flush=True)
    assert snr_ref > 60.0 and abs(snr_gpu - snr_ref) < 1.0
