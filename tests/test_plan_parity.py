"""The library's C++ FP64 plan against the oracle's independent plan: band
structure bit-equal (integers), tables to FP64 round-off."""
import numpy as np
import pytest

from oracle import OraclePlan
from workloads import PRESETS

CASES = [dict(fs=p.fs, fmin=p.fmin, fmax=p.fmax, bins_per_octave=p.bins_per_octave, slice_len=p.slice_len,
              transition=p.transition) for p in PRESETS.values()]
CASES += [
    dict(fs=44100.0, fmin=100.0, fmax=16000.0, bins_per_octave=12, slice_len=4096, transition=1024, min_win=8.0,
         window="blackman_harris"),
    dict(fs=44100.0, fmin=60.0, fmax=18000.0, bins_per_octave=24, slice_len=16384, transition=2048, scale="mel"),
    dict(fs=48000.0, fmin=50.0, fmax=15000.0, bins_per_octave=16, slice_len=8192, transition=1024, scale="bark"),
    dict(fs=44100.0, fmin=110.0, fmax=11025.0, bins_per_octave=12, slice_len=8192, transition=1024,
         slicing="sqrt_tukey"),
    dict(fs=8000.0, fmin=200.0, fmax=3000.0, bins_per_octave=48, slice_len=4096, transition=1024, min_win=4.0,
         m_policy="rect"),
    dict(fs=44100.0, fmin=32.7, fmax=22050.0, bins_per_octave=48, slice_len=65536, transition=8192,
         m_policy="smooth"),
    dict(fs=48000.0, fmin=27.5, fmax=20000.0, bins_per_octave=96, slice_len=16384, transition=2048,
         m_policy="smooth", window="blackman_harris"),
    dict(fs=100.0, fmin=6.0, fmax=40.0, bins_per_octave=4, slice_len=128, transition=16, min_win=4.0,
         m_policy="smooth"),
    dict(fs=64.0, fmin=4.0, fmax=16.0, bins_per_octave=3, slice_len=64, transition=8, min_win=0.0),
    dict(fs=100.0, fmin=6.0, fmax=40.0, bins_per_octave=4, slice_len=128, transition=16, min_win=4.0),
    dict(fs=44100.0, fmin=50.0, fmax=22000.0, bins_per_octave=48, slice_len=4096, transition=1024, min_win=8.0),
    dict(fs=22050.0, fmin=200.0, fmax=8000.0, bins_per_octave=7, slice_len=2048, transition=100, min_win=16.0,
         dual_slice="indicator"),
]


def _id(k):
    extra = "-".join(str(k[o]) for o in ("window", "scale", "slicing", "m_policy") if o in k)
    return f"B{k['bins_per_octave']}-2N{k['slice_len']}" + (f"-{extra}" if extra else "")


@pytest.mark.parametrize("kw", CASES, ids=_id)
def test_cpp_plan_matches_oracle(kw):
    import paper_1210_0084_amd as sq
    o = OraclePlan(**kw)
    p = sq.Plan(**kw)
    assert p.K == o.K and p.nbands == o.K + 2
    np.testing.assert_array_equal(p.M, o.Ms)
    np.testing.assert_array_equal(p.offsets, o.offsets)
    np.testing.assert_array_equal(p.starts, [b.start for b in o.bands])
    np.testing.assert_array_equal(p.lengths, [b.length for b in o.bands])
    assert p.coefs_per_slice == o.coefs_per_slice
    tol = 1e-15 if kw.get("scale", "cq") == "cq" else 1e-13   # pow / log10 of the scales
    np.testing.assert_allclose(p.fc[1:-1], o.xi, rtol=tol)
    np.testing.assert_allclose(p.bw[1:-1], o.omega, rtol=tol)
    assert abs(p.Q - o.Q) <= 1e-15 * o.Q
    g, gd, h0, hd, D = p.windows()
    np.testing.assert_allclose(g, np.concatenate([b.g for b in o.bands]), rtol=0, atol=4e-16 if tol < 1e-14 else 1e-12)
    np.testing.assert_allclose(gd, np.concatenate([b.gd for b in o.bands]), rtol=1e-14, atol=1e-18)
    np.testing.assert_allclose(h0, o.h0, rtol=0, atol=4e-16)
    np.testing.assert_allclose(hd, o.hd, rtol=1e-15, atol=1e-18)
    np.testing.assert_allclose(D, o.D, rtol=1e-14)
