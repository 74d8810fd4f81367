"""CPU parity of the library's kernels, compiled unmodified by g++ against a
thread-per-lane stand-in for the HIP runtime (tests/emu), against the FP64
oracle. This checks the kernels' index arithmetic and the launch geometry on
the host before any GPU run; the GPU tests check the same on the device."""
import numpy as np
import pytest

from oracle import OraclePlan, analyze, synthesize, adjoint, pack, unpack, num_slices
from tests.emu import harness as H


@pytest.fixture(scope="module", autouse=True)
def _runners():
    H.build_all()


TINY = dict(fs=64.0, fmin=4.0, fmax=16.0, bins_per_octave=3, slice_len=64, transition=8, min_win=0.0)
TINY2 = dict(fs=100.0, fmin=6.0, fmax=40.0, bins_per_octave=4, slice_len=128, transition=16, min_win=4.0)
SIXTEEN = dict(fs=16.0, fmin=2.0, fmax=6.0, bins_per_octave=2, slice_len=16, transition=2, min_win=1.0)
C4 = dict(fs=44100.0, fmin=65.4, fmax=16000.0, bins_per_octave=36, slice_len=16384, transition=2048)
C5 = dict(fs=48000.0, fmin=27.5, fmax=20000.0, bins_per_octave=96, slice_len=16384, transition=2048)
TOL = {0: 1e-5, 1: 1e-12}


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("dtype", [1, 0])
@pytest.mark.parametrize("kw,T,fused", [(TINY, 1, 0), (TINY, 100, 0), (TINY2, 300, 0), (SIXTEEN, 37, 0),
                                        (TINY, 1, 1), (TINY, 100, 1), (TINY2, 300, 1),
                                        (dict(TINY2, m_policy="smooth"), 300, 0),
                                        (dict(TINY, m_policy="smooth"), 100, 0)])
def test_emu_roundtrip_and_adjoint(kw, T, fused, dtype):
    # fused = 1: one workgroup per slice (half spectrum and band transforms in LDS)
    pl = OraclePlan(**kw)
    x = np.random.default_rng(T).standard_normal(T)
    c_ref = analyze(pl, x)
    ref = pack(pl, c_ref)
    assert rel(H.analyze(kw, x, dtype, fused=fused), ref) <= TOL[dtype]
    assert rel(H.synthesize(kw, ref, T, dtype, fused=fused), x) <= TOL[dtype]
    g = np.random.default_rng(T + 1)
    cr = g.standard_normal(len(ref)) + 1j * g.standard_normal(len(ref))
    S = num_slices(T, pl.two_n)
    assert rel(H.synthesize(kw, cr, T, dtype, adjoint=True, fused=fused),
               adjoint(pl, unpack(pl, cr, S), T)) <= TOL[dtype]
    assert rel(H.synthesize(kw, cr, T, dtype, fused=fused), synthesize(pl, unpack(pl, cr, S), T)) <= TOL[dtype]


class _Path:
    """The harness calls with the kernel path chosen (fused = 1: one workgroup per slice)."""

    def __init__(self, fused):
        self.analyze = lambda *a, **k: H.analyze(*a, fused=fused, **k)
        self.synthesize = lambda *a, **k: H.synthesize(*a, fused=fused, **k)
        self.analyze_batched = lambda *a, **k: H.analyze_batched(*a, fused=fused, **k)
        self.synthesize_batched = lambda *a, **k: H.synthesize_batched(*a, fused=fused, **k)


@pytest.mark.parametrize("fused", [0, 1])
def test_emu_chunked_and_batched(fused):
    kw = TINY
    E = _Path(fused)
    pl = OraclePlan(**kw)
    x = np.random.default_rng(5).standard_normal(500)
    ref = pack(pl, analyze(pl, x))
    assert rel(E.analyze(kw, x, 1, chunk=3), ref) < 1e-12
    assert rel(E.synthesize(kw, ref, 500, 1, chunk=3), x) < 1e-12
    # one slice per chunk: every shared output sample has its two slices in
    # different launches, the first slice's left neighbour (the last slice,
    # circularly) in a later one; two slices share both of their overlaps
    assert rel(E.synthesize(kw, ref, 500, 1, chunk=1), x) < 1e-12
    x2 = np.random.default_rng(6).standard_normal(64)
    r2 = pack(pl, analyze(pl, x2))
    assert num_slices(64, pl.two_n) == 2
    assert rel(E.synthesize(kw, r2, 64, 1, chunk=1), x2) < 1e-12
    assert rel(E.synthesize(kw, r2, 64, 0, chunk=1), x2) < 1e-5
    xs = [np.random.default_rng(i).standard_normal(n) for i, n in enumerate([100, 0, 64, 257])]
    cb = E.analyze_batched(kw, xs, 1)
    refb = np.concatenate([pack(pl, analyze(pl, v)) for v in xs if len(v)])
    assert rel(cb, refb) < 1e-12
    yb = E.synthesize_batched(kw, refb, [len(v) for v in xs], 1)
    assert rel(yb, np.concatenate(xs)) < 1e-12


@pytest.mark.parametrize("fused", [0, 1])
@pytest.mark.parametrize("kw", [C4, C5], ids=["c4", "c5"])
def test_emu_preset_shapes(kw, fused):
    # one pair of slices at full slice length: large band groups (M_k = 8192 in c4),
    # many overlapping narrow bands (c5), both thread-count variants of the band
    # kernels; fused = 1: one workgroup per slice, its spectrum and scratch in LDS
    pl = OraclePlan(**kw)
    T = 9000
    x = np.random.default_rng(3).standard_normal(T)
    ref = pack(pl, analyze(pl, x))
    assert rel(H.analyze(kw, x, 0, fused=fused), ref) <= 1e-5
    assert rel(H.synthesize(kw, ref, T, 0, fused=fused), x) <= 1e-5


@pytest.mark.parametrize("kw", [C4, C5], ids=["c4", "c5"])
def test_emu_smooth_policy_presets(kw):
    # M_k the smallest even 2^a, 3 2^a or 5 2^a: mixed-radix band kernels at
    # full slice length (many M = 12, 20, 24, 40 ... bands in c5)
    kw = dict(kw, m_policy="smooth")
    pl = OraclePlan(**kw)
    assert any(b.M % 3 == 0 for b in pl.bands) and any(b.M % 5 == 0 for b in pl.bands)
    T = 9000
    x = np.random.default_rng(4).standard_normal(T)
    ref = pack(pl, analyze(pl, x))
    assert rel(H.analyze(kw, x, 0), ref) <= 1e-5
    assert rel(H.synthesize(kw, ref, T, 0), x) <= 1e-5


def test_emu_slice_major_layout():
    # slice-major packing: slice m's coefficients c^m contiguous, band k at m*C + off_k
    kw = TINY2
    pl = OraclePlan(**kw)
    T = 300
    x = np.random.default_rng(21).standard_normal(T)
    c = analyze(pl, x)
    S = num_slices(T, pl.two_n)
    slice_major = np.concatenate([np.concatenate([ck[m] for ck in c]) for m in range(S)])
    assert rel(H.analyze(kw, x, 1, layout=1), slice_major) < 1e-12
    assert rel(H.synthesize(kw, slice_major, T, 1, layout=1), x) < 1e-12
    xs = [np.random.default_rng(i).standard_normal(n) for i, n in enumerate([100, 0, 257])]
    ref = np.concatenate([np.concatenate([np.concatenate([ck[m] for ck in analyze(pl, v)])
                                          for m in range(num_slices(len(v), pl.two_n))]) for v in xs if len(v)])
    assert rel(H.analyze_batched(kw, xs, 1, layout=1), ref) < 1e-12


def test_emu_streaming_server():
    # the streaming scheduler with the library's kernels on the CPU: every
    # stream's output reconstructs its input (Proposition 3, linear slicing),
    # is bit-identical alone and in the mix, and a snapshot replays bit for bit
    kw = TINY2
    sig = [np.random.default_rng(70 + i).standard_normal(n) for i, n in enumerate([700, 333, 520])]
    ys, stats = H.stream(kw, sig, hop=32, dtype=1, mode=0, max_streams=4, max_batch=6)
    for y, x in zip(ys, sig):
        assert np.abs(y - x).max() < 1e-12
    alone, _ = H.stream(kw, sig, hop=32, dtype=1, mode=2, max_streams=4, max_batch=6)
    assert np.array_equal(alone[0], ys[1])
    assert stats[0] == 4 and stats[1] == 0 and stats[2] > 0      # 3 streams + the snapshot replay


@pytest.mark.parametrize("opts", [dict(group_cap=64, lds_cap=512, pass_cap=256),
                                  dict(group_cap=4096, lds_cap=16384, pass_cap=1024)], ids=["small", "large"])
def test_emu_tuning_options(opts):
    # other work-item decompositions of the c4 shape (FP32): many small items and
    # lone large synthesis items; the largest items and wide slice-pass items
    kw = C4
    pl = OraclePlan(**kw)
    T = 9000
    x = np.random.default_rng(8).standard_normal(T)
    ref = pack(pl, analyze(pl, x))
    assert rel(H.analyze(kw, x, 0, **opts), ref) <= 1e-5
    assert rel(H.synthesize(kw, ref, T, 0, **opts), x) <= 1e-5


def test_emu_streaming_round_robin_under_overload():
    # more ready slices per tick than max_batch: every stream is still served
    # within a few ticks (the scan starts where the previous batch was cut
    # short), and after a drain every stream reconstructs its input
    kw = TINY2
    sig = [np.random.default_rng(90 + i).standard_normal(2000) for i in range(3)]
    ys, stats = H.stream(kw, sig, hop=128, dtype=1, mode=0, max_streams=4, max_batch=3)
    for y, x in zip(ys, sig):
        assert np.abs(y - x).max() < 1e-12
    assert stats[4] > 0          # by round 8 every stream has released output


FULLP = dict(fs=800.0, fmin=30.0, fmax=380.0, bins_per_octave=6, slice_len=64, transition=16, min_win=4.0)


@pytest.mark.parametrize("L,lattice", [(256, "slicq"), (8192, "painless"), (16384, "slicq")])
@pytest.mark.parametrize("dtype", [1, 0])
def test_emu_full_length(L, lattice, dtype):
    # the full-length kernels (one-block FFTs up to 4096 points, four-step
    # above, band gather, dual overlap-add) against the oracle: analysis, then
    # synthesis of the oracle's coefficients and reconstruction
    from oracle.fullnsgt import full_length_bands, nsgt_full, nsgt_full_synthesize
    opl = OraclePlan(**FULLP)
    bands = full_length_bands(opl, L, True, lattice)
    rng = np.random.default_rng(L)
    f = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    ref = np.concatenate(nsgt_full(bands, f))
    lat = {"slicq": 0, "painless": 1}[lattice]
    c = H.full("ana", FULLP, L, lat, f, dtype=dtype)
    assert rel(c, ref) <= TOL[dtype]
    assert all(b.length <= b.M for b in bands)      # this plan's lattices do not alias
    parts, o = [], 0
    for b in bands:
        parts.append(ref[o:o + b.M])
        o += b.M
    y = H.full("syn", FULLP, L, lat, ref, dtype=dtype)
    assert rel(y, nsgt_full_synthesize(bands, parts, L)) <= TOL[dtype]
    assert rel(y, f) <= TOL[dtype]
