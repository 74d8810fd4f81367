"""Pins of the oracle's transforms against definitions, closed forms and
invariants the paper fixes (equation CQ_coeff, Algorithms 1-4,
Propositions 1-3)."""
import math

import numpy as np
import pytest

from oracle import (OraclePlan, analyze, analyze_full, synthesize, synthesize_full,
                    adjoint, brute, plan_from_tables, analyze_stream, synthesize_stream,
                    pack, num_slices)
from oracle.transform import _band_ifft
from workloads import PRESETS, make_c1, noise_plus_sines

TINY = dict(fs=64.0, fmin=4.0, fmax=16.0, bins_per_octave=3, slice_len=64, transition=8, min_win=0.0)
TINY2 = dict(fs=100.0, fmin=6.0, fmax=40.0, bins_per_octave=4, slice_len=128, transition=16, min_win=4.0)


def tiny(**kw):
    return OraclePlan(**dict(TINY, **kw))


def maxdiff(a, b):
    return max(np.abs(x - y).max() for x, y in zip(a, b))


@pytest.mark.parametrize("kw", [TINY, TINY2])
@pytest.mark.parametrize("T", [1, 40, 64, 150, 256])
def test_fast_analysis_equals_inner_products(kw, T):
    # equation CQ_coeff: c_{n,k} = <x_m, T_{n a_k} F^{-1} g_k>, computed by explicit sums
    pl = OraclePlan(**kw)
    f = np.random.default_rng(T).standard_normal(T)
    fast = analyze(pl, f)
    slow = brute.slicq_coefficients(pl, f, pl.bands)
    assert maxdiff(fast, slow) < 1e-12


def test_complex_full_band_analysis_equals_inner_products():
    pl = OraclePlan(**TINY2)
    g = np.random.default_rng(3)
    f = g.standard_normal(200) + 1j * g.standard_normal(200)
    assert maxdiff(analyze_full(pl, f), brute.slicq_coefficients(pl, f)) < 1e-12


@pytest.mark.parametrize("j0", [0, 3, 5, 17, 31, 32, 40, 63])
def test_pure_tone_closed_form(j0):
    # x = e^{2 pi i j0 t / 2N} has X = sqrt(2N) delta_{j0}: c_{n,k} = sqrt(2N) g_k[j0] e^{2 pi i j0 n / M_k}
    pl = tiny(min_win=2.0)
    n2 = pl.two_n
    X = np.fft.fft(np.exp(2j * math.pi * j0 * np.arange(n2) / n2)) / math.sqrt(n2)
    for b in pl.all_bands:
        gk = brute.band_full(b, n2)[j0]
        expect = math.sqrt(n2) * gk * np.exp(2j * math.pi * j0 * np.arange(b.M) / b.M)
        np.testing.assert_allclose(_band_ifft(X, b, n2), expect, atol=1e-12)


def test_single_full_band_is_identity_times_sqrt_2n():
    # one band g = 1 on all bins, M = 2N: c^m_n = sqrt(2N) x_m[n]
    n2 = 32
    pl = plan_from_tables(n2, 4, [(0, np.ones(n2), n2)])
    f = np.random.default_rng(1).standard_normal(100)
    c = analyze_full(pl, f)[0]
    L = 128
    fp = np.zeros(L)
    fp[:100] = f
    for m in range(c.shape[0]):
        np.testing.assert_allclose(c[m], math.sqrt(n2) * brute.slice_vector(pl, fp, m), atol=1e-12)


def test_uniform_bands_are_a_sampled_stft():
    # Section 2.1, equation STFT: translates g_k = g(. - k b) in frequency give
    # c_{n,k} = e^{2 pi i k b n a / L} sum_l x[l] conj(phi[l - n a]) e^{-2 pi i l k b / L}
    n2, b_hop, width, M = 64, 8, 16, 16
    a = n2 // M
    base = 0.5 + 0.5 * np.cos(2 * math.pi * (np.arange(width) - width / 2 + 0.5) / width)
    bands = [(k * b_hop - width // 2, base, M) for k in range(n2 // b_hop)]
    pl = plan_from_tables(n2, 4, bands)
    x = np.random.default_rng(2).standard_normal(n2) + 0j
    X = np.fft.fft(x) / math.sqrt(n2)
    g0 = np.zeros(n2)
    g0[np.arange(-width // 2, width // 2) % n2] = base
    phi = np.fft.ifft(g0) * math.sqrt(n2)       # F^{-1} of the band centred at 0
    l = np.arange(n2)
    for k, bt in enumerate(pl.bands):
        nsg = _band_ifft(X, bt, n2)
        for n in range(M):
            stft = np.sum(x * np.conj(phi[(l - n * a) % n2]) * np.exp(-2j * math.pi * l * k * b_hop / n2))
            assert abs(nsg[n] * np.exp(-2j * math.pi * k * b_hop * n * a / n2) - stft) < 1e-12


@pytest.mark.parametrize("kw", [TINY, TINY2])
@pytest.mark.parametrize("T", [1, 63, 64, 65, 300])
def test_perfect_reconstruction_tiny(kw, T):
    # Propositions 1 and 3
    pl = OraclePlan(**kw)
    f = np.random.default_rng(T + 7).standard_normal(T)
    assert np.abs(synthesize(pl, analyze(pl, f), T) - f).max() < 1e-13


@pytest.mark.parametrize("name", ["c1", "c4"])
def test_perfect_reconstruction_presets(name):
    p = PRESETS[name]
    pl = OraclePlan(p.fs, p.fmin, p.fmax, p.bins_per_octave, p.slice_len, p.transition)
    f = make_c1() if name == "c1" else noise_plus_sines(50000, p.fs, 11)
    y = synthesize(pl, analyze(pl, f), f.shape[0])
    assert np.abs(y - f).max() / np.abs(f).max() < 1e-14


@pytest.mark.parametrize("kind", ["canonical", "indicator"])
def test_synthesis_equals_dual_atom_expansion(kind):
    # Algorithm 2/4 on arbitrary coefficients = sum_m h~_0 OLA of sum c phi~ with phi~ = S^{-1} phi
    pl = OraclePlan(**dict(TINY2, dual_slice=kind))
    g = np.random.default_rng(5)
    T = 256
    S = num_slices(T, pl.two_n)
    c = [g.standard_normal((S, b.M)) + 1j * g.standard_normal((S, b.M)) for b in pl.bands]
    K = pl.K
    c_all = c + [np.conj(c[2 * K + 2 - k]) for k in range(K + 2, 2 * K + 2)]
    expect = brute.slicq_synthesis_from_duals(pl, c_all, T, real=True)
    np.testing.assert_allclose(synthesize(pl, c, T), expect, atol=1e-12)
    cf = [g.standard_normal((S, b.M)) + 1j * g.standard_normal((S, b.M)) for b in pl.all_bands]
    np.testing.assert_allclose(synthesize_full(pl, cf, T),
                               brute.slicq_synthesis_from_duals(pl, cf, T, real=False), atol=1e-12)


def test_real_signal_symmetries():
    # mirrored bands carry conjugate coefficients; DC and Nyquist are real (Table 1, real signals)
    pl = OraclePlan(**TINY2)
    f = np.random.default_rng(9).standard_normal(256)
    c = analyze_full(pl, f.astype(complex))
    K = pl.K
    for k in range(1, K + 1):
        np.testing.assert_allclose(c[2 * K + 2 - k], np.conj(c[k]), atol=1e-13)
    assert np.abs(c[0].imag).max() < 1e-13 and np.abs(c[K + 1].imag).max() < 1e-13


def test_shift_by_n_moves_slices():
    # circular shift of f by N on L = T samples: c^m -> c^{m-1} (Algorithm 3 indexing)
    pl = OraclePlan(**TINY2)
    T = 512
    f = np.random.default_rng(4).standard_normal(T)
    c = analyze(pl, f)
    cs = analyze(pl, np.roll(f, pl.N))
    for a, b in zip(c, cs):
        np.testing.assert_allclose(b, np.roll(a, 1, axis=0), atol=1e-12)


def test_linearity():
    pl = OraclePlan(**TINY2)
    g = np.random.default_rng(6)
    f1, f2 = g.standard_normal(300), g.standard_normal(300)
    lhs = analyze(pl, 2.5 * f1 - 0.75 * f2)
    rhs = [2.5 * a - 0.75 * b for a, b in zip(analyze(pl, f1), analyze(pl, f2))]
    assert maxdiff(lhs, rhs) < 1e-12


@pytest.mark.parametrize("T", [1, 100, 256])
def test_adjoint_is_transpose_of_dense_analysis(T):
    pl = OraclePlan(**TINY2)
    A = brute.analysis_matrix(pl, T)
    g = np.random.default_rng(T)
    S = num_slices(T, pl.two_n)
    c = [g.standard_normal((S, b.M)) + 1j * g.standard_normal((S, b.M)) for b in pl.bands]
    np.testing.assert_allclose(adjoint(pl, c, T), np.real(A.conj().T @ pack(pl, c)), atol=1e-12)


def test_adjoint_dot_product_c1():
    p = PRESETS["c1"]
    pl = OraclePlan(p.fs, p.fmin, p.fmax, p.bins_per_octave, p.slice_len, p.transition)
    g = np.random.default_rng(8)
    T = 20000
    f = g.standard_normal(T)
    S = num_slices(T, pl.two_n)
    c = [g.standard_normal((S, b.M)) + 1j * g.standard_normal((S, b.M)) for b in pl.bands]
    lhs = np.real(np.vdot(pack(pl, c), pack(pl, analyze(pl, f))))
    assert math.isclose(lhs, float(np.dot(f, adjoint(pl, c, T))), rel_tol=1e-12)


def test_stream_form_equals_circular_without_wrap():
    # a signal with >= N trailing zeros in its padded length: linear and circular slices agree
    pl = OraclePlan(**TINY2)
    T = 300
    f = np.random.default_rng(12).standard_normal(T)
    L = 512                     # 2N ceil(T/2N); L - T = 212 >= N = 64
    S = num_slices(T, pl.two_n)
    a = analyze(pl, f)
    b = analyze_stream(pl, f, S)
    assert maxdiff(a, b) < 1e-13
    y = synthesize_stream(pl, b, L)
    np.testing.assert_allclose(y[:T], f, atol=1e-13)
    assert np.abs(y[T:]).max() < 1e-13


def test_pack_unpack_roundtrip():
    # band-major packing (band k, slice m, index n at S off_k + m M_k + n) and
    # its inverse; element positions checked one by one
    from oracle import OraclePlan, pack, unpack
    pl = OraclePlan(fs=100.0, fmin=6.0, fmax=40.0, bins_per_octave=4, slice_len=128, transition=16, min_win=4.0)
    S = 5
    g = np.random.default_rng(3)
    c = [g.standard_normal((S, b.M)) + 1j * g.standard_normal((S, b.M)) for b in pl.bands]
    flat = pack(pl, c)
    assert flat.shape == (S * pl.coefs_per_slice,)
    off = pl.offsets
    for k, b in enumerate(pl.bands):
        for m in (0, S - 1):
            for n in (0, b.M - 1):
                assert flat[S * off[k] + m * b.M + n] == c[k][m, n]
    back = unpack(pl, flat, S)
    assert all(np.array_equal(a, b) for a, b in zip(back, c))


def test_slice_ranges_partition_the_transform():
    # analysis restricted to slice ranges gives the rows of the full analysis;
    # synthesis contributions of a partition of the slices sum to the full
    # synthesis (the overlap-add is linear), and reconstruct the signal
    from oracle import OraclePlan, analyze, synthesize, analyze_slices, synthesize_slices
    pl = OraclePlan(fs=100.0, fmin=6.0, fmax=40.0, bins_per_octave=4, slice_len=128, transition=16, min_win=4.0)
    T = 700
    x = np.random.default_rng(8).standard_normal(T)
    full = analyze(pl, x)
    S = full[0].shape[0]
    cuts = [0, 3, 4, 9, S]
    parts = [analyze_slices(pl, x, a, b) for a, b in zip(cuts[:-1], cuts[1:])]
    for k in range(pl.nbands):
        assert np.array_equal(np.concatenate([p[k] for p in parts]), full[k])
    y = sum(synthesize_slices(pl, p, T, a, b) for p, a, b in zip(parts, cuts[:-1], cuts[1:]))[:T]
    np.testing.assert_allclose(y, synthesize(pl, full, T), rtol=0, atol=1e-13)
    np.testing.assert_allclose(y, x, rtol=0, atol=1e-12)
