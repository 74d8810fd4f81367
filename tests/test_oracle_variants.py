"""Pins of the oracle's frame variants and coefficient-domain functions
(Sections 4.3, 5.3, 6 and 7): window shapes, mel and Bark centres, the
square-root slicing windows, the rectangular representation, the adjoint of
synthesis, the 2-layer array, masks, transposition, the full-length NSGT and
the bound of Proposition 4. None re-types the oracle's formula: each checks
an invariant, a closed form or a brute-force definition."""
import json
import math
import os

import numpy as np
import pytest

from oracle import (OraclePlan, analyze, synthesize, synthesize_adjoint, analyze_full, synthesize_full,
                    num_slices, brute)
from oracle.plan import window_value, SCALES
from oracle.layers import layers, spectrogram, apply_mask, mask_gain, transpose
from oracle.fullnsgt import full_length_bands, nsgt_full, snr_db, prop4_bound

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SMALL = dict(fs=1000.0, fmin=40.0, fmax=400.0, bins_per_octave=6, slice_len=256, transition=64)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b)


def test_blackman_harris_shape():
    # the 4-term Blackman-Harris window: 1 at the centre, symmetric, about
    # 6e-5 at the support's edges, and its coefficients sum to one
    assert math.isclose(window_value("blackman_harris", 0.0), 1.0, abs_tol=1e-15)
    for x in (0.1, 0.27, 0.49):
        assert window_value("blackman_harris", x) == window_value("blackman_harris", -x)
    assert 0 < window_value("blackman_harris", 0.5) < 1e-4
    assert math.isclose(window_value("hann", 0.25), 0.5, abs_tol=1e-15)


@pytest.mark.parametrize("opts", [dict(window="blackman_harris"), dict(scale="mel"), dict(scale="bark"),
                                  dict(slicing="sqrt_tukey"), dict(m_policy="rect"), dict(m_policy="smooth"),
                                  dict(window="blackman_harris", slicing="sqrt_tukey", scale="mel"),
                                  dict(window="blackman_harris", m_policy="smooth", scale="bark")],
                         ids=["bh", "mel", "bark", "sqrt", "rect", "smooth", "combined", "combined-smooth"])
def test_variants_reconstruct_and_match_atoms(opts):
    # every variant is still a painless frame with a dual slicing window:
    # perfect reconstruction (Propositions 1-3), and the fast analysis equals
    # the inner products with the atoms (equation CQ_coeff)
    pl = OraclePlan(**SMALL, min_win=4, **opts)
    x = np.random.default_rng(1).standard_normal(700)
    c = analyze(pl, x)
    assert np.abs(synthesize(pl, c, 700) - x).max() < 1e-12
    S = num_slices(700, pl.two_n)
    xs = np.zeros(S * pl.N)
    xs[:700] = x
    m = 3
    xm = xs[(np.arange(pl.two_n) + (m - 1) * pl.N) % len(xs)] * pl.h0
    for k in (0, 1, pl.K // 2, pl.K + 1):
        ref = brute.coefficients(pl, xm, [pl.bands[k]])[0]
        assert np.abs(ref - c[k][m]).max() < 1e-10 * max(1.0, np.abs(ref).max())


def test_smooth_policy_lattice():
    # equation framecond1 with the even smooth numbers: M_k >= |J_k|, even,
    # 2^a, 3 2^a or 5 2^a, and no smaller such number holds the support
    # (brute enumeration); it never exceeds the power-of-two policy
    def ok(m):
        if m % 2:
            return False
        while m % 2 == 0:
            m //= 2
        return m in (1, 3, 5)
    for kw in (SMALL, dict(fs=44100.0, fmin=32.7, fmax=22050.0, bins_per_octave=48, slice_len=65536,
                           transition=8192)):
        ps = OraclePlan(**kw, min_win=4, m_policy="smooth")
        pp = OraclePlan(**kw, min_win=4)
        for bs, bp in zip(ps.bands, pp.bands):
            assert ok(bs.M) and bs.M >= max(bs.length, 2) and bs.M <= bp.M
            assert not any(ok(m) for m in range(max(bs.length, 2), bs.M)), (bs.k, bs.length, bs.M)
    assert sum(b.M for b in ps.bands) < 0.85 * sum(b.M for b in pp.bands)     # c2: 76,476 vs 94,416


def test_smooth_policy_is_painless_with_fractional_hops():
    # M_k need not divide 2N: the atoms are translated by a fraction of a
    # sample (a_k = 2N / M_k), the frame operator stays diagonal in frequency
    # with D = sum M_k g_k^2 (Proposition 2), and synthesis of coefficients
    # equals the expansion in the dense canonical dual atoms
    pl = OraclePlan(fs=100.0, fmin=6.0, fmax=40.0, bins_per_octave=4, slice_len=64, transition=16, min_win=4.0,
                    m_policy="smooth")
    assert any(pl.two_n % b.M for b in pl.bands)
    S_op = brute.frame_operator(pl)
    F = np.fft.fft(np.eye(pl.two_n)) / math.sqrt(pl.two_n)
    Sf = F @ S_op @ F.conj().T
    np.testing.assert_allclose(Sf, np.diag(pl.D), atol=1e-12)
    duals = brute.dual_atoms(pl)
    A = np.concatenate(brute.atoms(pl, window="gd"), axis=0)
    np.testing.assert_allclose(A, np.concatenate(duals, axis=0), atol=1e-12)


def test_sqrt_tukey_partition_of_squares():
    # Section 4.3's other design: sum_m h_m^2 = 1, so the canonical dual is h_0 itself
    pl = OraclePlan(**SMALL, slicing="sqrt_tukey")
    N = pl.N
    sq = pl.h0 ** 2
    tot = sq.copy()
    tot[N:] += sq[:N]
    tot[:N] += sq[N:]
    assert np.abs(tot - 1.0).max() < 1e-15
    np.testing.assert_allclose(pl.hd, pl.h0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("scale", ["mel", "bark"])
def test_scale_centres(scale):
    # centres equally spaced on the scale from fmin, bandwidth = distance of
    # the neighbouring centres (as Omega_k = xi_{k+1} - xi_{k-1} for constant Q)
    fwd, inv = SCALES[scale]
    assert math.isclose(inv(fwd(1234.5)), 1234.5, rel_tol=1e-12)
    pl = OraclePlan(44100, 100, 8000, 12, 16384, 2048, min_win=0, scale=scale)
    u = np.array([fwd(x) for x in pl.xi])
    d = np.diff(u)
    np.testing.assert_allclose(d, d[0], rtol=1e-9)
    assert math.isclose(pl.xi[0], 100.0, rel_tol=1e-12)
    k = np.arange(1, pl.K - 1)
    np.testing.assert_allclose(pl.omega[k], pl.xi[k + 1] - pl.xi[k - 1], rtol=1e-9)


def test_scale_reference_values():
    # published reference points: 1000 Hz is 1000 mel; Traunmueller's Bark
    # formula puts 1000 Hz at 8.53 Bark
    assert abs(SCALES["mel"][0](1000.0) - 1000.0) < 0.05
    assert abs(SCALES["bark"][0](1000.0) - 8.527) < 0.01


def test_rect_policy_is_uniform():
    pl = OraclePlan(**SMALL, min_win=4, m_policy="rect")
    widest = max(1 << (b.length - 1).bit_length() for b in pl.bands)
    assert set(pl.Ms) == {max(2, widest)}


def _real_coef_dot(c1, c2):
    return sum(float(np.real(np.vdot(b, a))) for a, b in zip(c1, c2))


def test_synthesis_adjoint_dot_product_and_dense():
    # <S c, y> = Re<c, S^T y> for random c, y; and S^T equals the transpose
    # of the dense real matrix of synthesis on a tiny plan
    pl = OraclePlan(**SMALL, min_win=4)
    T = 600
    S = num_slices(T, pl.two_n)
    g = np.random.default_rng(5)
    c = [g.standard_normal((S, b.M)) + 1j * g.standard_normal((S, b.M)) for b in pl.bands]
    y = g.standard_normal(T)
    lhs = float(np.dot(synthesize(pl, c, T), y))
    rhs = _real_coef_dot(c, synthesize_adjoint(pl, y, T))
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    tiny = OraclePlan(fs=64.0, fmin=4.0, fmax=16.0, bins_per_octave=3, slice_len=64, transition=8, min_win=0.0)
    T = 70
    S = num_slices(T, tiny.two_n)
    sizes = [S * b.M for b in tiny.bands]
    n = sum(sizes)
    cols = []
    for i in range(2 * n):            # real and imaginary parts of every coefficient
        flat = np.zeros(n, dtype=complex)
        flat[i % n] = 1.0 if i < n else 1j
        cs, pos = [], 0
        for b, sz in zip(tiny.bands, sizes):
            cs.append(flat[pos:pos + sz].reshape(S, b.M))
            pos += sz
        cols.append(synthesize(tiny, cs, T))
    A = np.array(cols).T              # T x 2n real matrix
    for t in (0, 17, 69):
        e = np.zeros(T)
        e[t] = 1.0
        adj = np.concatenate([a.reshape(-1) for a in synthesize_adjoint(tiny, e, T)])
        np.testing.assert_allclose(np.concatenate([adj.real, adj.imag]), A[t], atol=1e-12)


def test_complex_transform_reconstructs_and_is_linear():
    pl = OraclePlan(**SMALL, min_win=4)
    g = np.random.default_rng(6)
    a, b = g.standard_normal(500), g.standard_normal(500)
    f = a + 1j * b
    c = analyze_full(pl, f)
    assert np.abs(synthesize_full(pl, c, 500) - f).max() < 1e-12
    ca, cb = analyze(pl, a), analyze(pl, b)
    K = pl.K
    for k in range(K + 2):
        np.testing.assert_allclose(c[k], ca[k] + 1j * cb[k], atol=1e-12)
    for k in range(1, K + 1):                   # mirror 2K+2-k
        np.testing.assert_allclose(c[2 * K + 2 - k], np.conj(ca[k]) + 1j * np.conj(cb[k]), atol=1e-12)


def test_layers_follow_algorithm3_and_approximate_full_length():
    # the 2-layer array places slice m at (m-1) M/2 (Algorithm 3); s^0 + s^1
    # approximates the full-length coefficients rescaled by sqrt(2N/L)
    # (Proposition 4 in unitary normalisation), within the bound
    pl = OraclePlan(**SMALL, min_win=4, window="blackman_harris")
    L = 8 * pl.two_n
    f = np.random.default_rng(2).standard_normal(L)
    c = analyze(pl, f)
    lay = layers(pl, c)
    S = c[0].shape[0]
    for k in (0, 3):
        M = pl.bands[k].M
        s0, s1 = lay[k]
        assert len(s0) == S * M // 2
        np.testing.assert_array_equal(s1[:M], c[k][1])
        np.testing.assert_array_equal(s0[-M // 2:], c[k][0][:M // 2])     # slice 0 starts at -M/2
        np.testing.assert_array_equal(s0[:M // 2], c[k][0][M // 2:])
    cf = nsgt_full(full_length_bands(pl, L, all_bands=False), f)
    r = math.sqrt(pl.two_n / L)
    bound = prop4_bound(pl, L, np.linalg.norm(f))
    worst = 0.0
    for k, ((s0, s1), ck, bk) in enumerate(zip(lay, cf, bound)):
        half = pl.bands[k].M // 2
        err = np.abs(s0 + s1 - r * ck).reshape(-1, half).max(axis=0)
        assert np.all(err <= bk * (1 + 1e-9)), k
        worst = max(worst, float((err / bk).max()))
    assert worst > 1e-3                           # the bound is not vacuous


def test_approximation_improves_with_minimal_filter_length():
    # Section 5.3: below a minimal length of 8 samples the sliCQ differs
    # visibly, above 16 it is largely equivalent to the full-length transform
    facts = json.load(open(os.path.join(GOLDEN, "paper_facts.json")))["minimal_filter_length"]
    snr = {}
    for mw in (4, facts["visibly_different_below"], facts["equivalent_above"]):
        pl = OraclePlan(44100, 100, 16000, 12, 4096, 1024, min_win=mw, window="blackman_harris")
        L = 16 * pl.two_n
        f = np.random.default_rng(3).standard_normal(L) + 1j * np.random.default_rng(4).standard_normal(L)
        c = analyze_full(pl, f)
        lay = layers(pl, c[:pl.K + 2])
        cf = nsgt_full(full_length_bands(pl, L, all_bands=False), f)
        r = math.sqrt(pl.two_n / L)
        snr[mw] = snr_db([r * x for x in cf], [a + b for a, b in lay])
    assert snr[4] < snr[8] < snr[16]
    assert snr[16] > 60.0


def test_masks_in_db():
    pl = OraclePlan(**SMALL, min_win=4)
    c = analyze(pl, np.random.default_rng(7).standard_normal(800))
    S = c[0].shape[0]
    ones = [np.ones(S * b.M // 2) for b in pl.bands]
    assert all(np.array_equal(a, b) for a, b in zip(apply_mask(pl, c, ones), c))
    zeros = [np.zeros(S * b.M // 2) for b in pl.bands]
    assert all(np.allclose(a, 1e-5 * b, rtol=1e-14) for a, b in zip(apply_mask(pl, c, zeros), c))
    assert math.isclose(float(mask_gain(0.5)), 10 ** -2.5, rel_tol=1e-14)     # -50 dB
    # a mask that is 1 on one band only keeps that band
    k = 4
    one_band = [np.ones(S * b.M // 2) if i == k else np.zeros(S * b.M // 2) for i, b in enumerate(pl.bands)]
    masked = apply_mask(pl, c, one_band)
    assert np.array_equal(masked[k], c[k]) and np.allclose(masked[k + 1], 1e-5 * c[k + 1])


def test_transposition_moves_a_tone_by_two_semitones():
    # Section 6: 8 bands up at 48 bands per octave are 2 semitones; with the
    # rectangular representation (one M for all bands) the band shift moves a
    # stationary tone's frequency by 2^(8/48)
    facts = json.load(open(os.path.join(GOLDEN, "paper_facts.json")))["transposition"]
    B, d = facts["bins_per_octave"], facts["bins"]
    pl = OraclePlan(8000.0, 200.0, 3000.0, B, 4096, 1024, min_win=4, m_policy="rect")
    T = 8 * 4096
    k0 = pl.K // 2
    f0 = pl.xi[k0 - 1]
    x = np.cos(2 * math.pi * f0 * np.arange(T) / pl.fs)
    c = analyze(pl, x)
    y = synthesize(pl, transpose(pl, c, d), T)
    spec = np.abs(np.fft.rfft(y[T // 4:3 * T // 4] * np.hanning(T // 2)))
    f_peak = np.argmax(spec) * pl.fs / (T // 2)
    assert abs(f_peak / f0 - 2 ** (facts["semitones"] / 12)) < 0.01
    sp = spectrogram(pl, transpose(pl, c, d))
    energy = [float(s.sum()) for s in sp]
    assert int(np.argmax(energy)) == k0 + d
