"""Pins of the oracle's full-length CQ-NSGT (Algorithms 1 and 2 at the signal
length L, Sections 2-3; the band windows of Proposition 4) against the
definitions: inner products with the time-domain atoms, the dense frame
operator and its inverse, perfect reconstruction, and the sampling relation
g_k[j] = g^L_k[j L / 2N]."""
import math

import numpy as np
import pytest

from oracle import OraclePlan
from oracle.fullnsgt import full_dual, full_length_bands, nsgt_full, nsgt_full_synthesize

TINY2 = dict(fs=100.0, fmin=6.0, fmax=40.0, bins_per_octave=4, slice_len=128, transition=16, min_win=4.0)
SMALLP = dict(fs=800.0, fmin=30.0, fmax=380.0, bins_per_octave=6, slice_len=64, transition=16, min_win=4.0)


def _atoms(bands, L):
    """phi_{n,k}[t] = L^{-1/2} sum_{j in J_k} g_k[j] e^{2 pi i j (t - n a_k) / L},
    a_k = L / M_k: the translates T_{n a_k} of the inverse DFT of g_k
    (equation CQ_coeff's atoms), one row per (k, n)."""
    t = np.arange(L)
    rows = []
    for b in bands:
        a = L // b.M
        j = b.bins()
        for n in range(b.M):
            e = np.exp(2j * np.pi * np.outer(t - n * a, j) / L)
            rows.append(e @ b.g / math.sqrt(L))
    return np.array(rows)


@pytest.mark.parametrize("lattice", ["slicq", "painless"])
@pytest.mark.parametrize("r", [1, 4])
def test_analysis_is_inner_products_with_atoms(lattice, r):
    pl = OraclePlan(**SMALLP)
    L = r * pl.two_n
    bands = full_length_bands(pl, L, all_bands=True, lattice=lattice)
    rng = np.random.default_rng(11)
    f = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    c = np.concatenate(nsgt_full(bands, f))
    ref = _atoms(bands, L).conj() @ f
    np.testing.assert_allclose(c, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_slicq_lattice_and_sampling_relation():
    # Proposition 4: g_k[j] = g^L_k[j L / 2N]; the slicq lattice keeps the hop
    # a_k = 2N / M_k = L / M^L_k
    pl = OraclePlan(**SMALLP)
    r = 8
    L = r * pl.two_n
    bL = full_length_bands(pl, L, all_bands=False)
    for b, f in zip(pl.bands, bL):
        assert L // f.M == pl.two_n // b.M and f.M == r * b.M
        pos = {int(j): v for j, v in zip(f.bins(), f.g)}
        for j, v in zip(b.bins(), b.g):
            assert abs(pos[int(j) * r] - v) < 1e-12, (b.k, j)
    # at L = 2N the full-length bands are the slice plan's bands
    b1 = full_length_bands(pl, pl.two_n, all_bands=False)
    for b, f in zip(pl.bands, b1):
        assert f.start == b.start and f.M == b.M
        np.testing.assert_allclose(f.g, b.g, atol=1e-15)


def test_painless_lattice_covers_every_support():
    pl = OraclePlan(**TINY2)
    for r in (1, 2, 16):
        for b in full_length_bands(pl, r * pl.two_n, lattice="painless"):
            assert b.M >= b.length and b.M & (b.M - 1) == 0 and b.M >= 2
            assert b.M < 2 * max(b.length, 2)


def test_synthesis_is_the_canonical_dual_frame():
    # Proposition 2: with M^L_k >= |J^L_k| the frame operator S = sum phi phi^H
    # is diagonal in frequency; synthesis of coefficients c is sum c_{n,k}
    # S^{-1} phi_{n,k} (dense, brute force)
    pl = OraclePlan(**SMALLP)
    L = 2 * pl.two_n
    bands = full_length_bands(pl, L, lattice="painless")
    A = _atoms(bands, L)
    S = A.T @ A.conj()
    rng = np.random.default_rng(5)
    c = rng.standard_normal(A.shape[0]) + 1j * rng.standard_normal(A.shape[0])
    ref = np.linalg.solve(S, A.T @ c)
    parts, o = [], 0
    for b in bands:
        parts.append(c[o:o + b.M])
        o += b.M
    got = nsgt_full_synthesize(bands, parts, L)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
    # and the frame operator's diagonal is D^L (F S F^H = diag D)
    F = np.fft.fft(np.eye(L)) / math.sqrt(L)
    Dg = np.real(np.diag(F @ S @ F.conj().T))
    D_ref = np.zeros(L)
    for b in bands:
        np.add.at(D_ref, b.bins() % L, b.M * b.g ** 2)
    np.testing.assert_allclose(Dg, D_ref, rtol=1e-12, atol=1e-12)
    for b, gd in zip(bands, full_dual(bands, L)):
        np.testing.assert_allclose(gd * D_ref[b.bins() % L], b.g, rtol=1e-14, atol=0)


@pytest.mark.parametrize("preset,r", [(TINY2, 8), (SMALLP, 32)])
def test_perfect_reconstruction_painless(preset, r):
    pl = OraclePlan(**preset)
    L = r * pl.two_n
    bands = full_length_bands(pl, L, lattice="painless")
    rng = np.random.default_rng(r)
    f = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    y = nsgt_full_synthesize(bands, nsgt_full(bands, f), L)
    assert np.linalg.norm(y - f) <= 1e-13 * np.linalg.norm(f)


def test_pure_tone_peaks_in_its_band():
    # a complex exponential at bin j0 lands only in bands whose support holds j0:
    # |c_{n,k}| = sqrt(L) g_k[j0] for every n (closed form: the unitary DFT of the
    # tone is sqrt(L) at j0)
    pl = OraclePlan(**SMALLP)
    L = 4 * pl.two_n
    bands = full_length_bands(pl, L, lattice="painless")
    j0 = 3 * L // 16
    f = np.exp(2j * np.pi * j0 * np.arange(L) / L)
    for b, c in zip(bands, nsgt_full(bands, f)):
        j = b.bins()
        hit = np.nonzero(j % L == j0)[0]
        expect = float(b.g[hit[0]]) * math.sqrt(L) if len(hit) else 0.0
        np.testing.assert_allclose(np.abs(c), expect, atol=1e-10)
