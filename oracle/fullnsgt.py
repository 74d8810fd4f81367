"""The full-length constant-Q NSGT that the sliCQ approximates, and the
approximation bound of Proposition 4 (Sections 3 and 4.3, Section 5.3).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

For a sliCQ plan with slice length 2N and a signal length L (a multiple of
2N), the full-length system uses the same band windows in Hz, sampled on the
L-point grid: g^L_k[j L / 2N] = g_k[j] (Proposition 4's relation). Two
lattices: "slicq" takes L / a_k = M_k L / 2N coefficients per band, so that
both transforms sample the same time-frequency lattice (the comparison of
Proposition 4); "painless" takes the smallest power of two >= |J^L_k| (at
least 2; one M for all bands on a rectangular plan), the condition of
Proposition 2 under which the frame operator is diagonal. Its coefficients
are (Algorithm 1 at length L, unitary DFT)
c_{n,k} = sum_j (F_L f)[j] g^L_k[j] e^{2 pi i j n / M^L_k}, and synthesis is
Algorithm 2 at length L with the canonical duals g^L_k / D^L,
D^L = sum_k M^L_k |g^L_k|^2 over all 2K+2 bands.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np

from .plan import BandTable, window_value


def full_length_bands(plan, L: int, all_bands: bool = True, lattice: str = "slicq") -> List[BandTable]:
    """Band windows of ``plan`` (same centres, bandwidths, widening and
    plateaus, in Hz) on the L-point grid; M^L_k = M_k L / 2N ("slicq") or
    the smallest power of two >= |J^L_k| ("painless")."""
    if lattice not in ("slicq", "painless"):
        raise ValueError("lattice must be 'slicq' or 'painless'")
    fs, two_n = plan.fs, plan.two_n
    if L % two_n:
        raise ValueError("L must be a multiple of 2N")
    r = L // two_n
    out = []
    K = plan.K
    for b in plan.bands:
        if b.k == 0 or b.k == K + 1:
            centre = 0 if b.k == 0 else L // 2
            R = (plan.xi[0] if b.k == 0 else fs / 2 - plan.xi[K - 1])
            om = plan.omega[0] if b.k == 0 else plan.omega[K - 1]
            w = min(om / 2, R)
            e = 0
            while (e + 1) * fs / L < R:
                e += 1
            j = np.arange(centre - e, centre + e + 1)
            d = np.abs(j - centre) * fs / L
            g = np.where(d <= R - w, 1.0, 0.5 + 0.5 * np.cos(math.pi * (d - R + w) / w))
            out.append(BandTable(b.k, centre - e, g, b.M * r))
        else:
            xi, om = plan.xi[b.k - 1], plan.omega[b.k - 1]
            lo = int(math.floor((xi - om / 2) * L / fs)) - 2
            hi = int(math.ceil((xi + om / 2) * L / fs)) + 2
            js = [j for j in range(lo, hi + 1) if abs((j * fs / L - xi) / om) < 0.5]
            g = np.array([window_value(plan.window, (j * fs / L - xi) / om) for j in js])
            out.append(BandTable(b.k, js[0], g, b.M * r))
    if lattice == "painless":
        for b in out:
            b.M = max(2, 1 << max(0, int(b.length - 1).bit_length()))
        if getattr(plan, "m_policy", "pow2") == "rect":
            Mr = max(b.M for b in out)
            for b in out:
                b.M = Mr
    if all_bands:
        for k in range(K + 2, 2 * K + 2):
            src = out[2 * K + 2 - k]
            out.append(BandTable(k, -(src.start + src.length - 1), src.g[::-1].copy(), src.M))
    return out


def nsgt_full(bands, f) -> List[np.ndarray]:
    """Full-length NSGT coefficients of f (length L) on ``bands`` (Algorithm 1
    at length L with the unitary DFT); one array of M^L_k values per band."""
    f = np.asarray(f, dtype=np.complex128)
    L = f.shape[0]
    X = np.fft.fft(f) / math.sqrt(L)
    out = []
    for b in bands:
        j = b.bins()
        buf = np.zeros(b.M, dtype=np.complex128)
        np.add.at(buf, j % b.M, X[j % L] * b.g)
        out.append(np.fft.ifft(buf) * b.M)
    return out


def full_dual(bands, L: int) -> List[np.ndarray]:
    """Canonical dual windows g^L_k / D^L over each J^L_k (Proposition 2 at
    length L), D^L[j] = sum_k M^L_k g^L_k[j]^2 over the given bands (all
    2K+2 of them for the complex transform)."""
    D = np.zeros(L)
    for b in bands:
        np.add.at(D, b.bins() % L, b.M * b.g ** 2)
    if np.any(D <= 0):
        raise ValueError("frame condition fails: D^L has a zero")
    return [b.g / D[b.bins() % L] for b in bands]


def nsgt_full_synthesize(bands, coefs, L: int) -> np.ndarray:
    """Algorithm 2 at length L: C_k = DFT_{M_k}(c_k) (unnormalised, e^-),
    Z[j] = sum_k gd_k[j] C_k[j mod M_k] over j in J^L_k, then the unitary
    inverse DFT of length L. The inverse of ``nsgt_full`` when every band
    satisfies M^L_k >= |J^L_k| (the painless case)."""
    Z = np.zeros(L, dtype=np.complex128)
    for b, gd, c in zip(bands, full_dual(bands, L), coefs):
        C = np.fft.fft(np.asarray(c, dtype=np.complex128))
        j = b.bins()
        np.add.at(Z, j % L, gd * C[j % b.M])
    return np.fft.ifft(Z) * math.sqrt(L)


def snr_db(c, approx) -> float:
    """20 log10 ||c|| / ||c - approx|| over all bands (Section 5.3)."""
    num = math.sqrt(sum(float(np.sum(np.abs(x) ** 2)) for x in c))
    den = math.sqrt(sum(float(np.sum(np.abs(x - y) ** 2)) for x, y in zip(c, approx)))
    return 20.0 * math.log10(num / den) if den > 0 else math.inf


def prop4_bound(plan, L: int, f_norm: float) -> List[np.ndarray]:
    """Right-hand side of Proposition 4 (equation inner_outer) in this
    build's normalisation, per stored band k and n^s < N / a_k:

        |s^0 + s^1 - sqrt(2N / L) c|  <=  sqrt(2N / L) ||f||_2 (
            ||(1 - h_0 - h_1) T_{n^s a_k} g^L_k||_2
          + ||(h_0 + h_1) sum_{j=1}^{L/2N - 1} T_{n^s a_k + 2jN} g^L_k||_2 )

    with g^L_k = F_L^{-1} of the band window on the L grid (unitary), h_0
    the slicing window centred on sample 0 and h_1 = T_N h_0, both as
    L-periodic sequences. The factor sqrt(2N / L) is the ratio of the two
    unitary DFT normalisations: the 2N-periodic extension of the L-point atom
    is sqrt(L / 2N) times the 2N-point atom (periodisation identity of the
    proof). The bound holds for every slice pair m, m + 1 (translation)."""
    two_n, N = plan.two_n, plan.N
    r = L // two_n
    t = np.arange(L)
    # slicing windows on the circle of length L: h_0 centred on 0, h_1 on N
    h0 = np.zeros(L)
    idx = (np.arange(two_n) - N) % L          # window position j - N for j < 2N
    h0[idx] = plan.h0
    w = h0 + np.roll(h0, N)
    out = []
    for bL in full_length_bands(plan, L, all_bands=False):
        G = np.zeros(L, dtype=np.complex128)
        j = bL.bins()
        G[j % L] = bL.g
        atom = np.fft.ifft(G) * math.sqrt(L)     # unitary inverse DFT
        a = L // bL.M                            # hop on the L grid (= a_k of the slice plan)
        Ms = bL.M // r // 2                      # n^s < N / a_k
        bk = np.zeros(Ms)
        for ns in range(Ms):
            at = np.roll(atom, ns * a)
            over = np.zeros(L, dtype=np.complex128)
            for q in range(1, r):
                over += np.roll(at, 2 * q * N)
            bk[ns] = np.linalg.norm((1.0 - w) * at) + np.linalg.norm(w * over)
        out.append(math.sqrt(two_n / L) * f_norm * bk)
    del t
    return out
