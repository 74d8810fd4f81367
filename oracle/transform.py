"""FP64 sliCQ analysis, synthesis and adjoint, following Algorithms 1-4.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Conventions (readings where the paper is silent):
* Unitary DFT  F f[j] = (2N)^{-1/2} sum_l f[l] e^{-2 pi i l j / 2N}  (Section 2.1).
* Coefficients are the inner products of equation CQ_coeff:
  c^m_{n,k} = <F x_m, M_{-n a_k} g_k> = sum_{j in J_k} X_m[j] g_k[j] e^{2 pi i j n / M_k},
  i.e. the band product is wrapped at the absolute bin index j mod M_k and
  transformed by an unnormalised inverse DFT of length M_k (Algorithm 1).
* Synthesis (Algorithm 2): C_k = unnormalised DFT_{M_k}(c_k); the slice
  spectrum is sum_k g~_k[j] C_k[j mod M_k]; unitary inverse DFT.
* Slices (Algorithm 3): L = 2N ceil(T / 2N) by zero padding, S = L / N
  slices, x_m[j] = f[(j + (m-1)N) mod L] h_0[j - N] (indices circular).
* Overlap-add (Algorithm 4): f~[(j + (m-1)N) mod L] += y_m[j] h~_0[j - N].
* Real signals: only bands 0..K+1 are stored; the mirrored bands carry the
  conjugate coefficients, and synthesis returns the real part of the full
  synthesis (the frame of Table 1 is symmetric about Nyquist).

Library FFTs (numpy.fft) are used as steps of the algorithms; nothing is
fused or reordered beyond the algorithms' own loops.
"""
from __future__ import annotations

import math
from typing import List

import numpy as np


def padded_length(T: int, two_n: int) -> int:
    """L = 2N ceil(T / 2N): the signal is zero padded to a multiple of 2N (Section 4.1)."""
    return two_n * ((int(T) + two_n - 1) // two_n)


def num_slices(T: int, two_n: int) -> int:
    """S = L / N slices (Algorithm 3 loops m = 0, ..., L/N - 1)."""
    return 2 * padded_length(T, two_n) // two_n


def _slice_index(m: int, N: int, L: int) -> np.ndarray:
    return (np.arange(2 * N) + (m - 1) * N) % L


def _band_ifft(X: np.ndarray, b, two_n: int) -> np.ndarray:
    """Algorithm 1 inner step for one band: wrap X g_k at j mod M_k, inverse DFT."""
    j = b.bins()
    buf = np.zeros(b.M, dtype=np.complex128)
    buf[j % b.M] = X[j % two_n] * b.g
    return np.fft.ifft(buf) * b.M


def analyze(plan, f) -> List[np.ndarray]:
    """sliCQ analysis of a real signal (Algorithm 3 with Algorithm 1 per slice).

    Returns one array per stored band k = 0..K+1, of shape (S, M_k), complex128.
    """
    f = np.asarray(f, dtype=np.float64)
    return _analyze(plan, f, plan.bands)


def analyze_full(plan, f) -> List[np.ndarray]:
    """Analysis of a complex signal onto every band of the plan (no mirroring)."""
    f = np.asarray(f, dtype=np.complex128)
    return _analyze(plan, f, plan.all_bands)


def _analyze(plan, f, bands, m0: int = 0, m1=None):
    two_n, N = plan.two_n, plan.N
    T = f.shape[0]
    L = padded_length(T, two_n)
    S = 2 * L // two_n
    m1 = S if m1 is None else min(int(m1), S)
    fp = np.zeros(L, dtype=f.dtype)
    fp[:T] = f
    out = [np.zeros((max(m1 - m0, 0), b.M), dtype=np.complex128) for b in bands]
    scale = 1.0 / math.sqrt(two_n)
    for m in range(m0, m1):
        xm = fp[_slice_index(m, N, L)] * plan.h0
        X = np.fft.fft(xm) * scale
        for kk, b in enumerate(bands):
            out[kk][m - m0] = _band_ifft(X, b, two_n)
    return out


def analyze_slices(plan, f, m0: int, m1: int) -> List[np.ndarray]:
    """Slices m0 .. m1-1 of ``analyze(plan, f)`` (Algorithm 3's loop over m
    restricted to a range; slices are independent given the signal), so that
    a pool of processes can share the slices of one signal."""
    return _analyze(plan, np.asarray(f, dtype=np.float64), plan.bands, m0, m1)


def _slice_synthesis(plan, coefs_m, bands, window) -> np.ndarray:
    """Algorithm 2 for one slice: DFT_{M_k}, multiply by ``window``, add, inverse DFT."""
    two_n = plan.two_n
    Z = np.zeros(two_n, dtype=np.complex128)
    for c, b in zip(coefs_m, bands):
        C = np.fft.fft(c)
        j = b.bins()
        w = b.gd if window == "dual" else b.g
        np.add.at(Z, j % two_n, w * C[j % b.M])
    return np.fft.ifft(Z) * math.sqrt(two_n)


def _mirror_coefs(plan, c, m):
    """Coefficients of all 2K+2 bands of slice m from the stored bands 0..K+1."""
    K = plan.K
    stored = [c[k][m] for k in range(K + 2)]
    mirrored = [np.conj(c[2 * K + 2 - k][m]) for k in range(K + 2, 2 * K + 2)]
    return stored + mirrored


def synthesize(plan, c, T: int) -> np.ndarray:
    """sliCQ synthesis of a real signal (Algorithm 4 with Algorithm 2 per slice).

    ``c`` holds the stored bands 0..K+1 as arrays (S, M_k). The mirrored
    bands take the conjugate coefficients and the result is the real part of
    the full synthesis.
    """
    two_n = plan.two_n
    L = padded_length(T, two_n)
    return synthesize_slices(plan, c, T, 0, 2 * L // two_n)[:T]


def synthesize_slices(plan, c, T: int, m0: int, m1: int) -> np.ndarray:
    """The contribution of slices m0 .. m1-1 to the overlap-add of Algorithm 4,
    over all L samples of the padded signal (``c`` holds those slices only,
    as arrays (m1 - m0, M_k)). Summing the contributions of a partition of
    the slices gives ``synthesize`` (before truncation to T)."""
    two_n, N = plan.two_n, plan.N
    L = padded_length(T, two_n)
    out = np.zeros(L)
    for m in range(m0, m1):
        y = _slice_synthesis(plan, _mirror_coefs(plan, c, m - m0), plan.all_bands, "dual")
        np.add.at(out, _slice_index(m, N, L), y.real * plan.hd)
    return out


def synthesize_full(plan, c, T: int) -> np.ndarray:
    """Complex synthesis from every band of the plan (no mirroring, no real part)."""
    two_n, N = plan.two_n, plan.N
    L = padded_length(T, two_n)
    S = 2 * L // two_n
    out = np.zeros(L, dtype=np.complex128)
    for m in range(S):
        y = _slice_synthesis(plan, [ck[m] for ck in c], plan.all_bands, "dual")
        np.add.at(out, _slice_index(m, N, L), y * plan.hd)
    return out[:T]


def adjoint(plan, c, T: int) -> np.ndarray:
    """Adjoint of the real-input analysis onto the stored bands: Re(A^H c).

    A maps real x (length T) to the coefficients of bands 0..K+1 (equation
    CQ_coeff after slicing by Algorithm 3). Its adjoint transposes each step:
    per band g_k * DFT_{M_k}(c_k) placed on J_k, unitary inverse DFT of the
    slice, multiplication by h_0, transpose of the circular slice gather,
    truncation to T samples, real part.
    """
    two_n, N = plan.two_n, plan.N
    L = padded_length(T, two_n)
    S = 2 * L // two_n
    out = np.zeros(L)
    for m in range(S):
        y = _slice_synthesis(plan, [ck[m] for ck in c], plan.bands, "analysis")
        np.add.at(out, _slice_index(m, N, L), y.real * plan.h0)
    return out[:T]


def synthesize_adjoint(plan, y, T: int) -> List[np.ndarray]:
    """Adjoint of ``synthesize`` for the real inner products (the gradient of
    a loss of the synthesised signal with respect to the coefficients).

    Synthesis writes y = sum_k w_k Re(c_k gamma_k) over the stored bands,
    with gamma_k the dual atoms (dual windows g~_k on the 2N grid, dual
    slicing window h~_0, Algorithms 2 and 4) and w_k = 2 for bands 1..K
    (each also synthesises through its conjugate mirror) and 1 for the
    self-mirrored DC and Nyquist bands. Its transpose maps y to
    w_k <y, gamma_k>: the analysis of y (Algorithm 3 with Algorithm 1) with
    h~_0 in place of h_0 and g~_k in place of g_k, times w_k.
    """
    two_n, N = plan.two_n, plan.N
    y = np.asarray(y, dtype=np.float64)
    L = padded_length(T, two_n)
    S = 2 * L // two_n
    yp = np.zeros(L)
    yp[:len(y)] = y
    out = [np.zeros((S, b.M), dtype=np.complex128) for b in plan.bands]
    scale = 1.0 / math.sqrt(two_n)
    K = plan.K
    for m in range(S):
        Y = np.fft.fft(yp[_slice_index(m, N, L)] * plan.hd) * scale
        for kk, b in enumerate(plan.bands):
            j = b.bins()
            buf = np.zeros(b.M, dtype=np.complex128)
            buf[j % b.M] = Y[j % two_n] * b.gd
            w = 1.0 if kk in (0, K + 1) else 2.0
            out[kk][m] = w * np.fft.ifft(buf) * b.M
    return out


def pack_full(plan, c) -> np.ndarray:
    """Band-major packing over every band of the plan (stored bands 0..K+1,
    then the mirrors K+2..2K+1): the layout of the complex-signal transform."""
    return np.concatenate([ck.reshape(-1) for ck in c])


def unpack_full(plan, flat, S: int) -> List[np.ndarray]:
    out = []
    pos = 0
    for b in plan.all_bands:
        n = S * b.M
        out.append(np.asarray(flat[pos:pos + n]).reshape(S, b.M))
        pos += n
    return out


def pack(plan, c) -> np.ndarray:
    """Band-major packing: band k, slice m, index n at S*off_k + m*M_k + n."""
    return np.concatenate([ck.reshape(-1) for ck in c])


def unpack(plan, flat, S: int) -> List[np.ndarray]:
    out = []
    pos = 0
    for b in plan.bands:
        n = S * b.M
        out.append(np.asarray(flat[pos:pos + n]).reshape(S, b.M))
        pos += n
    return out


# --- linear (streaming) form --------------------------------------------------

def analyze_stream(plan, f, n_slices: int) -> List[np.ndarray]:
    """Slices of an unbounded signal that is zero before sample 0 and after f.

    Slice m is centred on sample m N and reads f[j + (m-1) N] for j < 2N
    without circular wrap; this is the form a real-time stream computes.
    """
    f = np.asarray(f, dtype=np.float64)
    two_n, N = plan.two_n, plan.N
    T = f.shape[0]
    out = [np.zeros((n_slices, b.M), dtype=np.complex128) for b in plan.bands]
    scale = 1.0 / math.sqrt(two_n)
    for m in range(n_slices):
        pos = np.arange(2 * N) + (m - 1) * N
        ok = (pos >= 0) & (pos < T)
        xm = np.zeros(2 * N)
        xm[ok] = f[pos[ok]]
        X = np.fft.fft(xm * plan.h0) * scale
        for kk, b in enumerate(plan.bands):
            out[kk][m] = _band_ifft(X, b, two_n)
    return out


def synthesize_stream(plan, c, T_out: int) -> np.ndarray:
    """Linear overlap-add of the slices in ``c`` into samples [0, T_out)."""
    two_n, N = plan.two_n, plan.N
    S = c[0].shape[0]
    out = np.zeros(T_out)
    for m in range(S):
        y = _slice_synthesis(plan, _mirror_coefs(plan, c, m), plan.all_bands, "dual")
        pos = np.arange(2 * N) + (m - 1) * N
        ok = (pos >= 0) & (pos < T_out)
        np.add.at(out, pos[ok], (y.real * plan.hd)[ok])
    return out
