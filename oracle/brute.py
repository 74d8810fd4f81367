"""Plain definitions, for tiny inputs: atoms, inner products, frame operator.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* Atoms (Section 2.2): phi_{n,k} = T_{n a_k} g^vee_k with g^vee_k = F^{-1} g_k,
  a_k = 2N / M_k. The inverse DFT is written as an explicit sum; the
  translation is the modulation e^{-2 pi i j n / M_k} of the band's signed
  bins (a circular shift when M_k divides 2N).
* Coefficients (equation CQ_coeff): c_{n,k} = <x, phi_{n,k}> = sum_l x[l] conj(phi[l]).
* Frame operator (equation frameop): S = sum_{n,k} phi phi^H.
* Canonical dual atoms (equation candual): S^{-1} phi.
* sliCQ by definition (Algorithm 3): x_m = (f T_{mN} h_0)[j + (m-1)N]
  with circular indices, coefficients of x_m as above.
"""
from __future__ import annotations

import math

import numpy as np


def idft_matrix(n: int) -> np.ndarray:
    """Unitary inverse DFT as an explicit matrix: E[t, j] = n^{-1/2} e^{2 pi i j t / n}."""
    t = np.arange(n)
    return np.exp(2j * math.pi * np.outer(t, t) / n) / math.sqrt(n)


def band_full(b, two_n: int) -> np.ndarray:
    """g_k as a length-2N vector (circular support)."""
    g = np.zeros(two_n)
    g[b.bins() % two_n] = b.g
    return g


def atoms(plan, bands=None, window: str = "g") -> list:
    """List over bands of arrays (M_k, 2N): row n is T_{n a_k} F^{-1} w_k.

    ``window`` is "g" for the analysis windows or "gd" for the dual windows.
    The translation by n a_k = n 2N / M_k is the modulation of the band's
    bins j (signed, j in J_k) by e^{-2 pi i j n / M_k}: for M_k dividing 2N a
    circular shift by an integer, otherwise the band-limited translation by
    a fraction of a sample (equation CQ_coeff with L / a_k = M_k).
    """
    two_n = plan.two_n
    t = np.arange(two_n)
    out = []
    for b in (plan.all_bands if bands is None else bands):
        w = b.g if window == "g" else b.gd
        j = b.bins()
        E = np.exp(2j * math.pi * np.outer(t, j) / two_n) / math.sqrt(two_n)     # (2N, |J_k|)
        mod = np.exp(-2j * math.pi * np.outer(np.arange(b.M), j) / b.M)         # (M_k, |J_k|)
        out.append((mod * w) @ E.T)
    return out


def coefficients(plan, x, bands=None) -> list:
    """c_{n,k} = <x, phi_{n,k}> for one slice-length vector x."""
    x = np.asarray(x)
    return [A.conj() @ x for A in atoms(plan, bands)]


def frame_operator(plan, bands=None) -> np.ndarray:
    """S = sum_{n,k} phi_{n,k} phi_{n,k}^H as a dense (2N, 2N) matrix."""
    Phi = np.concatenate(atoms(plan, bands), axis=0)   # rows are atoms
    return Phi.T @ Phi.conj()


def dual_atoms(plan, bands=None) -> list:
    """Canonical dual atoms S^{-1} phi_{n,k}, by dense linear algebra."""
    S = frame_operator(plan, bands)
    return [np.linalg.solve(S, A.T).T for A in atoms(plan, bands)]


def slice_vector(plan, f, m: int) -> np.ndarray:
    """x_m[j] = f[(j + (m-1)N) mod L] h_0[j - N] (Algorithm 3), f already of length L."""
    two_n, N = plan.two_n, plan.N
    L = f.shape[0]
    return np.array([f[(j + (m - 1) * N) % L] * plan.h0[j] for j in range(two_n)])


def slicq_coefficients(plan, f, bands=None) -> list:
    """Coefficients of every slice by the definition; arrays (S, M_k)."""
    two_n = plan.two_n
    T = len(f)
    L = two_n * ((T + two_n - 1) // two_n)
    fp = np.zeros(L, dtype=np.asarray(f).dtype)
    fp[:T] = f
    S = 2 * L // two_n
    A = atoms(plan, bands)
    out = [np.zeros((S, a.shape[0]), dtype=np.complex128) for a in A]
    for m in range(S):
        xm = slice_vector(plan, fp, m)
        for kk, a in enumerate(A):
            out[kk][m] = a.conj() @ xm
    return out


def slicq_synthesis_from_duals(plan, c_all, T: int, real: bool) -> np.ndarray:
    """f~ = sum_m h~_0-weighted OLA of sum_{n,k} c^m_{n,k} (S^{-1} phi_{n,k}).

    ``c_all`` covers every band of ``plan.all_bands``; with ``real`` the real
    part of each slice is taken (real-signal synthesis).
    """
    two_n, N = plan.two_n, plan.N
    L = two_n * ((T + two_n - 1) // two_n)
    S = 2 * L // two_n
    D = dual_atoms(plan)
    out = np.zeros(L, dtype=np.float64 if real else np.complex128)
    for m in range(S):
        y = np.zeros(two_n, dtype=np.complex128)
        for ck, d in zip(c_all, D):
            y += d.T @ ck[m]
        if real:
            y = y.real
        for j in range(two_n):
            out[(j + (m - 1) * N) % L] += y[j] * plan.hd[j]
    return out[:T]


def analysis_matrix(plan, T: int) -> np.ndarray:
    """Dense matrix of the real-input analysis onto the stored bands.

    Rows follow the band-major packing (band k, slice m, index n); column t
    is the response to the unit impulse at sample t.
    """
    cols = []
    for t in range(T):
        e = np.zeros(T)
        e[t] = 1.0
        c = slicq_coefficients(plan, e, plan.bands)
        cols.append(np.concatenate([ck.reshape(-1) for ck in c]))
    return np.stack(cols, axis=1)
