"""Coefficient-domain views and processing of sliCQ coefficients.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* The 2-layer array of Algorithm 3: slice m's coefficients of band k go to
  layer l = m mod 2 at positions (m - 1) M_k / 2 + n (n < M_k), indices
  circular modulo L / a_k = S M_k / 2.
* The sliCQ spectrogram |s^0 + s^1|^2 (Section 4.3, after Proposition 4).
* Masks drawn in dB (Section 6): a mask value v in [0, 1] scales the
  coefficients at its time-frequency position by 10^{(v - 1) 100 / 20}
  (0 is -100 dB, 1 is 0 dB); one mask value serves both layers.
* Transposition (Section 6): moving a component up by d bands (8 bands = 2
  semitones at 48 bands per octave) moves the coefficients of band k to band
  k + d; it needs equal M_k over the bands it moves (the rectangular
  representation of Section 6, or a run of equal M_k).
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np


def layers(plan, c) -> List[Tuple[np.ndarray, np.ndarray]]:
    """(s^0_k, s^1_k) for each stored band, each of length S M_k / 2,
    placed as Algorithm 3 places them."""
    out = []
    for ck, b in zip(c, plan.bands):
        S, M = ck.shape
        n_l = S * M // 2
        s = [np.zeros(n_l, dtype=np.complex128), np.zeros(n_l, dtype=np.complex128)]
        for m in range(S):
            pos = ((m - 1) * (M // 2) + np.arange(M)) % n_l
            s[m % 2][pos] = ck[m]
        out.append((s[0], s[1]))
    return out


def spectrogram(plan, c) -> List[np.ndarray]:
    """|s^0_k + s^1_k|^2 per stored band."""
    return [np.abs(s0 + s1) ** 2 for s0, s1 in layers(plan, c)]


def mask_gain(v):
    """dB mask value in [0, 1] to an amplitude factor: 0 -> 1e-5, 1 -> 1."""
    return 10.0 ** ((np.asarray(v, dtype=np.float64) - 1.0) * 5.0)


def apply_mask(plan, c, masks) -> List[np.ndarray]:
    """Coefficients scaled by the dB mask of their layer position: masks[k]
    has S M_k / 2 values; coefficient n of slice m sits at position
    (m - 1) M_k / 2 + n (circular), as in ``layers``."""
    out = []
    for ck, mk in zip(c, masks):
        S, M = ck.shape
        n_l = S * M // 2
        g = mask_gain(mk)
        o = np.zeros_like(ck)
        for m in range(S):
            pos = ((m - 1) * (M // 2) + np.arange(M)) % n_l
            o[m] = ck[m] * g[pos]
        out.append(o)
    return out


def transpose(plan, c, d: int) -> List[np.ndarray]:
    """Band k + d takes band k's coefficients (constant-Q bands 1..K; bands
    shifted past either end are dropped, vacated bands and the DC and
    Nyquist bands are zero). Needs M_k = M_{k+d} for every moved band."""
    K = plan.K
    out = [np.zeros_like(ck) for ck in c]
    for k in range(1, K + 1):
        t = k + d
        if 1 <= t <= K:
            if c[k].shape != out[t].shape:
                raise ValueError("transposition needs equal M_k over the moved bands")
            out[t] = c[k].copy()
    return out
