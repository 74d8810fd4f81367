"""FP64 plan of the constant-Q painless nonstationary Gabor frame and of the
Tukey slicing windows.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sources in the paper
--------------------
* Section 3 and Table 1: centre frequencies xi_k = xi_min 2^{(k-1)/B},
  bandwidths Omega_k = xi_k / Q with Q = (2^{1/B} - 2^{-1/B})^{-1}, a DC band
  and a Nyquist band built from plateau functions, mirrored bands
  K+2..2K+1 for real signals, g_k[j] = H((j xi_s / L - xi_k) / Omega_k).
* Section 2.2, equation framecond1: the hop a_k satisfies L / a_k >= L_k,
  here L / a_k = M_k is the number of coefficients per band.
* Proposition 2 (equations painlessframe1/2): the frame operator is the
  multiplication by D[j] = sum_k (L/a_k) |g_k[j]|^2 and the canonical dual
  windows are g_k / D.
* Section 4.3: Tukey slicing window h_0 with essential length N and
  transitions of length M, zero padded to 2N; uniform partition of unity
  (equation BUPU) and a dual h~_0 with sum_m T_{mN}(h_0 h~_0) = 1
  (equation dualwincond).
* Section 5.3: a lower bound on the filter length ("minimal filter length").

Readings where the paper is silent:
* Hann H(x) = 1/2 + 1/2 cos(2 pi x) on |x| < 1/2.
* Minimal filter length: Omega_k is widened to ``min_win * fs / 2N`` with the
  centre kept.
* K: the smallest K0 with xi_K0 >= xi_max, then reduced until
  xi_K + Omega_K / 2 < fs / 2 (the paper's K cannot exceed Nyquist).
* Plateaus: flat top 1 with a raised-cosine flank of width Omega_1/2
  (Omega_K/2) ending at xi_1 (at xi_K), so that g_0 + g_1 = 1 and
  g_K + g_{K+1} = 1 on the flanks. Distances are measured in whole bins from
  0 and from N so that both plateaus are exactly symmetric.
* M_k is the smallest power of two >= |J_k| and >= 2, so M_k divides 2N.
* h_0 is a raised cosine centred on sample 0 (needs N - M even); the
  canonical dual is h_0 / sum_m T_{mN} h_0^2.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


def q_factor(B: int) -> float:
    """Q = (2^{1/B} - 2^{-1/B})^{-1} (Section 3)."""
    return 1.0 / (2.0 ** (1.0 / B) - 2.0 ** (-1.0 / B))


# Nonlinear frequency scales (Section 7 names mel and Bark as the obvious
# generalisations): a scale maps Hz to a unit in which the centre frequencies
# are equally spaced. Constant-Q is log2 (equally spaced in octaves).
def _mel(f):
    return 2595.0 * math.log10(1.0 + f / 700.0)


def _mel_inv(u):
    return 700.0 * (10.0 ** (u / 2595.0) - 1.0)


def _bark(f):
    # Traunmueller's critical-band rate
    return 26.81 * f / (1960.0 + f) - 0.53


def _bark_inv(z):
    return 1960.0 * (z + 0.53) / (26.28 - z)


SCALES = {"mel": (_mel, _mel_inv), "bark": (_bark, _bark_inv)}


def window_value(kind: str, x: float) -> float:
    """Frequency window shape on |x| < 1/2 (x in units of the bandwidth):
    Hann (the configurations) or the 4-term Blackman-Harris window the paper
    uses for its approximation study (Section 5.3)."""
    if kind == "hann":
        return 0.5 + 0.5 * math.cos(2.0 * math.pi * x)
    if kind == "blackman_harris":
        return (0.35875 + 0.48829 * math.cos(2.0 * math.pi * x) + 0.14128 * math.cos(4.0 * math.pi * x)
                + 0.01168 * math.cos(6.0 * math.pi * x))
    raise ValueError("window is 'hann' or 'blackman_harris'")


def _next_pow2(n: int) -> int:
    return 1 << (max(n, 1) - 1).bit_length()


def smooth_even_at_least(n: int) -> int:
    """Smallest even integer >= max(n, 2) whose only prime factors are 2, 3
    and 5 with at most one factor 3 or 5 (2^a, 3 2^a, 5 2^a; a >= 1)."""
    n = max(int(n), 2)
    best = None
    for r in (1, 3, 5):
        m = 2 * r
        while m < n:
            m *= 2
        best = m if best is None else min(best, m)
    return best


@dataclasses.dataclass
class BandTable:
    """One band k: values of g_k over its circular support J_k.

    ``start`` is the signed first bin of J_k (a negative bin j stands for
    2N + j); J_k = {start, ..., start + len(g) - 1}.
    """
    k: int
    start: int
    g: np.ndarray          # g_k over J_k, float64
    M: int                 # M_k = L / a_k, coefficients per slice
    gd: Optional[np.ndarray] = None   # dual window over J_k
    xi: float = 0.0        # centre frequency in Hz (Table 1)
    omega: float = 0.0     # bandwidth in Hz (Table 1)

    @property
    def length(self) -> int:
        return int(self.g.shape[0])

    def bins(self) -> np.ndarray:
        return self.start + np.arange(self.length)


def _interval(pred, guess_lo: int, guess_hi: int, margin: int = 3):
    """Integer interval [a, b] on which ``pred`` holds, searched around guesses.

    ``pred`` must hold on an interval; the guesses come from the continuous
    bounds and the exact bounds are settled by evaluating ``pred`` itself.
    """
    lo = guess_lo - margin
    hi = guess_hi + margin
    pts = [j for j in range(lo, hi + 1) if pred(j)]
    if not pts:
        return None
    a, b = pts[0], pts[-1]
    # extend in case the guesses were off by more than the margin
    while pred(a - 1):
        a -= 1
    while pred(b + 1):
        b += 1
    return a, b


class OraclePlan:
    """Constant-Q sliCQ plan for real signals (Section 3, Table 1; Section 4).

    Bands 0..K+1 (DC, constant-Q bands 1..K, Nyquist) are the stored bands;
    bands K+2..2K+1 are their mirrors g_{2K+2-k}[j] = g_k[2N - j] and enter
    only through the frame operator and, for synthesis, through conjugate
    coefficients.
    """

    def __init__(self, fs: float, fmin: float, fmax: float, bins_per_octave: int,
                 slice_len: int, transition: int, min_win: float = 16.0,
                 dual_slice: str = "canonical", window: str = "hann", scale: str = "cq",
                 slicing: str = "tukey", m_policy: str = "pow2"):
        fs = float(fs)
        fmin = float(fmin)
        fmax = float(fmax)
        B = int(bins_per_octave)
        two_n = int(slice_len)
        Mt = int(transition)
        if not (fs > 0 and 0 < fmin < fmax and fmin < fs / 2 and B >= 1):
            raise ValueError("need fs > 0, 0 < fmin < fmax, fmin < fs/2, B >= 1")
        if two_n < 16 or two_n & (two_n - 1):
            raise ValueError("slice length 2N must be a power of two >= 16")
        N = two_n // 2
        if not (0 < Mt < N) or (N - Mt) % 2:
            raise ValueError("transition M needs 0 < M < N and N - M even")
        if dual_slice not in ("canonical", "indicator"):
            raise ValueError("dual_slice is 'canonical' or 'indicator'")
        window_value(window, 0.0)
        if scale not in ("cq", "mel", "bark"):
            raise ValueError("scale is 'cq', 'mel' or 'bark'")
        if slicing not in ("tukey", "sqrt_tukey"):
            raise ValueError("slicing is 'tukey' or 'sqrt_tukey'")
        if m_policy not in ("pow2", "rect", "smooth"):
            raise ValueError("m_policy is 'pow2', 'rect' or 'smooth'")
        self.window, self.scale, self.slicing, self.m_policy = window, scale, slicing, m_policy
        self.fs, self.fmin, self.fmax, self.B = fs, fmin, fmax, B
        self.two_n, self.N, self.M = two_n, N, Mt
        self.min_win = float(min_win)
        self.dual_slice = dual_slice
        self.Q = q_factor(B)

        # --- centres and bandwidths (Table 1; readings on K and min_win) ---
        K0 = 1 + math.ceil(B * math.log2(fmax / fmin) - 1e-12)
        bw_min = self.min_win * fs / two_n
        if scale == "cq":
            xi = [fmin * 2.0 ** ((k - 1) / B) for k in range(1, K0 + 1)]
            om = [max(x / self.Q, bw_min) for x in xi]
        else:
            # as many bands as constant-Q would place, equally spaced on the
            # scale from fmin to fmax; the bandwidth is the distance between
            # the two neighbouring centres, which for constant-Q is xi_k / Q
            fwd, inv = SCALES[scale]
            u0, u1 = fwd(fmin), fwd(fmax)
            du = (u1 - u0) / max(K0 - 1, 1)
            ext = [inv(u0 + (k - 1) * du) for k in range(0, K0 + 2)]   # xi_0 .. xi_{K0+1}
            xi = ext[1:K0 + 1]
            om = [max(ext[k + 1] - ext[k - 1], bw_min) for k in range(1, K0 + 1)]
        K = K0
        while K >= 1 and not (xi[K - 1] + om[K - 1] / 2 < fs / 2):
            K -= 1
        if K < 1:
            raise ValueError("no constant-Q band fits below Nyquist")
        self.K0, self.K = K0, K
        self.xi = np.array(xi[:K])
        self.omega = np.array(om[:K])

        bands: List[BandTable] = []
        # DC band: plateau around 0 of radius xi_1, flank width min(Omega_1/2, xi_1)
        R0 = xi[0]
        w0 = min(om[0] / 2, R0)
        bands.append(self._plateau_band(0, 0, R0, w0, 0.0, 2.0 * xi[0]))
        # constant-Q bands 1..K
        for k in range(1, K + 1):
            bands.append(self._hann_band(k, xi[k - 1], om[k - 1]))

        # Nyquist band: plateau around N of radius fs/2 - xi_K
        RN = fs / 2 - xi[K - 1]
        wN = min(om[K - 1] / 2, RN)
        bands.append(self._plateau_band(K + 1, N, RN, wN, fs / 2, fs - 2 * xi[K - 1]))
        if m_policy == "rect":
            # rectangular representation (Section 6): one M for every band,
            # the smallest power of two that holds the widest support
            Mr = max(b.M for b in bands)
            for b in bands:
                b.M = Mr
        elif m_policy == "smooth":
            # equation framecond1 asks only M_k >= |J_k| (integer); Algorithm 3
            # places slice m at (m - 1) M_k / 2, so M_k is even: the smallest
            # even number 2^a, 3 2^a or 5 2^a that holds the support
            for b in bands:
                b.M = smooth_even_at_least(b.length)
        # validity of the real-signal band layout
        for b in bands:
            if b.length == 0:
                raise ValueError("band %d has empty support; raise min_win" % b.k)
        for b in bands[1:K + 1]:
            if b.start < 1 or b.start + b.length - 1 > N - 1:
                raise ValueError("a constant-Q band reaches bin 0 or bin N; raise fmin or lower min_win")
        # mirrored bands K+2..2K+1: g_{2K+2-k}[j] = g_k[2N-j]
        mirrors = []
        for k in range(K + 2, 2 * K + 2):
            src = bands[2 * K + 2 - k]
            start = -(src.start + src.length - 1)
            mirrors.append(BandTable(k, start, src.g[::-1].copy(), src.M,
                                     xi=fs - src.xi, omega=src.omega))
        self.bands = bands
        self.all_bands = bands + mirrors
        self._finish_dual()
        self._slicing_windows()

    # -- band constructors ---------------------------------------------------
    def _hann_band(self, k, xi_k, om_k) -> BandTable:
        """Band k: the window shape (Hann unless ``window`` says otherwise) on
        the open interval |nu - xi_k| < Omega_k / 2."""
        fs, two_n = self.fs, self.two_n

        def x_of(j):
            return (j * fs / two_n - xi_k) / om_k

        def inside(j):
            x = x_of(j)
            return -0.5 < x < 0.5

        glo = int(math.floor((xi_k - om_k / 2) * two_n / fs))
        ghi = int(math.ceil((xi_k + om_k / 2) * two_n / fs))
        iv = _interval(inside, glo, ghi)
        if iv is None:
            return BandTable(k, 0, np.zeros(0), 2, xi=xi_k, omega=om_k)
        a, b = iv
        g = np.array([window_value(self.window, x_of(j)) for j in range(a, b + 1)])
        return BandTable(k, a, g, max(2, _next_pow2(b - a + 1)), xi=xi_k, omega=om_k)

    def _plateau_band(self, k, centre_bin, R, w, xi_hz, om_hz) -> BandTable:
        """Plateau P(d; R, w) in the distance d (Hz) from the centre bin."""
        fs, two_n = self.fs, self.two_n

        def dist(j):
            return abs(j - centre_bin) * fs / two_n

        e = 0
        while (e + 1) * fs / two_n < R:
            e += 1
        a, b = centre_bin - e, centre_bin + e
        d = np.array([dist(j) for j in range(a, b + 1)])
        g = np.where(d <= R - w, 1.0,
                     0.5 + 0.5 * np.cos(math.pi * (d - R + w) / w))
        return BandTable(k, a, g, max(2, _next_pow2(b - a + 1)), xi=xi_hz, omega=om_hz)

    # -- frame operator, dual, windows --------------------------------------
    def _finish_dual(self):
        two_n = self.two_n
        D = np.zeros(two_n)
        for b in self.all_bands:
            np.add.at(D, b.bins() % two_n, b.M * b.g ** 2)
        if not np.all(D > 0):
            raise ValueError("frame condition fails: D has a zero (Proposition 2)")
        self.D = D
        for b in self.all_bands:
            b.gd = b.g / D[b.bins() % two_n]

    def _slicing_windows(self):
        N, Mt = self.N, self.M
        t = np.arange(-N, N)           # index j = t + N
        a = np.abs(t)
        flat = (N - Mt) // 2
        h = np.where(a <= flat, 1.0,
                     np.where(a < (N + Mt) / 2,
                              0.5 + 0.5 * np.cos(math.pi * (a - flat) / Mt), 0.0))
        if getattr(self, "slicing", "tukey") == "sqrt_tukey":
            # the other slicing design of Section 4.3: sum_m h_m^2 = 1, so the
            # same windows serve in the overlap-add (the canonical dual is h_0)
            h = np.sqrt(h)
        self.h0 = h
        if self.dual_slice == "indicator":
            self.hd = (h != 0).astype(np.float64)
        else:
            # sum over the translates by -N, 0, N that meet [-N, N)
            sq = h ** 2
            den = sq.copy()
            den[N:] += sq[:N]      # translate by +N: h_0[t - N] for t >= 0
            den[:N] += sq[N:]      # translate by -N: h_0[t + N] for t < 0
            self.hd = np.where(h != 0, h / np.where(den > 0, den, 1.0), 0.0)

    # -- summaries --------------------------------------------------------------
    @property
    def nbands(self) -> int:
        return self.K + 2

    @property
    def Ms(self) -> np.ndarray:
        return np.array([b.M for b in self.bands], dtype=np.int64)

    @property
    def offsets(self) -> np.ndarray:
        """off_k = sum_{k' < k} M_k' (band-major packing of the stored bands)."""
        return np.concatenate([[0], np.cumsum(self.Ms)[:-1]]).astype(np.int64)

    @property
    def coefs_per_slice(self) -> int:
        return int(self.Ms.sum())


def plan_from_tables(two_n: int, transition: int, bands, dual_slice: str = "canonical"):
    """Plan from explicit band tables, for complex signals and any band set.

    ``bands`` is a list of (start, g, M) with g over {start, ..., start+len-1}
    (circular). All listed bands are analysed; there is no mirroring. Used for
    the textbook special cases (single band, uniform STFT bands).
    """
    p = OraclePlan.__new__(OraclePlan)
    p.two_n = int(two_n)
    p.N = p.two_n // 2
    p.M = int(transition)
    p.dual_slice = dual_slice
    p.K = None
    tabs = []
    for k, (start, g, M) in enumerate(bands):
        g = np.asarray(g, dtype=np.float64)
        if len(g) > M or p.two_n % M:
            raise ValueError("need |J_k| <= M_k and M_k | 2N")
        tabs.append(BandTable(k, int(start), g, int(M)))
    p.bands = tabs
    p.all_bands = tabs
    p._finish_dual()
    p._slicing_windows()
    return p
