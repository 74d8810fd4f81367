"""Seeded synthetic inputs and named parameter sets for the sliCQ workloads.

This module is shared by the FP64 oracle, the tests and the benchmark. It
holds no arithmetic of the transform itself: only signal generators and
parameter presets. Every generator draws from numpy's PCG64 with an explicit
seed and renders in float64.

The paper times random signals at 44.1 kHz (Section 5.2) and measures
approximation on random complex signals and music excerpts (Section 5.3);
none of its signals ship with it, so these seeded stand-ins take their place:

* ``noise_plus_sines``: unit-variance white Gaussian noise plus five
  sinusoids (frequency uniform in [110, 8000] Hz, amplitude uniform in
  [0.1, 1], phase uniform in [0, 2 pi)).
* ``pink_plus_tones``: pink noise (white Gaussian spectrum shaped by
  f^-1/2, DC removed, unit variance) plus consecutive 0.5 s harmonic notes
  (f0 uniform in [55, 880] Hz, partials h = 1..10 below Nyquist with
  amplitude 0.5/h and random phase, 5 ms raised-cosine fades).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Preset", "PRESETS", "rng", "noise_plus_sines", "pink_noise",
    "harmonic_tones", "pink_plus_tones", "batch_lengths", "make_c1", "make_c2",
    "make_c3", "make_c3_cut", "make_c4", "make_c5_stream",
]


@dataclasses.dataclass(frozen=True)
class Preset:
    """Transform parameters of one named workload (Section 3 and 4 notation)."""
    name: str
    fs: float            # sampling rate xi_s in Hz
    fmin: float          # xi_min in Hz
    fmax: float          # xi_max in Hz
    bins_per_octave: int  # B
    slice_len: int       # 2N
    transition: int      # M, Tukey transition length
    dtype: str           # arithmetic type of the GPU path for this workload


PRESETS = {
    "c1": Preset("c1", 44100.0, 110.0, 11025.0, 12, 8192, 1024, "f64"),
    "c2": Preset("c2", 44100.0, 32.7, 22050.0, 48, 65536, 8192, "f32"),
    "c3": Preset("c3", 44100.0, 41.2, 22050.0, 24, 32768, 4096, "f32"),
    "c4": Preset("c4", 44100.0, 65.4, 16000.0, 36, 16384, 2048, "f32"),
    "c5": Preset("c5", 48000.0, 27.5, 20000.0, 96, 16384, 2048, "f32"),
}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def noise_plus_sines(T: int, fs: float, seed: int, n_sines: int = 5) -> np.ndarray:
    """White N(0,1) noise plus ``n_sines`` random sinusoids, float64."""
    g = rng(seed)
    x = g.standard_normal(T)
    t = np.arange(T, dtype=np.float64) / fs
    f = g.uniform(110.0, 8000.0, n_sines)
    a = g.uniform(0.1, 1.0, n_sines)
    p = g.uniform(0.0, 2.0 * math.pi, n_sines)
    for i in range(n_sines):
        x += a[i] * np.sin(2.0 * math.pi * f[i] * t + p[i])
    return x


def pink_noise(T: int, g: np.random.Generator) -> np.ndarray:
    """Unit-variance pink noise: white spectrum times f^-1/2, DC bin zeroed."""
    if T == 0:
        return np.zeros(0)
    w = g.standard_normal(T)
    W = np.fft.rfft(w)
    f = np.arange(W.shape[0], dtype=np.float64)
    shape = np.zeros_like(f)
    shape[1:] = 1.0 / np.sqrt(f[1:])
    x = np.fft.irfft(W * shape, n=T)
    sd = x.std()
    return x / sd if sd > 0 else x


def harmonic_tones(T: int, fs: float, g: np.random.Generator,
                   note_s: float = 0.5, fade_s: float = 0.005) -> np.ndarray:
    """Consecutive harmonic notes with 1/h partial amplitudes."""
    x = np.zeros(T)
    note = int(round(note_s * fs))
    fade = max(1, int(round(fade_s * fs)))
    ramp = 0.5 - 0.5 * np.cos(math.pi * (np.arange(fade) + 0.5) / fade)
    for start in range(0, T, note):
        n = min(note, T - start)
        f0 = g.uniform(55.0, 880.0)
        t = np.arange(n, dtype=np.float64) / fs
        seg = np.zeros(n)
        for h in range(1, 11):
            ph = g.uniform(0.0, 2.0 * math.pi)
            if h * f0 < fs / 2:
                seg += (0.5 / h) * np.sin(2.0 * math.pi * h * f0 * t + ph)
        env = np.ones(n)
        m = min(fade, n)
        env[:m] *= ramp[:m]
        env[n - m:] *= ramp[:m][::-1]
        x[start:start + n] = seg * env
    return x


def pink_plus_tones(T: int, fs: float, seed: int) -> np.ndarray:
    g = rng(seed)
    return pink_noise(T, g) + harmonic_tones(T, fs, g)


def batch_lengths(n: int, fs: float, seed: int, lo_s: float = 5.0, hi_s: float = 30.0) -> np.ndarray:
    """Signal lengths uniform in [lo_s*fs, hi_s*fs] samples (integers)."""
    g = rng(seed)
    return g.integers(int(round(lo_s * fs)), int(round(hi_s * fs)) + 1, size=n)


# --- the named workloads -------------------------------------------------

def make_c1() -> np.ndarray:
    """2^16 samples at 44.1 kHz of noise plus 5 sines, seed 1 (float64)."""
    return noise_plus_sines(1 << 16, 44100.0, 1)


def make_c2(seconds: float = 60.0) -> np.ndarray:
    """Stereo pink noise plus tones, seeds 2 (left) and 3 (right): shape (2, T)."""
    T = int(round(seconds * 44100.0))
    return np.stack([pink_plus_tones(T, 44100.0, 2), pink_plus_tones(T, 44100.0, 3)])


def make_c3(n_signals: int = 256, seed: int = 4, lo_s: float = 5.0, hi_s: float = 30.0):
    """Ragged batch: list of float64 signals, lengths uniform in [5 s, 30 s]."""
    lens = batch_lengths(n_signals, 44100.0, seed, lo_s, hi_s)
    return [pink_plus_tones(int(T), 44100.0, seed * 1_000_003 + i) for i, T in enumerate(lens)]


def make_c3_cut(n_signals: int = 256, seed: int = 4):
    """The ragged batch's lengths (as ``make_c3`` draws them) with content cut
    at seeded offsets from one 60 s pink-plus-tones recording: (lengths,
    offsets, recording). Rendering 256 distinct recordings takes minutes of
    host time, and the transform's cost does not depend on the content."""
    lens = [int(t) for t in batch_lengths(n_signals, 44100.0, seed)]
    base = pink_plus_tones(int(60 * 44100), 44100.0, 4_000_012)
    g = rng(seed)
    offs = [int(g.integers(0, len(base) - t + 1)) for t in lens]
    return lens, offs, base


def make_c4(batch: int = 32, T: int = 264600, target: bool = False) -> np.ndarray:
    """Batch of noise-plus-sines signals; seeds 5+b (input) or 1005+b (target)."""
    base = 1005 if target else 5
    return np.stack([noise_plus_sines(T, 44100.0, base + 1000 * b if b else base) for b in range(batch)])


def make_c5_stream(stream_id: int, T: int) -> np.ndarray:
    """Signal of one stream of the streaming workload (fs = 48 kHz)."""
    return pink_plus_tones(T, 48000.0, 5_000_000 + stream_id)
