"""Pins of the oracle's plan against what the paper fixes (Section 3, Table 1,
Proposition 2, Section 4.3). None of these re-types the oracle's own formula:
each checks an independent characterisation."""
import json
import math
import os

import numpy as np
import pytest

from oracle import OraclePlan, brute
from workloads import PRESETS

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def preset_plan(name, **kw):
    p = PRESETS[name]
    return OraclePlan(p.fs, p.fmin, p.fmax, p.bins_per_octave, p.slice_len, p.transition, **kw)


TINY = dict(fs=64.0, fmin=4.0, fmax=16.0, bins_per_octave=3, slice_len=64, transition=8, min_win=0.0)


@pytest.mark.parametrize("name", list(PRESETS))
def test_bandwidth_is_neighbour_spacing(name):
    # Section 3: Omega_k = xi_{k+1} - xi_{k-1} for interior bands gives constant Q.
    pl = preset_plan(name)
    xi, om = pl.xi, pl.omega
    k = np.arange(1, pl.K - 1)
    unwidened = om[k] > pl.min_win * pl.fs / pl.two_n
    spacing = xi[k + 1] - xi[k - 1]
    np.testing.assert_allclose(om[k][unwidened], spacing[unwidened], rtol=1e-12)
    np.testing.assert_allclose(xi[k] / spacing, pl.Q, rtol=1e-12)


@pytest.mark.parametrize("B", [1, 3, 12, 24, 48, 96])
def test_q_closed_forms(B):
    # Q = (2^{1/B} - 2^{-1/B})^{-1} equals 2^{1/B} / (2^{2/B} - 1)
    pl = OraclePlan(44100, 100, 1000, B, 1 << 18, 512, min_win=0)
    assert math.isclose(pl.Q, 2 ** (1 / B) / (2 ** (2 / B) - 1), rel_tol=1e-13)


@pytest.mark.parametrize("name", list(PRESETS))
def test_centres_geometric(name):
    pl = preset_plan(name)
    assert pl.xi[0] == pl.fmin
    r = pl.xi[1:] / pl.xi[:-1]
    np.testing.assert_allclose(r, 2 ** (1 / pl.B), rtol=1e-13)
    if pl.K > pl.B:
        assert math.isclose(pl.xi[pl.B], 2 * pl.fmin, rel_tol=1e-13)   # one octave up


def test_k_choice_below_and_at_nyquist():
    # fmax below Nyquist: smallest K with xi_K >= xi_max (Section 3)
    pl = preset_plan("c1")
    assert pl.xi[-1] >= pl.fmax > pl.xi[-2]
    assert pl.K == pl.K0
    # fmax = fs/2 cannot satisfy xi_K < fs/2 with the last band inside: K is reduced
    for name in ("c2", "c3"):
        pl = preset_plan(name)
        assert pl.K < pl.K0
        assert pl.xi[-1] + pl.omega[-1] / 2 < pl.fs / 2
        nxt = pl.xi[-1] * 2 ** (1 / pl.B)
        assert nxt + max(nxt / pl.Q, pl.min_win * pl.fs / pl.two_n) / 2 >= pl.fs / 2


@pytest.mark.parametrize("name", list(PRESETS) + ["tiny"])
def test_supports_and_lattice(name):
    pl = OraclePlan(**TINY) if name == "tiny" else preset_plan(name)
    binw = pl.fs / pl.two_n
    for b in pl.bands[1:pl.K + 1]:
        # support: the bins strictly inside (xi_k - Omega_k/2, xi_k + Omega_k/2)
        lo = (b.xi - b.omega / 2) / binw
        hi = (b.xi + b.omega / 2) / binw
        expect = [j for j in range(int(lo) - 2, int(hi) + 3) if lo < j < hi]
        assert list(b.bins()) == expect
        assert np.all(b.g > 0) and np.all(b.g <= 1)
        # H peaks at the centre: the largest value sits on the bin nearest xi_k
        assert abs(b.bins()[np.argmax(b.g)] - b.xi / binw) <= 0.5 + 1e-9
    for b in pl.all_bands:
        # framecond1: L/a_k = M_k >= |J_k|; M_k divides 2N
        assert b.M >= b.length and pl.two_n % b.M == 0 and b.M & (b.M - 1) == 0


@pytest.mark.parametrize("name", ["c1", "c4", "c5"])
def test_plateau_flanks_partition(name):
    # DC and Nyquist plateaus meet the first / last Hann band as a partition of unity
    pl = preset_plan(name)
    full = {b.k: brute.band_full(b, pl.two_n) for b in pl.bands}
    K = pl.K
    j = np.arange(pl.two_n // 2 + 1)
    nu = j * pl.fs / pl.two_n
    dc_flank = (nu > pl.xi[0] - min(pl.omega[0] / 2, pl.xi[0])) & (nu < pl.xi[0])
    np.testing.assert_allclose((full[0] + full[1])[j[dc_flank]], 1.0, atol=1e-12)
    ny_flank = (nu > pl.xi[-1]) & (nu < pl.xi[-1] + pl.omega[-1] / 2)
    assert ny_flank.any()
    np.testing.assert_allclose((full[K] + full[K + 1])[j[ny_flank]], 1.0, atol=1e-12)
    # the plateaus are flat at their centres
    assert full[0][0] == 1.0 and full[K + 1][pl.two_n // 2] == 1.0


@pytest.mark.parametrize("name", ["c1", "c5", "tiny"])
def test_mirrored_bands(name):
    pl = OraclePlan(**TINY) if name == "tiny" else preset_plan(name)
    K, n2 = pl.K, pl.two_n
    assert len(pl.all_bands) == 2 * K + 2
    for k in range(1, K + 1):
        g = brute.band_full(pl.all_bands[k], n2)
        gm = brute.band_full(pl.all_bands[2 * K + 2 - k], n2)
        np.testing.assert_array_equal(gm, g[(-np.arange(n2)) % n2])
    for k in (0, K + 1):   # DC and Nyquist are their own mirrors
        g = brute.band_full(pl.all_bands[k], n2)
        np.testing.assert_array_equal(g, g[(-np.arange(n2)) % n2])


@pytest.mark.parametrize("kw", [TINY, dict(TINY, min_win=3.0), dict(fs=100.0, fmin=6.0, fmax=40.0,
                                bins_per_octave=4, slice_len=128, transition=16, min_win=4.0)])
def test_frame_operator_is_diagonal(kw):
    # Proposition 2: S = F^H diag(D) F with D = sum_k M_k g_k^2 > 0
    pl = OraclePlan(**kw)
    assert np.all(pl.D > 0)
    S = brute.frame_operator(pl)
    E = brute.idft_matrix(pl.two_n)
    np.testing.assert_allclose(S, E @ np.diag(pl.D) @ E.conj().T, atol=1e-12 * pl.D.max())


def test_canonical_dual_atoms():
    # equation candual: S^{-1} phi_{n,k} are the atoms of the dual windows g_k / D
    pl = OraclePlan(**dict(TINY, min_win=2.0))
    for d, a in zip(brute.dual_atoms(pl), brute.atoms(pl, window="gd")):
        np.testing.assert_allclose(d, a, atol=1e-13)


@pytest.mark.parametrize("N,M", [(32, 8), (32, 30), (4096, 1024), (8192, 2048), (16, 2)])
@pytest.mark.parametrize("kind", ["canonical", "indicator"])
def test_slicing_windows(N, M, kind):
    pl = OraclePlan(2.0 * N, 4.0, N / 2, 2, 2 * N, M, min_win=2.0, dual_slice=kind)
    h, hd = pl.h0, pl.hd
    # essential length N with transitions M: N + M - 1 non-zero samples
    assert np.count_nonzero(h) == N + M - 1
    assert h[N] == 1.0 and np.all(h <= 1)
    np.testing.assert_array_equal(h[1:], h[1:][::-1])        # symmetric about t = 0
    # equation BUPU: sum_m T_{mN} h_0 = 1 on every sample of a long circle
    L = 8 * N
    s = np.zeros(L)
    sd = np.zeros(L)
    for m in range(L // N):
        idx = (np.arange(2 * N) + (m - 1) * N) % L
        np.add.at(s, idx, h)
        np.add.at(sd, idx, h * hd)
    np.testing.assert_allclose(s, 1.0, atol=2e-16 * 4)
    # equation dualwincond: sum_m T_{mN} (h_0 conj(h~_0)) = 1
    np.testing.assert_allclose(sd, 1.0, atol=1e-15)
    assert np.all(hd[h == 0] == 0)                            # dual supported on supp h_0


def test_transposition_fact_golden():
    # Section 6: at 48 bins per octave, 2 semitones are 8 bins
    with open(os.path.join(GOLDEN, "paper_facts.json")) as fh:
        facts = json.load(fh)
    t = facts["transposition"]
    pl = OraclePlan(44100, 50, 20000, t["bins_per_octave"], 65536, 16384)
    r = pl.xi[t["bins"]:] / pl.xi[:-t["bins"]]
    np.testing.assert_allclose(r, 2 ** (t["semitones"] / 12), rtol=1e-13)


@pytest.mark.parametrize("bad", [
    dict(fs=44100, fmin=0, fmax=100, bins_per_octave=12, slice_len=4096, transition=512),
    dict(fs=44100, fmin=200, fmax=100, bins_per_octave=12, slice_len=4096, transition=512),
    dict(fs=44100, fmin=100, fmax=1000, bins_per_octave=12, slice_len=4000, transition=512),
    dict(fs=44100, fmin=100, fmax=1000, bins_per_octave=12, slice_len=4096, transition=2048),
    dict(fs=44100, fmin=100, fmax=1000, bins_per_octave=12, slice_len=4096, transition=511),
    dict(fs=44100, fmin=5, fmax=1000, bins_per_octave=12, slice_len=256, transition=32),
])
def test_invalid_parameters(bad):
    with pytest.raises(ValueError):
        OraclePlan(**bad)


DERIVED = json.load(open(os.path.join(GOLDEN, "derived_constants.json")))


@pytest.mark.parametrize("name", list(PRESETS))
def test_derived_constants(name):
    # constants an independent pre-build computation of the same readings gave
    # (K below Nyquist, minimal filter length 16 bins, power-of-two M_k)
    import collections
    d = DERIVED[name]
    pl = preset_plan(name)
    assert math.isclose(pl.Q, d["Q"], abs_tol=5e-5)
    assert (pl.K0, pl.K, pl.nbands) == (d["K0"], d["K"], d["nbands"])
    assert int(np.sum(pl.xi / pl.Q < pl.min_win * pl.fs / pl.two_n)) == d["widened"]
    assert sum(b.length for b in pl.bands) == d["sum_J"]
    assert pl.coefs_per_slice == d["sum_M"]
    hist = collections.Counter(str(int(b.M)) for b in pl.bands)
    assert dict(hist) == d["M_hist"]
    assert (pl.bands[0].M, pl.bands[0].length) == (d["M_dc"], d["J_dc"])
    assert (pl.bands[-1].M, pl.bands[-1].length) == (d["M_nyq"], d["J_nyq"])
    assert abs(pl.D.min() - d["D_min"]) <= 0.01 and abs(pl.D.max() - d["D_max"]) <= 0.01
    assert abs(pl.xi[-1] - d["xi_K"]) <= 0.05


@pytest.mark.parametrize("name", list(PRESETS))
def test_minimal_filter_length(name):
    # Section 5.3: filters shorter than about 16 samples change the
    # coefficients visibly, so every constant-Q band is at least min_win bins
    # wide. Checked on the band tables themselves, not on the bandwidth
    # formula: the support of a Hann band is the open interval of width
    # Omega_k around xi_k, so it spans at least min_win - 1 whole bins, is
    # centred on xi_k, and is never wider than the bound requires.
    pl = preset_plan(name)
    binw = pl.fs / pl.two_n
    for b in pl.bands[1:pl.K + 1]:
        assert b.length >= pl.min_win - 1, (b.k, b.length)
        centre = (b.start + b.start + b.length - 1) / 2 * binw
        assert abs(centre - b.xi) <= binw, (b.k, centre, b.xi)
        cq_bins = b.xi / pl.Q / binw                 # constant-Q width in bins (Table 1)
        need = max(cq_bins, pl.min_win)
        # integer points strictly inside an open interval of width `need`
        assert need - 1 - 1e-9 <= b.length <= need + 1 + 1e-9, (b.k, b.length, need)
    # without the bound the narrowest bands of the long-slice presets hold
    # fewer bins than the bound asks for (the widening is doing work)
    raw = preset_plan("c2", min_win=0.0)
    assert min(b.length for b in raw.bands[1:raw.K + 1]) < 8
    with pytest.raises(ValueError):
        preset_plan("c5", min_win=0.0)            # some bands would hold no bin at all


def test_minimal_filter_length_matches_paper_threshold():
    # the default bound is the length the paper calls largely equivalent
    facts = json.load(open(os.path.join(GOLDEN, "paper_facts.json")))["minimal_filter_length"]
    pl = preset_plan("c1")
    assert pl.min_win == facts["equivalent_above"]
