"""Pins of the oracle's 9/7 lifting DWT (T.800 Annex F) and subband gains."""
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "t800_97_taps.txt")


def _taps():
    d = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        d[k] = np.array([float(t) for t in v])
    return d


def _impulse_response(ref, band_high, n=64):
    """Analysis taps seen by one mid-signal output coefficient (1-D, FP64)."""
    out = []
    c = n // 4 if not band_high else n // 2 + n // 4
    for k in range(n):
        e = np.zeros((1, n))
        e[0, k] = 1.0
        y = ref.dwt(e.T, 1, f64=True).T   # column transform on an n x 1 signal
        out.append(y[0, c])
    return np.array(out)


def test_analysis_taps_match_t800(ref):
    t = _taps()
    h0 = _impulse_response(ref, False)
    h1 = _impulse_response(ref, True)
    c0 = 2 * (64 // 4)          # the low output i reads input samples around 2i
    c1 = 2 * (64 // 4) + 1      # the high output i reads around 2i+1
    for k, v in enumerate(t["lowpass"]):
        assert h0[c0 + k] == pytest.approx(v, abs=1e-12)
        assert h0[c0 - k] == pytest.approx(v, abs=1e-12)
    for k, v in enumerate(t["highpass"]):
        assert h1[c1 + k] == pytest.approx(v, abs=1e-12)
        assert h1[c1 - k] == pytest.approx(v, abs=1e-12)
    # support: 9 and 7 taps, nothing else
    assert np.count_nonzero(np.abs(h0) > 1e-14) == 9
    assert np.count_nonzero(np.abs(h1) > 1e-14) == 7
    # normalisation: DC gain 1 (low), zero DC and Nyquist gain 2 (high)
    assert h0.sum() == pytest.approx(1.0, abs=1e-12)
    assert h1.sum() == pytest.approx(0.0, abs=1e-12)
    assert abs(np.sum(h1 * (-1.0) ** np.arange(64))) == pytest.approx(2.0, abs=1e-12)


@pytest.mark.parametrize("shape,L", [((2, 2), 1), ((3, 5), 1), ((7, 2), 1), ((17, 33), 4), ((64, 64), 6),
                                      ((181, 360), 5), ((91, 180), 5), ((1, 9), 0), ((40, 3), 1)])
def test_perfect_reconstruction(ref, shape, L):
    rng = np.random.default_rng(sum(shape) + L)
    x = rng.standard_normal(shape)
    L = ref.levels_eff(*shape, L)
    y = ref.dwt(ref.dwt(x, L, f64=True), L, inverse=True, f64=True)
    assert np.abs(y - x).max() <= 1e-12 * max(1.0, np.abs(x).max())
    xf = x.astype(np.float32)
    yf = ref.dwt(ref.dwt(xf, L), L, inverse=True)
    assert np.abs(yf.astype(np.float64) - xf).max() <= 2e-6 * np.abs(xf).max() * max(L, 1)


def test_fp32_tracks_fp64(ref):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((121, 250)).astype(np.float32)
    a = ref.dwt(x, 5).astype(np.float64)
    b = ref.dwt(x.astype(np.float64), 5, f64=True)
    assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max()


@pytest.mark.parametrize("deg", [0, 1, 2, 3])
def test_vanishing_moments(ref, deg):
    """The 9/7 analysis high-pass has 4 vanishing moments: polynomials of
    degree <= 3 give zero detail coefficients away from the borders."""
    n = 128
    t = np.arange(n, dtype=np.float64) / n
    x = np.tile(t ** deg, (1, 1)).T          # n x 1 column signal
    y = ref.dwt(x, 1, f64=True)[:, 0]
    hi = y[n // 2:]
    assert np.abs(hi[4:-4]).max() < 1e-12


def test_degree4_not_annihilated(ref):
    n = 128
    t = np.arange(n, dtype=np.float64) / n
    y = ref.dwt((t ** 4)[:, None], 1, f64=True)[:, 0]
    assert np.abs(y[n // 2 + 4: -4]).max() > 1e-9


def test_constant_field(ref):
    """A constant field transforms to the same constant in LL and zero
    elsewhere (DC gain 1, symmetric extension keeps the edges exact)."""
    x = np.full((37, 53), 2.5)
    L = ref.levels_eff(37, 53, 5)
    y = ref.dwt(x, L, f64=True)
    h, w = 37, 53
    for _ in range(L):
        h, w = (h + 1) // 2, (w + 1) // 2
    assert np.abs(y[:h, :w] - 2.5).max() < 1e-12
    y[:h, :w] = 0
    assert np.abs(y).max() < 1e-12


def test_alternating_columns(ref):
    """(-1)^j along rows: all energy goes to the horizontal high band with
    magnitude 2 (Nyquist gain 2), nothing to the low band."""
    x = np.tile((-1.0) ** np.arange(16), (8, 1))
    y = ref.dwt(x, 1, f64=True)
    assert np.abs(y[:, :8]).max() < 1e-12
    assert np.abs(np.abs(y[:4, 8:]) - 2.0).max() < 1e-12


def test_levels_clamp(ref):
    assert ref.levels_eff(181, 360, 5) == 5
    assert ref.levels_eff(16, 1000, 9) == 4
    assert ref.levels_eff(17, 1000, 9) == 4
    assert ref.levels_eff(1, 100, 5) == 0
    assert ref.levels_eff(2, 2, 5) == 1


def test_band_gains_closed_form(ref):
    """g_b = round(log2 ||synthesis basis||): LL_l -> l, HL_l/LH_l -> l-1,
    HH_l -> l-2 for the JPEG2000 9/7 normalisation."""
    for l in range(1, 9):
        assert ref.band_log2_gain(l, 0) == l
        assert ref.band_log2_gain(l, 1) == l - 1
        assert ref.band_log2_gain(l, 2) == l - 1
        assert ref.band_log2_gain(l, 3) == l - 2
    assert ref.band_log2_gain(0, 0) == 0
    # the exponents are not near a rounding boundary
    for l in range(1, 9):
        for o in range(4):
            f = np.log2(ref.band_norm(l, o))
            assert abs(f - np.round(f)) < 0.45


@pytest.mark.parametrize("level,orient", [(1, 1), (1, 2), (1, 3), (2, 3), (3, 0), (3, 1), (4, 2)])
def test_band_norm_by_2d_impulse(ref, level, orient):
    """The separable gain equals the norm of a 2-D impulse pushed through the
    FP32 2-D inverse transform (an independent path: 2-D, FP32)."""
    n = 256
    L = level
    sizes = [n]
    for _ in range(L):
        sizes.append((sizes[-1] + 1) // 2)
    hl, hp = sizes[L], sizes[L - 1]
    c = np.zeros((n, n), np.float32)
    mid = hl // 2
    if orient == 0:
        c[mid, mid] = 1
    elif orient == 1:      # HL: horizontal high -> columns in the high half
        c[mid, hl + (hp - hl) // 2] = 1
    elif orient == 2:
        c[hl + (hp - hl) // 2, mid] = 1
    else:
        c[hl + (hp - hl) // 2, hl + (hp - hl) // 2] = 1
    y = ref.dwt(c, L, inverse=True).astype(np.float64)
    assert np.sqrt((y ** 2).sum()) == pytest.approx(ref.band_norm(level, orient), rel=1e-5)
