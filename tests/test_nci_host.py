"""Host logic of the package's numerical-Cherenkov module (no GPU): its
growth-rate fit and Eq. (17) curve against the oracle's independent ones,
and the spectrum peak picker."""
import numpy as np

from oracle import spectral
from oracle.growth import growth_rate as oracle_growth
from paper_1412_2480_amd import nci


def test_growth_rate_agrees_with_oracle_fit():
    rng = np.random.default_rng(0)
    t = np.arange(600) * 0.5
    for rate in (0.02, 0.1, 0.3):
        w = 1e-8 * (1 + 0.1 * rng.random(t.size)) * np.exp(2 * rate * t)
        w = np.minimum(w, 1.0) + 1e-8 * rng.random(t.size)
        a, b = nci.growth_rate(t, w), oracle_growth(t, w)
        assert a is not None and b is not None
        assert abs(a["rate"] - b["rate"]) <= 1e-10 * b["rate"]
        assert abs(a["rate"] - rate) <= 0.05 * rate
        assert (a["t0"], a["t1"], a["samples"]) == (b["t0"], b["t1"], b["samples"])
    flat = 1e-6 * (1 + 0.01 * rng.random(t.size))
    assert nci.growth_rate(t, flat) is None and oracle_growth(t, flat) is None


def test_cherenkov_locus_matches_oracle_closed_form():
    V = np.sqrt(1 - 1e-4)
    for sigma in (0.5, 0.8, 1.0):
        kx = np.linspace(0.01, np.pi, 300)
        a = nci.cherenkov_locus(kx, sigma, V)
        b = spectral.cherenkov_ky(kx, V, sigma, sigma)
        assert np.array_equal(np.isfinite(a), np.isfinite(b))
        ok = np.isfinite(a)
        assert np.allclose(a[ok], b[ok], rtol=0, atol=1e-12)


def test_spectrum_peaks_and_locus_distance():
    p = np.zeros((16, 32))
    p[3, 5] = 2.0       # kx = 2 pi 5/32, ky = 2 pi 3/16
    p[16 - 3, 32 - 5] = 2.0
    p[0, 1] = 1.0
    kx, ky, pw = nci.spectrum_peaks(p, count=3)
    assert np.allclose(sorted(pw), [1.0, 2.0, 2.0])
    assert np.allclose(sorted(np.abs(kx[pw == 2.0])), [2 * np.pi * 5 / 32] * 2)
    assert np.allclose(np.abs(ky[pw == 2.0]), 2 * np.pi * 3 / 16)
    # a point placed on the curve is at distance zero
    ky0 = nci.cherenkov_locus(np.array([1.2]), 0.5)
    assert np.isfinite(ky0[0])
    assert nci.locus_distance(np.array([1.2]), ky0, 0.5)[0] < 1e-14
