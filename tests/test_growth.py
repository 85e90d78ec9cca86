"""Pin of the growth-rate fit (a reading: the paper does not say how its
growth rates were measured) on synthetic histories with a known rate."""
import numpy as np

from oracle.growth import growth_rate


def _history(rate, n=600, dt=0.1, floor=1e-8, sat=1e-2, seed=0):
    t = np.arange(n) * dt
    rng = np.random.default_rng(seed)
    wb = floor * (1 + 0.05 * rng.standard_normal(n)) + floor * 1e-3 * np.exp(2 * rate * t)
    wb = np.minimum(wb, sat)
    return t, wb


def test_growth_rate_recovers_known_rate():
    for rate in (0.2, 0.5, 1.0):
        t, wb = _history(rate, n=int(40 / rate) * 3)
        g = growth_rate(t, wb)
        assert g is not None
        assert abs(g["rate"] - rate) < 0.02 * rate


def test_no_exponential_phase():
    t = np.arange(500) * 0.1
    wb = 1e-8 * (1 + 0.05 * np.random.default_rng(1).standard_normal(500))
    assert growth_rate(t, wb) is None
