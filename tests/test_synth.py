"""Pins of the seeded input generator: Philox known-answer vectors and the
moments of the Maxwell-Juettner load against Bessel-function closed forms."""
import math

import numpy as np
import pytest
from scipy.special import kv

from synth import loads
from synth.philox import Stream, philox4x32

# Known-answer vectors published with the Philox definition (Random123
# distribution, kat_vectors: philox4x32 with 10 rounds).
KAT = [
    ([0, 0, 0, 0], [0, 0], [0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8]),
    ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2, [0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD]),
    ([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0],
     [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_kat(ctr, key, want):
    got = philox4x32(np.array(ctr, dtype=np.uint32), np.array(key, dtype=np.uint32))
    assert [int(v) for v in got] == want


def test_uniforms_open_interval_and_moments():
    a, b = Stream(5, 1).uniforms(np.arange(200000), 3)
    for u in (a, b):
        assert u.min() > 0 and u.max() < 1
        assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / u.size)
    assert abs(np.corrcoef(a, b)[0, 1]) < 0.01


@pytest.mark.parametrize("T", [0.01, 0.1, 1.0])
def test_mj_rest_frame_mean_gamma(T):
    """<gamma> of Maxwell-Juettner = K1(1/T)/K2(1/T) + 3T."""
    u = loads.mj_speed(Stream(11, 2), np.arange(300000), T)
    g = np.sqrt(1 + u * u)
    want = kv(1, 1 / T) / kv(2, 1 / T) + 3 * T
    assert abs(g.mean() - want) < 5 * g.std() / math.sqrt(g.size)


def test_drifting_mj_lab_moments():
    """Lab frame of a drifting Juettner-Synge gas: <u_x> = G beta K3/K2 and
    <gamma> = G (<gamma'> + T) - T/G (from the perfect-fluid stress tensor)."""
    T, G = 0.01, 20.0
    ux, uy, uz = loads.drifting_mj(3, 0, 400000, T, G)
    beta = math.sqrt(1 - 1 / G ** 2)
    want_ux = G * beta * kv(3, 1 / T) / kv(2, 1 / T)
    gp = kv(1, 1 / T) / kv(2, 1 / T) + 3 * T
    g = np.sqrt(1 + ux ** 2 + uy ** 2 + uz ** 2)
    assert abs(ux.mean() - want_ux) < 5 * ux.std() / math.sqrt(ux.size)
    assert abs(g.mean() - (G * (gp + T) - T / G)) < 5 * g.std() / math.sqrt(g.size)
    assert abs(uy.mean()) < 5 * uy.std() / math.sqrt(uy.size)
    # transverse momentum is not boosted: <uy^2> equals the rest-frame value
    # weighted by the flux factor; at least it is T-sized
    assert 0.5 * T < (uy * uy).mean() < 2 * T


def test_stratified_positions_exact_ppc():
    nx, ny, ppc = 7, 5, 6
    x, y = loads.stratified_positions(9, nx, ny, 0.1, 0.2, ppc)
    ci = np.floor(x / 0.1).astype(int)
    cj = np.floor(y / 0.2).astype(int)
    counts = np.bincount(cj * nx + ci, minlength=nx * ny)
    assert np.all(counts == ppc)


def test_load_reproducible_per_item():
    a = loads.drifting_mj(4, 1, 1000, 0.01, 40.0)
    b = loads.drifting_mj(4, 1, 300, 0.01, 40.0, first_item=700)
    for u, v in zip(a, b):
        assert np.array_equal(u[700:], v)
