"""The periodic reordering of each tile's particles (pic_options.sort_every):
it changes only the storage order, so runs with and without it agree to
roundoff (the order of the deposit's additions), in both forms, on a shock
run with injection and in graph mode; and the stored order is the
documented one (cell-major runs dealt out one per wavefront lane)."""
import sys

import numpy as np
import pytest

from pic_cases import Case, relerr

pytestmark = pytest.mark.gpu

NAMES = ("Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz")


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _compare(a, b, case, tol, run=0):
    for n in NAMES:
        e = relerr(a.get_field(run, n), b.get_field(run, n))
        assert e <= tol, (n, e)
    for s in range(2):
        pa = a.read_particles(run, s, case.species[s].n + 64)
        pb = b.read_particles(run, s, case.species[s].n + 64)
        assert len(pa["ix"]) == len(pb["ix"]) == case.species[s].n
        assert np.array_equal(pa["ix"], pb["ix"]) and np.array_equal(pa["iy"], pb["iy"])
        for k in ("fx", "fy", "ux", "uy", "uz"):
            assert np.abs(pa[k] - pb[k]).max() <= tol * max(1.0, np.abs(pb[k]).max()), (s, k)


# (precision, period, tile, ppc) on 16 x 16 tiles: at 6 particles/cell a
# tile's arrays are staged in LDS whole; at 40 (12,800 slots) in 2 (FP32) or 3
# (FP64) chunks; at 64 in FP64 and 96 in FP32 more than 4 chunks would be
# needed and the path that gathers from global memory is taken
SORT_CASES = [("fp64", 1, (16, 16), 6), ("fp64", 3, (16, 16), 6), ("fp32", 2, (16, 16), 6),
              ("fp32", 2, (16, 16), 40), ("fp64", 2, (16, 16), 40),
              ("fp64", 2, (16, 16), 64), ("fp32", 2, (16, 16), 96)]


@pytest.mark.parametrize("precision,every,tile,ppc", SORT_CASES)
def test_sorted_run_equals_unsorted(precision, every, tile, ppc):
    _say(f"sort_every={every} vs none, {precision}, tile {tile}, ppc {ppc}")
    case = Case(64, 48, 3, ppc=ppc, gamma0=5.0, T=0.05, seed=7, field_amp=0.3, rtol=1e-12)
    a = case.gpu_sim(precision, tile=tile)
    b = case.gpu_sim(precision, tile=tile, sort_every=every)
    a.timing(True)
    b.timing(True)
    a.step(7)
    b.step(7)
    assert b.get_timing()["sort"]["launches"] == 7 // every
    assert a.get_timing()["sort"]["launches"] == 0
    _compare(a, b, case, 1e-12 if precision == "fp64" else 1e-5)
    a.close()
    b.close()


@pytest.mark.parametrize("side,ppc", [(16, 9), (16, 40), (16, 64)])
def test_sorted_storage_order(side, ppc):
    """One side x side tile, ids off (reads return storage order): after a
    sorted step, position q = 64 w + l holds the w-th particle of lane l's run
    of the cell-sorted order (runs of L or L - 1, the longer ones first). The
    FP64 arrays are staged whole at 9 particles/cell, in 3 chunks at 40, and
    gathered from global memory at 64."""
    _say(f"sorted storage order, {side}x{side} tile, ppc {ppc}")
    case = Case(side, side, 2, ppc=ppc, gamma0=3.0, T=0.1, seed=3, field_amp=0.2)
    sim = case.gpu_sim("fp64", tile=(side, side), track_ids=False, sort_every=1)
    sim.step(2)
    for s in range(2):
        g = sim.read_particles(0, s, 1 << 16)
        n = len(g["ix"])
        assert n == case.species[s].n
        cell = g["iy"].astype(np.int64) * side + g["ix"]
        L = (n + 63) // 64
        full = n - 64 * (L - 1)
        # sorted position of every storage position
        p_of_q = np.empty(n, np.int64)
        for lane in range(64):
            start = lane * L if lane < full else full * L + (lane - full) * (L - 1)
            length = L if lane < full else L - 1
            for w in range(length):
                p_of_q[w * 64 + lane] = start + w
        assert np.array_equal(np.sort(p_of_q), np.arange(n))
        in_p_order = np.empty(n, np.int64)
        in_p_order[p_of_q] = cell
        assert np.all(np.diff(in_p_order) >= 0), "not cell-sorted"
        # a full wavefront covers distinct cells
        w0 = cell[:64]
        assert len(np.unique(w0)) == 64
    sim.close()


def test_sorted_shock_run_with_injection():
    from test_gpu_shock import Shock, _inject_both
    _say("shock run, sort_every=2 vs none")
    case = Shock(48, 24, 2, ppc=4, seed=5, field_amp=0.2, rtol=1e-12)
    a = case.gpu_sim("fp64")
    b = case.gpu_sim("fp64", sort_every=2)
    for step in range(6):
        _inject_both(case, step, a, None)
        _inject_both(case, step, b, None)
        a.step(1)
        b.step(1)
    for n in NAMES:
        assert relerr(a.get_field(0, n), b.get_field(0, n)) <= 1e-12, n
    for s in range(2):
        ga = a.read_particles(0, s, 1 << 20)
        gb = b.read_particles(0, s, 1 << 20)
        assert len(ga["ix"]) == len(gb["ix"])
        assert np.array_equal(ga["ix"], gb["ix"]) and np.array_equal(ga["iy"], gb["iy"])
        for k in ("fx", "fy", "ux", "uy", "uz"):
            assert np.abs(ga[k] - gb[k]).max() <= 1e-12 * max(1.0, np.abs(gb[k]).max())
    a.close()
    b.close()


@pytest.mark.parametrize("sort_every", [4, 3, 1])
def test_sorted_graph_mode(sort_every):
    """Every two-step window replays from a graph, also those that end a step
    with a reordering (period 4: after the second step; 3: after the first or
    the second, from either buffer parity; 1: after both), and the run agrees
    with plain launches without reordering."""
    _say(f"graph mode with sort_every={sort_every}")
    case = Case(48, 32, 2, ppc=4, gamma0=5.0, T=0.05, seed=9, field_amp=0.3, rtol=1e-12)
    a = case.gpu_sim("fp64")
    b = case.gpu_sim("fp64", graph=True, sort_every=sort_every)
    a.step(24)
    b.step(24)
    assert b.get_timing()["graph_replays"] == 12
    _compare(a, b, case, 1e-12)
    a.close()
    b.close()
