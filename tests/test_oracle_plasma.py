"""Whole-step pins of the oracle on small plasmas; CPU only."""
import numpy as np
import pytest

from synth import loads


def _pair_sim(ora, nx, ny, ppc, gamma0, T, order, cfl, theta, seed=0, rtol=1e-8, dx=0.1):
    sp = loads.pair_plasma(nx, ny, dx, dx, ppc, gamma0, T, seed)
    Q = loads.macro_charge(max(gamma0, 1.0), dx, dx, ppc)
    species = []
    for s, q in zip(sp, (-Q, Q)):
        species.append(ora.Particles.from_xy(s["x"], s["y"], s["ux"], s["uy"], s["uz"], q, Q,
                                             dx, dx))
    return ora.Sim(nx, ny, dx, dx, cfl, theta, order, species, rtol=rtol)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_gauss_law_invariant_with_loose_cg(ora, order):
    """div E - 4 pi rho is constant in time to roundoff even when the CG
    stops early: the update changes E only by curls and -4 pi dt J, and the
    Esirkepov J satisfies discrete continuity (Eqs. (5)-(6) with Sec. 1's
    density decomposition)."""
    sim = _pair_sim(ora, 16, 12, 4, 5.0, 0.05, order, 1.0, 0.6, seed=3, rtol=1e-3)
    g0 = sim.gauss_residual()
    scale = 4 * np.pi * max(np.abs(sim.species[0].q) / (sim.dx * sim.dy), 1e-300)
    for _ in range(6):
        sim.step()
    g1 = sim.gauss_residual()
    assert np.abs(g0).max() < 1e-12 * scale
    assert np.abs(g1 - g0).max() < 1e-11 * scale
    assert max(sim.last["cg_relres"]) > 1e-6       # the CG really was loose


def test_thermal_plasma_energy_within_one_percent(ora):
    """Total energy W_E + W_B + (W_K(n-1/2) + W_K(n+1/2))/2 of a thermal pair
    plasma stays within 1 % (the paper's figure for its runs, Sec. 3.2)."""
    sim = _pair_sim(ora, 16, 16, 8, 1.0, 0.01, 2, 1.0, 0.6, seed=1)
    tot = []
    for _ in range(60):
        r = sim.step()
        tot.append(r["W_E"] + r["W_B"] + 0.5 * (r["W_K_minus"] + r["W_K_plus"]))
    tot = np.array(tot)
    assert np.abs(tot / tot[0] - 1).max() < 0.01


def test_drifting_pair_energy_and_cg(ora):
    """A short run like the 64x64 one (gamma0 = 20, order 1, sigma = 1, theta = 0.6) keeps
    total energy within 1 % and the CG meets 1e-8 in at most 17 iterations
    (kappa <= 1 + 8 (theta sigma)^2 bounds CG at 1e-8)."""
    sim = _pair_sim(ora, 16, 16, 4, 20.0, 0.01, 1, 1.0, 0.6, seed=0)
    tot = []
    for _ in range(20):
        r = sim.step()
        tot.append(r["W_E"] + r["W_B"] + 0.5 * (r["W_K_minus"] + r["W_K_plus"]))
        assert max(r["cg_iters"]) <= 17
        assert max(r["cg_relres"]) <= 1e-8
    tot = np.array(tot)
    assert np.abs(tot / tot[0] - 1).max() < 0.01


def test_pair_load_is_charge_neutral(ora):
    sim = _pair_sim(ora, 8, 8, 4, 20.0, 0.01, 3, 1.0, 0.6)
    rho = sim.rho()
    assert np.abs(rho).max() < 1e-14 * abs(sim.species[1].q) / (sim.dx * sim.dy)


def test_threads_change_only_the_summation_order(ora):
    """The oracle's OpenMP threads (per-thread deposit buffers and partial
    sums, added in thread order) give the one-thread result to roundoff, and
    the same result on every repetition with the same thread count."""
    def run(threads):
        ora.set_threads(threads)
        sim = _pair_sim(ora, 24, 16, 6, 10.0, 0.05, 3, 1.0, 0.6, seed=4)
        rec = [sim.step() for _ in range(4)]
        return sim, rec
    try:
        a, ra = run(1)
        b, rb = run(4)
        c, rc = run(4)
    finally:
        ora.set_threads(0)
    for k in range(3):
        for x, y, z in ((a.E[k], b.E[k], c.E[k]), (a.B[k], b.B[k], c.B[k]),
                        (a.J[k], b.J[k], c.J[k])):
            assert np.array_equal(y, z)
            assert np.abs(x - y).max() <= 1e-12 * max(np.abs(x).max(), 1e-300)
    for p, q in zip(a.species, b.species):
        assert np.array_equal(p.ix, q.ix)
        assert np.abs(p.ux - q.ux).max() <= 1e-12 * np.abs(p.ux).max()
    for u, v in zip(ra, rb):
        assert abs(u["W_K_plus"] - v["W_K_plus"]) <= 1e-12 * abs(u["W_K_plus"])


def test_explicit_scheme_plasma(ora):
    """The explicit Yee scheme (Eqs. (3)-(4)) in a whole step at sigma = 0.5:
    Gauss's law constant to roundoff and a thermal plasma's total energy
    within 1 % (the paper's figure for its runs, Sec. 3.2)."""
    sp = loads.pair_plasma(16, 16, 0.1, 0.1, 8, 1.0, 0.01, 1)
    Q = loads.macro_charge(1.0, 0.1, 0.1, 8)
    species = [ora.Particles.from_xy(s["x"], s["y"], s["ux"], s["uy"], s["uz"], q, Q, 0.1, 0.1)
               for s, q in zip(sp, (-Q, Q))]
    sim = ora.Sim(16, 16, 0.1, 0.1, 0.5, 0.6, 2, species, scheme="explicit")
    g0 = sim.gauss_residual()
    tot = []
    for _ in range(60):
        r = sim.step()
        assert r["cg_iters"] == [0, 0, 0]
        tot.append(r["W_E"] + r["W_B"] + 0.5 * (r["W_K_minus"] + r["W_K_plus"]))
    tot = np.array(tot)
    assert np.abs(tot / tot[0] - 1).max() < 0.01
    scale = 4 * np.pi * Q / (0.1 * 0.1)
    assert np.abs(sim.gauss_residual() - g0).max() < 1e-11 * scale
