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
    """A short C1-like run (gamma0 = 20, order 1, sigma = 1, theta = 0.6) keeps
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
