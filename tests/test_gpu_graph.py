"""Graph mode (HIP graphs of two captured steps, replayed) gives the same
results as plain launches: periodic and shock runs, batched runs, the learned
solver (with its variant switched between replays) and diagnostics steps that
fall back to plain launches."""
import sys

import numpy as np
import pytest

from pic_cases import Case, relerr

pytestmark = pytest.mark.gpu

FIELDS = ("Ex", "Ey", "Ez", "Bx", "By", "Bz")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _compare(a, b, tol, runs=1):
    for r in range(runs):
        for n in FIELDS:
            assert relerr(a.get_field(r, n), b.get_field(r, n)) <= tol, (r, n)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_matches_plain_launches(precision):
    _say(f"graph vs plain, {precision}")
    case = Case(48, 40, 2, ppc=4, gamma0=10.0, T=0.05, seed=3, field_amp=0.2)
    a = case.gpu_sim(precision, diag_every=5, history_cap=64)
    b = case.gpu_sim(precision, diag_every=5, history_cap=64, graph=True)
    for n in (1, 4, 7, 2):
        a.step(n)
        b.step(n)
    tol = 1e-12 if precision == "fp64" else 1e-5
    _compare(a, b, tol)
    assert a.get_timing()["graph_replays"] == 0
    assert b.get_timing()["graph_replays"] >= 3   # the graph path really ran
    ha, hb = a.history(0), b.history(0)
    assert [h["step"] for h in ha] == [h["step"] for h in hb] == [0, 5, 10]
    for x, y in zip(ha, hb):
        assert abs(x["W_B"] - y["W_B"]) <= tol * max(1e-30, abs(x["W_B"]))
    a.close()
    b.close()


def test_graph_learned_and_batched():
    import paper_1412_2480_amd as pic
    _say("graph: batched runs with the learned solver switched on and off")
    cases = [Case(40, 36, 1, ppc=3, gamma0=5.0, seed=1), Case(56, 24, 3, ppc=3, gamma0=5.0, seed=2)]
    runs = [c.run_desc() for c in cases]
    sims = []
    for graph in (False, True):
        sim = pic.Sim(runs, pic.make_options("fp64", solver="learned", graph=graph))
        for r, c in enumerate(cases):
            c.load_into(sim, r)
        sims.append(sim)
    for sim in sims:
        sim.precond_use(False)
        sim.step(4)
        sim.precond_use(True)
        st = sim.step(4)
        assert all(max(s["relres"]) <= 1e-8 for s in st)
        sim.precond_use(False)
        sim.step(3)
    _compare(sims[0], sims[1], 1e-12, runs=2)
    assert sims[1].get_timing()["graph_replays"] >= 4
    for sim in sims:
        sim.close()


def test_graph_shock_with_injection():
    from test_gpu_shock import Shock, _inject_both
    _say("graph: shock run with injection between replays")
    case = Shock(48, 24, 2, ppc=4, seed=5, field_amp=0.2)
    a = case.gpu_sim("fp64")
    b = case.gpu_sim("fp64", graph=True)
    for step in range(0, 8, 2):
        _inject_both(case, step, a, None)
        _inject_both(case, step, b, None)
        a.step(2)
        b.step(2)
    _compare(a, b, 1e-12)
    assert b.get_timing()["graph_replays"] == 4
    for s in range(2):
        assert len(a.read_particles(0, s, 1 << 20)["ix"]) == len(b.read_particles(0, s, 1 << 20)["ix"])
    a.close()
    b.close()
