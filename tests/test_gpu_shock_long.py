"""The shock workload as configured: 4096 x 512 cells with a reflecting wall at
x = 0 and the pair flow (gamma0 = 40, 32 particles/cell/species, order 2,
CFL 1.0, theta = 0.6) injected on the device at x_out every step, for 10,000
steps. The learned aid is trained on (b, dB) pairs recorded across the first
500 steps (solved by plain CG), then every field solve of the remaining 9,500
steps runs the learned PCG: invariants checked on the way (no plain-CG
fallback, true residual <= 1e-8, Gauss's law between the wall and the
outflow region at FP32 roundoff, the particle count against the injected
and removed numbers)."""
import math
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.timeout(900)
def test_shock_10000_steps_learned():
    import paper_1412_2480_amd as pic
    from synth import loads
    nx, ny, ppc, g0, T, order = 4096, 512, 32, 40.0, 0.01, 2
    x_out = nx - pic.PIC_WALL_GAP
    Q = loads.macro_charge(g0, 0.1, 0.1, ppc)
    run = pic.run_desc(nx, ny, 0.1, 1.0, 0.6, order, [(-Q, Q, ppc), (Q, Q, ppc)], cg_rtol=1e-8,
                       cg_maxit=200, bc="shock")
    # the shock compresses the flow behind it and the reflected beam adds to
    # that: with 5x the upstream slots a tile near the wall overflowed near
    # step 6000, so tiles get 10x
    sim = pic.Sim([run], pic.make_options("fp32", tile=(4, 32), tile_split=2, slack=9.0, track_ids=False, solver="learned",
                                          precond_slots=16, sort_every=4, graph=True))
    for s in range(2):
        sim.load_plasma(0, s, ppc, g0, T, seed=0, direction=-1, x_cells=x_out)
    sim.set_inflow(0, ppc, g0, T, seed=0)
    n0 = x_out * ny * ppc
    t0 = time.time()
    # plain CG for the first 500 steps; one (b, dB) pair recorded every 31 steps
    sim.precond_use(False)
    plain_iters = []
    for k in range(16):
        sim.step(30)
        sim.precond_collect(True)
        st = sim.step(1)[0]
        sim.precond_collect(False)
        plain_iters.append(sum(st["iters"]))
    sim.step(4)
    _say(f"500 plain-CG steps in {time.time() - t0:.0f} s, iterations {plain_iters[-1]}")
    tr = sim.precond_train(epochs=50)
    _say(f"trained on 16 pairs: loss {tr['loss_first']:.3e} -> {tr['loss_last']:.3e}")
    assert tr["loss_last"] < 0.05 * tr["loss_first"]
    sim.precond_use(True)
    done = 500
    learned = []
    while done < 10000:
        k = min(500, 10000 - done)
        sim.step(k - 1)
        st = sim.step(1)[0]
        done += k
        d = sim.diag(0)
        learned.append(max(st["learned_iters"]))
        _say(f"step {done}: learned iterations {st['learned_iters']}, relres "
             f"{max(st['relres']):.1e}, fallbacks {d['fallbacks']}, particles "
             f"{d['n_particles'][:2]}, gauss {d['gauss_max']:.2e} ({time.time() - t0:.0f} s)")
        assert d["fallbacks"] == 0
        assert max(st["relres"]) <= 1e-8
    rho_scale = 4 * np.pi * Q / (0.1 * 0.1)
    assert d["gauss_max"] <= 1e-3 * rho_scale
    # particle count: the initial load plus the inflow, minus what left at x_out
    w = math.sqrt(1.0 - 1.0 / g0 ** 2) * 1.0
    injected = math.floor(ppc * w * 10000) * ny
    for s in range(2):
        assert n0 < d["n_particles"][s] <= n0 + injected
    assert max(learned) < min(plain_iters) / 3 + 1
    sim.close()
