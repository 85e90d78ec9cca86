"""The device-side plasma loader against the seeded host generator, and the
large single-GPU share (periodic 8192 x 2048, pair plasma at gamma0 = 40,
64 particles/cell/species: 2.1e9 particles in FP32, cubic shape, CFL 1,
theta 0.6, with the learned aid) at full size on outputs the FP64 oracle can
compute piecewise or whole (the field solve)."""
import sys

import numpy as np
import pytest

import oracle
from pic_cases import relerr
from synth import loads
from synth.philox import Stream

pytestmark = pytest.mark.gpu

DX = 0.1


def _say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("shock", [False, True])
def test_device_load_matches_host_generator(precision, shock):
    import paper_1412_2480_amd as pic
    _say(f"device loader vs host generator ({precision}, shock={shock})")
    nx, ny, ppc, g0, T, seed = 40, 36, 5, 20.0, 0.01, 3
    x_cells = nx - pic.PIC_WALL_GAP if shock else nx
    direction = -1 if shock else 1
    Q = loads.macro_charge(g0, DX, DX, ppc)
    run = pic.run_desc(nx, ny, DX, 1.0, 0.6, 2, [(-Q, Q, ppc), (Q, Q, ppc)],
                       bc="shock" if shock else "periodic")
    sim = pic.Sim([run], pic.make_options(precision, slack=0.5))
    ref = loads.pair_plasma_cells(x_cells, ny, ppc, g0, T, seed, direction=direction)
    n = x_cells * ny * ppc
    for s in range(2):
        sim.load_plasma(0, s, ppc, g0, T, seed, direction=direction,
                        x_cells=x_cells if shock else 0)
        g = sim.read_particles(0, s, n)
        r = ref[s]
        assert len(g["ix"]) == n
        cast = (lambda a: a.astype(np.float32).astype(np.float64)) if precision == "fp32" \
            else (lambda a: a)
        assert np.array_equal(g["ix"], r["ix"]) and np.array_equal(g["iy"], r["iy"])
        assert np.array_equal(g["fx"], cast(r["fx"])) and np.array_equal(g["fy"], cast(r["fy"]))
        u = np.stack([g["ux"], g["uy"], g["uz"]])
        ur = np.stack([cast(r["ux"]), cast(r["uy"]), cast(r["uz"])])
        scale = np.maximum(np.abs(ur).max(axis=0), 1e-300)
        d = np.abs(u - ur).max(axis=0) / scale
        # the device's and numpy's log/sin/cos may differ in the last place, so
        # a rejection decision can rarely flip; everything else agrees to ulps
        tol = 1e-13 if precision == "fp64" else 1.2e-7
        flips = int(np.sum(d > tol))
        _say(f"  species {s}: max rel diff {np.sort(d)[-2] if n > 1 else 0:.2e}, "
             f"differing draws {flips} of {n}")
        assert flips <= max(2, n // 1000)
    sim.close()


def test_large_share_fullsize_fp32():
    import paper_1412_2480_amd as pic
    NX, NY, PPC, G0, ORDER, T, SEED = 8192, 2048, 64, 40.0, 3, 0.01, 0
    Q = loads.macro_charge(G0, DX, DX, PPC)
    run = pic.run_desc(NX, NY, DX, 1.0, 0.6, ORDER, [(-Q, Q, PPC), (Q, Q, PPC)], cg_rtol=1e-8)
    # the launch configuration and the learned aid as the timed form uses
    # them (2 x 64 tiles, one work-group per tile, reordering every 4 steps,
    # slack 0.5; plain CG first, recording training pairs, then the trained
    # network): the fourth step ends with a reordering, so the learned step
    # runs on a reordered store
    opts = pic.make_options("fp32", tile=(2, 64), tile_split=1, track_ids=False,
                            solver="learned", precond_slots=4, sort_every=4, slack=0.5)
    _say(f"large share: workspace {pic.plan([run], opts).workspace_bytes / 1e9:.1f} GB")
    sim = pic.Sim([run], opts)
    _say(f"large share: context created ({sim.L.pic_last_error(sim.ctx).decode() or 'ok'})")
    for s in range(2):
        sim.load_plasma(0, s, PPC, G0, T, SEED)
    d0 = sim.diag(0)
    assert d0["n_particles"] == [NX * NY * PPC] * 2
    sim.precond_use(False)
    sim.precond_collect(True)
    _say("large share: first step (fields start at zero)")
    sim.step(1)
    J = [sim.get_field(0, k) for k in ("Jx", "Jy", "Jz")]
    F1 = {k: sim.get_field(0, k) for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")}
    dt = DX
    rng = np.random.default_rng(1)
    # ---- current on sampled node boxes from the generator's items near them:
    # with zero fields the push leaves u unchanged and x moves by dt u/gamma
    for b in range(3):
        i0 = int(rng.integers(8, NX - 16))
        j0 = int(rng.integers(8, NY - 16))
        Jr = [np.zeros((24, 24)) for _ in range(3)]   # box with a 5-cell margin, local grid
        for s, q in enumerate((-Q, Q)):
            xs, ys, us = [], [], []
            for j in range(j0 - 5, j0 + 13):
                c0, c1 = j * NX + (i0 - 5), j * NX + (i0 + 13)
                items = np.arange(c0 * PPC, c1 * PPC, dtype=np.int64)
                r0, r1 = Stream(SEED, loads.TAG_POS).uniforms(items, 0)
                cell = items // PPC
                xs.append(cell % NX - (i0 - 8) + r0)
                ys.append(cell // NX - (j0 - 8) + r1)
                us.append(loads.drifting_mj(SEED, s, items.size, T, G0, 1,
                                            first_item=int(c0 * PPC)))
            X = np.concatenate(xs)
            Y = np.concatenate(ys)
            ux = np.concatenate([u[0] for u in us])
            uy = np.concatenate([u[1] for u in us])
            uz = np.concatenate([u[2] for u in us])
            # the GPU holds offsets and momenta in FP32
            ix = np.floor(X).astype(np.int32)
            iy = np.floor(Y).astype(np.int32)
            p = oracle.Particles(ix, iy, (X - ix).astype(np.float32), (Y - iy).astype(np.float32),
                                 ux.astype(np.float32), uy.astype(np.float32),
                                 uz.astype(np.float32), q, Q)
            old = p.copy()
            oracle.move(p, dt, DX, DX)
            oracle.deposit(24, 24, ORDER, DX, DX, dt, old, p, Jr)
        jscale = [Q / (DX * dt) * PPC, Q / (DX * dt) * PPC, Q * PPC / (DX * DX)]
        for c in range(3):
            err = np.abs(J[c][j0:j0 + 8, i0:i0 + 8] - Jr[c][8:16, 8:16]).max()
            _say(f"  box {b} J{'xyz'[c]}: err/scale {err / jscale[c]:.2e}")
            assert err <= 1e-6 * jscale[c]
    # ---- field solve on the whole grid from the GPU's current, FP64 oracle
    _say("large share: oracle field solve on the whole grid")
    ref = oracle.Sim(NX, NY, DX, DX, 1.0, 0.6, ORDER, [], rtol=1e-8)
    for c in range(3):
        ref.J[c][...] = J[c]
    ref.field_solve()
    for k, name in enumerate(("Ex", "Ey", "Ez")):
        e = relerr(F1[name], ref.E[k])
        _say(f"  {name} relerr {e:.2e}")
        assert e <= 1e-6
    for k, name in enumerate(("Bx", "By", "Bz")):
        e = relerr(F1[name], ref.B[k])
        _say(f"  {name} relerr {e:.2e}")
        assert e <= 1e-6
    del ref, J, F1
    _say("large share: 3 more steps, Gauss's law")
    st = sim.step(3)[0]
    assert max(st["relres"]) <= 1e-8
    assert sim.precond_collect(False) == 4
    d = sim.diag(0)
    rho_scale = 4 * np.pi * Q / (DX * DX)
    _say(f"  gauss {d['gauss_max']:.3e} (scale {rho_scale:.3e}), cg {st['iters']}")
    assert d["gauss_max"] <= 1e-4 * rho_scale
    assert d["n_particles"] == [NX * NY * PPC] * 2
    # ---- learned aid at full size: trained on the 4 recorded pairs (64-cell
    # windows), then one step whose field solve is checked against the
    # oracle's from the same E^n, B^n and J^{n+1/2}
    tr = sim.precond_train(epochs=25)
    _say(f"large share: trained, loss {tr['loss_first']:.2e} -> {tr['loss_last']:.2e}")
    assert tr["loss_last"] < 0.01 * tr["loss_first"]
    sim.precond_use(True)
    F0 = {k: sim.get_field(0, k) for k in ("Ex", "Ey", "Ez", "Bx", "By", "Bz")}
    sl = sim.step(1)[0]
    _say(f"  learned step: iterations {sl['learned_iters']}, fallback {sl['fallback']}, "
         f"relres {max(sl['relres']):.2e} (plain CG {st['iters']})")
    assert sl["fallback"] == 0 and max(sl["relres"]) <= 1e-8
    assert sum(sl["learned_iters"]) < sum(st["iters"])
    ref = oracle.Sim(NX, NY, DX, DX, 1.0, 0.6, ORDER, [], rtol=1e-8)
    for k in range(3):
        ref.E[k][...] = F0[("Ex", "Ey", "Ez")[k]]
        ref.B[k][...] = F0[("Bx", "By", "Bz")[k]]
        ref.J[k][...] = sim.get_field(0, ("Jx", "Jy", "Jz")[k])
    del F0
    ref.field_solve()
    for k, name in enumerate(("Ex", "Ey", "Ez", "Bx", "By", "Bz")):
        e = relerr(sim.get_field(0, name), ref.E[k] if k < 3 else ref.B[k - 3])
        _say(f"  {name} relerr {e:.2e}")
        assert e <= 1e-6
    sim.close()
