"""The paper's relativistic shock runs (Sec. 4) on the GPU library.

Set-up of Sec. 4: 5650 x 990 cells, a pair flow at Gamma = 100 (V = 0.9999 c)
with a flow-frame thermal speed of 0.05 c (T = 0.0025 m c^2), 50 particles per
cell per species initially, second-order shape, theta = 0.501, CFL 0.5 or
1.0, followed to omega_pe t = 177 in the frame of the reflecting wall, where
the shock moves away from the wall into the flow. The paper injects at the
left and reflects at the right; this library's shock set-up (PIC_BC_SHOCK) is
its mirror image: the conducting, reflecting wall at x = 0 and the flow
entering through x_out on the right, moving towards -x. Profiles are
therefore functions of the distance from the wall. The paper does not state
the cell size; 0.1 c/omega_pe is taken (that of the other workloads).

Outputs (Figs. 7-8): transverse averages of the electron density and of B_z,
normalised by the upstream density and by sqrt(4 pi n m Gamma c^2) (= Gamma
in the code units, where c = 1, |q| = m and the flow's plasma frequency
sqrt(4 pi n q^2 / (m Gamma)) is one), and the transverse mean of B_z^2 in
the same normalisation (the magnetic energy density over the upstream kinetic one,
within a factor 2 for the two species).
"""
import argparse
import json
import sys
import time

import numpy as np

GAMMA = 100.0
T_FLOW = 0.0025     # flow-frame thermal speed 0.05 c
DX = 0.1


def run(pic, sigma=1.0, t_end=177.0, nx=5650, ny=990, ppc=50, order=2, theta=0.501,
        gamma0=GAMMA, T=T_FLOW, slack=5.0, precision="fp32", learned_pairs=8,
        profile_times=(), tile=(2, 66), tile_split=1, sort_every=8, log=None):
    """One shock run to omega_pe t = t_end; returns the profiles at t_end
    (and at each of profile_times), particle counts and timings. The tile
    height should divide ny (990 = 15 x 66): tile slots are sized for the
    largest tile, and a last tile that absorbs a tail is taller. The shocked
    plasma behind the front is about three times denser than the flow, and
    filaments add to that: tiles get 6x the flow's particles (slack 5)."""
    from synth import loads
    x_out = nx - pic.PIC_WALL_GAP
    Q = loads.macro_charge(gamma0, DX, DX, ppc)
    desc = pic.run_desc(nx, ny, DX, sigma, theta, order, [(-Q, Q, ppc), (Q, Q, ppc)],
                        cg_rtol=1e-8, cg_maxit=300, bc="shock")
    sim = pic.Sim([desc], pic.make_options(precision, tile=tile, tile_split=tile_split,
                                           slack=slack, track_ids=False,
                                           solver="learned", precond_slots=learned_pairs,
                                           sort_every=sort_every, graph=True))
    for s in range(2):
        sim.load_plasma(0, s, ppc, gamma0, T, seed=0, direction=-1, x_cells=x_out)
    sim.set_inflow(0, ppc, gamma0, T, seed=0)
    dt = sigma * DX
    steps = int(round(t_end / dt))
    n_up = ppc / (DX * DX)            # upstream (lab) density per species
    b_norm = gamma0                   # sqrt(4 pi n m Gamma c^2) in these units

    def profiles():
        ne = sim.transverse_average(0, "n0") / n_up
        bz = sim.transverse_average(0, "Bz") / b_norm
        b2 = sim.get_field(0, "Bz")
        b2 = (b2 * b2).mean(axis=0) / (b_norm * b_norm)
        return dict(x=(np.arange(nx) * DX).tolist(), electron_density=ne.tolist(),
                    bz_mean=bz.tolist(), bz2_mean=b2.tolist())

    t0 = time.perf_counter()
    # learned aid: plain CG on the first steps, recorded as training pairs
    sim.precond_use(False)
    sim.precond_collect(True)
    sim.step(learned_pairs)
    sim.precond_collect(False)
    sim.precond_train(50, 0.0)
    sim.precond_use(True)
    done = learned_pairs
    snaps = {}
    marks = sorted(set(int(round(t / dt)) for t in profile_times if 0 < t < t_end))
    for m in marks + [steps]:
        while done < m:
            k = min(200, m - done)
            sim.step(k)
            done += k
            if log:
                d = sim.diag(0)
                log(f"shock sigma {sigma}: step {done}/{steps}, particles "
                    f"{d['n_particles'][0] + d['n_particles'][1]}, "
                    f"{time.perf_counter() - t0:.0f} s")
        snaps[round(m * dt, 6)] = profiles()
    elapsed = time.perf_counter() - t0
    d = sim.diag(0)
    st = sim.step(0)[0]
    out = dict(sigma=sigma, theta=theta, order=order, nx=nx, ny=ny, ppc=ppc, gamma0=gamma0,
               T=T, dx=DX, steps=steps, t_end=steps * dt, seconds=elapsed,
               ms_per_step=elapsed * 1e3 / steps,
               particles_end=int(d["n_particles"][0] + d["n_particles"][1]),
               gauss_max=d["gauss_max"], fallbacks=int(d["fallbacks"]),
               learned_iters_last=st["learned_iters"], profiles=snaps)
    sim.close()
    return out


def shock_front(profile, x, level=2.0):
    """Distance from the wall (x = 0) of the last point, going outwards, where
    the transverse-mean density still exceeds `level` times the upstream
    value: the position of the density jump."""
    n = np.asarray(profile)
    idx = np.flatnonzero(n > level)
    return float(np.asarray(x)[idx[-1]]) if idx.size else 0.0


def main(argv=None):
    ap = argparse.ArgumentParser(description="paper-scale relativistic shock run (Sec. 4)")
    ap.add_argument("--sigma", type=float, default=1.0)
    ap.add_argument("--t-end", type=float, default=177.0)
    ap.add_argument("--nx", type=int, default=5650)
    ap.add_argument("--ny", type=int, default=990)
    ap.add_argument("--ppc", type=int, default=50)
    ap.add_argument("--out", default="")
    a = ap.parse_args(argv)
    import paper_1412_2480_amd as pic

    def log(m):
        print(m, file=sys.stderr, flush=True)
    r = run(pic, a.sigma, a.t_end, a.nx, a.ny, a.ppc, log=log)
    prof = r["profiles"][max(r["profiles"])]
    r["shock_front_x"] = shock_front(prof["electron_density"], prof["x"])
    log(f"shock sigma {a.sigma}: {r['steps']} steps in {r['seconds']:.1f} s "
        f"({r['ms_per_step']:.1f} ms/step), front at x = {r['shock_front_x']:.1f}")
    text = json.dumps(r)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    else:
        print(json.dumps({k: v for k, v in r.items() if k != "profiles"}))


if __name__ == "__main__":
    main()
