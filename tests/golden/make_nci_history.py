"""Write tests/golden/nci_history_128x64.json: the FP64 oracle's energy history
of a whole run in which the numerical Cherenkov instability grows from noise
and saturates, plus the growth rate measured from it.

Run: python tests/golden/make_nci_history.py   (about a minute, one CPU core)

Workload: periodic 128 x 64 grid, dx = dy = 0.1 c/omega_pe, pair plasma
drifting along +x at gamma0 = 40 with rest-frame temperature T = 0.01 m c^2,
16 particles/cell/species (stratified, e- and e+ co-located), cubic (order-3)
shape, CFL 1.0, theta = 0.6, field CG to 1e-8, 250 steps, seed 0. This is the
1024 x 256 single-run workload on a smaller grid (same physics per cell).
Only the oracle and the seeded input generator are used.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from oracle.growth import growth_rate  # noqa: E402
from synth import loads  # noqa: E402

CASE = dict(nx=128, ny=64, dx=0.1, ppc=16, gamma0=40.0, T=0.01, order=3, cfl=1.0, theta=0.6,
            rtol=1e-8, steps=250, seed=0)
OUT = os.path.join(HERE, "nci_history_128x64.json")


def main():
    c = CASE
    Q = loads.macro_charge(c["gamma0"], c["dx"], c["dx"], c["ppc"])
    ld = loads.pair_plasma_cells(c["nx"], c["ny"], c["ppc"], c["gamma0"], c["T"], c["seed"])
    sp = [oracle.Particles(d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"], q, Q)
          for d, q in zip(ld, (-Q, Q))]
    sim = oracle.Sim(c["nx"], c["ny"], c["dx"], c["dx"], c["cfl"], c["theta"], c["order"], sp,
                     rtol=c["rtol"])
    recs = []
    t0 = time.time()
    for n in range(c["steps"]):
        r = sim.step()
        recs.append([r["W_E"], r["W_B"], r["W_K_minus"], r["W_K_plus"], max(r["cg_iters"])])
        if n % 50 == 49:
            print(f"step {n + 1}: W_B = {r['W_B']:.4e} ({time.time() - t0:.0f} s)", flush=True)
    a = np.array(recs)
    t = np.arange(c["steps"]) * c["cfl"] * c["dx"]
    g = growth_rate(t, a[:, 1])
    out = dict(case=c, macro_charge=Q, columns=["W_E", "W_B", "W_K_minus", "W_K_plus",
                                                "max_cg_iters"],
               records=a.tolist(), growth=g,
               note="FP64 oracle; record n holds W_E, W_B at step n and W_K at n -/+ 1/2")
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("growth", g)


if __name__ == "__main__":
    main()
