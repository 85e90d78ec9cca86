"""Write tests/golden/nci_history_<case>.json: the FP64 oracle's energy history
of a whole run in which the numerical Cherenkov instability grows from noise
and saturates, plus the growth rate measured from it.

Run: python tests/golden/make_nci_history.py [128x64|1024x256] [nodal|staggered]
  128x64    about a minute on one CPU core
  1024x256  hours of CPU time: run it with the oracle's OpenMP threads
            (OMP_NUM_THREADS = the host's cores; about half an hour on 8)

Workloads: periodic grid, dx = dy = 0.1 c/omega_pe, pair plasma drifting
along +x at gamma0 = 40 with rest-frame temperature T = 0.01 m c^2
(stratified, e- and e+ co-located), cubic (order-3) shape, CFL 1.0,
theta = 0.6, field CG to 1e-8, seed 0.
  128x64    16 particles/cell/species, 250 steps: the 1024 x 256 single-run
            workload on a smaller grid (same physics per cell);
  1024x256  64 particles/cell/species, 300 steps: the single-run workload
            itself, through the growth and saturation of the instability.
The gather is the method's node-averaged momentum-conserving interpolation
("nodal", written to nci_history_<case>_nodal.json) or the staggered
alternative ("staggered", written to nci_history_<case>.json, the files that
predate the nodal reading; their case records no "gather" key).
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

CASES = {
    "128x64": dict(nx=128, ny=64, dx=0.1, ppc=16, gamma0=40.0, T=0.01, order=3, cfl=1.0,
                   theta=0.6, rtol=1e-8, steps=250, seed=0),
    "1024x256": dict(nx=1024, ny=256, dx=0.1, ppc=64, gamma0=40.0, T=0.01, order=3, cfl=1.0,
                     theta=0.6, rtol=1e-8, steps=300, seed=0),
}


def main(name="128x64", gather="nodal"):
    c = dict(CASES[name], gather=gather)
    suffix = "_nodal" if gather == "nodal" else ""
    out_path = os.path.join(HERE, f"nci_history_{name}{suffix}.json")
    Q = loads.macro_charge(c["gamma0"], c["dx"], c["dx"], c["ppc"])
    ld = loads.pair_plasma_cells(c["nx"], c["ny"], c["ppc"], c["gamma0"], c["T"], c["seed"])
    sp = [oracle.Particles(d["ix"], d["iy"], d["fx"], d["fy"], d["ux"], d["uy"], d["uz"], q, Q)
          for d, q in zip(ld, (-Q, Q))]
    sim = oracle.Sim(c["nx"], c["ny"], c["dx"], c["dx"], c["cfl"], c["theta"], c["order"], sp,
                     rtol=c["rtol"], gather=gather)
    recs = []
    t0 = time.time()
    for n in range(c["steps"]):
        r = sim.step()
        recs.append([r["W_E"], r["W_B"], r["W_K_minus"], r["W_K_plus"], max(r["cg_iters"])])
        if n % 50 == 49 or c["nx"] > 256:
            print(f"step {n + 1}: W_B = {r['W_B']:.4e} ({time.time() - t0:.0f} s)", flush=True)
    a = np.array(recs)
    t = np.arange(c["steps"]) * c["cfl"] * c["dx"]
    g = growth_rate(t, a[:, 1])
    out = dict(case=c, macro_charge=Q, columns=["W_E", "W_B", "W_K_minus", "W_K_plus",
                                                "max_cg_iters"],
               records=a.tolist(), growth=g, oracle_threads=oracle.get_threads(),
               note="FP64 oracle; record n holds W_E, W_B at step n and W_K at n -/+ 1/2")
    with open(out_path, "w") as f:
        json.dump(out, f)
    print("growth", g)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "128x64",
         sys.argv[2] if len(sys.argv) > 2 else "nodal")
