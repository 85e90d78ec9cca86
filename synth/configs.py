"""Workload tables (parameters only; no arithmetic of the method).

The batched parameter sweep: 48 periodic pair-plasma runs at gamma0 = 20,
T = 0.01, dx = 0.1, 500 steps each, over CFL {0.5..1.0} x shape order {1,2,3}
x theta {0.5, 0.6} (the scans of Sec. 3.2-3.3 in spirit). 6 x 3 x 2 = 36
combinations; runs 0-35 are that factorial (CFL-major, then order, then
theta) and runs 36-47 repeat the 12 (CFL, theta) pairs at order 2 (the
paper's default order, Sec. 3) with seed + 1000. Grid and ppc cycle so the
runs are uneven: grid = [128x64, 256x64, 256x128, 512x128][r mod 4],
ppc = [8, 16, 32][(r div 4) mod 3], seed = r.
"""

CFLS = (0.5, 0.6, 0.7, 0.8, 0.9, 1.0)
ORDERS = (1, 2, 3)
THETAS = (0.5, 0.6)
GRIDS = ((128, 64), (256, 64), (256, 128), (512, 128))
PPCS = (8, 16, 32)


def sweep_runs():
    runs = []
    for r in range(48):
        if r < 36:
            cfl = CFLS[r // 6]
            order = ORDERS[(r // 2) % 3]
            theta = THETAS[r % 2]
            seed = r
        else:
            k = r - 36
            cfl = CFLS[k // 2]
            order = 2
            theta = THETAS[k % 2]
            seed = r + 1000
        nx, ny = GRIDS[r % 4]
        ppc = PPCS[(r // 4) % 3]
        runs.append(dict(run=r, nx=nx, ny=ny, ppc=ppc, cfl=cfl, order=order, theta=theta,
                         gamma0=20.0, T=0.01, dx=0.1, seed=seed, steps=500))
    return runs
