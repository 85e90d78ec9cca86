"""The paper's numerical-Cherenkov studies (Sec. 3) on the GPU library.

Set-up of Sec. 3: a periodic 128 x 128 grid, cell = Debye length (0.1 c/omega_pe
with the rest-frame thermal speed 0.1 c, i.e. T = 0.01 m c^2), electrons and
positrons at 100 particles per cell drifting along +x at Gamma = 100
(V = 0.9999 c), fields zero at t = 0, second-order shape and theta = 0.501
unless a scan varies them. Time is measured in dx/c, as in the paper's
figures.

* cfl_scan: growth of the magnetic energy for CFL numbers 0.4 ... 1.0
  (Fig. 4; the fast-growing instability, suppressed at sigma = 1.0);
* theta_scan: the slowly growing mode at sigma = 1.0 over t ~ 5000 dx/c for
  several implicitness factors and shape orders (Figs. 5-6);
* cherenkov_locus: the resonance curve of Eq. (17) and the B_z power
  spectrum peaks against it (Fig. 3);
* growth_rate: half the least-squares slope of ln W_B over the exponential
  phase (the paper does not say how it measured its rates; this reading: the
  phase starts at the first sample above 10x the median of the first 51
  samples and ends at the first sample above 0.1 x max W_B, needs >= 20
  samples and a coefficient of determination >= 0.95).

Each scan runs all its cases as one batched context (one launch per kernel
for all runs). Runs of one context share precision and tile shape.
"""
import math

import numpy as np

DX = 0.1            # cell = Debye length, in c/omega_pe
GAMMA = 100.0       # bulk Lorentz factor of the flow
T_REST = 0.01       # rest-frame temperature (thermal speed 0.1 c)
NCELL = 128
PPC = 100


def growth_rate(t, wb, n_floor=51, min_samples=20, min_r2=0.95):
    """Amplitude growth rate (per unit of t) from a magnetic-energy history,
    or None when no exponential phase is found."""
    t = np.asarray(t, dtype=np.float64)
    w = np.asarray(wb, dtype=np.float64)
    if w.size < max(n_floor, min_samples) or not np.all(np.isfinite(w)):
        return None
    start = np.flatnonzero(w > 10.0 * np.median(w[:n_floor]))
    if start.size == 0:
        return None
    stop = np.flatnonzero(w > 0.1 * w.max())
    i0 = int(start[0])
    i1 = int(stop[0]) if stop.size else w.size - 1
    n = i1 - i0 + 1
    if n < min_samples or np.any(w[i0:i1 + 1] <= 0):
        return None
    x = t[i0:i1 + 1]
    y = np.log(w[i0:i1 + 1])
    xm, ym = x.mean(), y.mean()
    sxx = float(((x - xm) ** 2).sum())
    sxy = float(((x - xm) * (y - ym)).sum())
    syy = float(((y - ym) ** 2).sum())
    if sxx <= 0 or syy <= 0:
        return None
    slope = sxy / sxx
    r2 = sxy * sxy / (sxx * syy)
    if r2 < min_r2:
        return None
    return dict(rate=0.5 * slope, t0=float(x[0]), t1=float(x[-1]), r2=r2, samples=n)


def cherenkov_locus(kx_dx, sigma, V=None):
    """ky dy of Eq. (17) at the given kx dx (dx = dy): where the entropy mode
    omega = V kx crosses the theta = 1/2 dispersion surface of Eq. (15);
    NaN where there is no crossing."""
    if V is None:
        V = math.sqrt(1.0 - 1.0 / GAMMA ** 2)
    kx_dx = np.asarray(kx_dx, dtype=np.float64)
    half = 0.5 * V * sigma * kx_dx          # V kx dt / 2
    sx = sigma * np.sin(0.5 * kx_dx)
    with np.errstate(invalid="ignore"):
        inner = np.sqrt(np.tan(half) ** 2 - sx ** 2) / sigma
        return 2.0 * np.arcsin(inner)


def _run_descs(pic, cases, rtol):
    from synth import loads
    descs = []
    for c in cases:
        Q = loads.macro_charge(GAMMA, DX, DX, c["ppc"])
        descs.append(pic.run_desc(c["n"], c["n"], DX, c["cfl"], c["theta"], c["order"],
                                  [(-Q, Q, c["ppc"]), (Q, Q, c["ppc"])], cg_rtol=rtol,
                                  cg_maxit=400))
    return descs


def run_batch(pic, cases, steps, precision="fp32", spectra_at=None, seed=0, rtol=1e-8,
              tile=(16, 16), on_chunk=None):
    """Run the cases (dicts: n, ppc, cfl, theta, order) as one context for
    `steps` steps, recording W_E, W_B every step. Returns per case the time
    (dx/c), W_B, W_E, the growth rate and, if spectra_at = t (dx/c), the B_z
    power spectrum at the first step with t >= that value."""
    descs = _run_descs(pic, cases, rtol)
    sim = pic.Sim(descs, pic.make_options(precision, tile=tile, track_ids=False, diag_every=1,
                                          history_cap=steps + 1, slack=1.0))
    for r, c in enumerate(cases):
        for s in range(2):
            sim.load_plasma(r, s, c["ppc"], GAMMA, T_REST, seed + r)
    spectra = [None] * len(cases)
    done = 0
    while done < steps:
        k = min(100, steps - done)
        if spectra_at is not None:
            # stop at the step where a case first reaches the spectrum time
            for r, c in enumerate(cases):
                if spectra[r] is None:
                    n_at = int(math.ceil(spectra_at / c["cfl"]))
                    if done < n_at <= done + k:
                        k = n_at - done
        sim.step(k)
        done += k
        if spectra_at is not None:
            for r, c in enumerate(cases):
                if spectra[r] is None and done * c["cfl"] >= spectra_at:
                    spectra[r] = sim.spectrum(r, "Bz")
        if on_chunk:
            on_chunk(done)
    out = []
    for r, c in enumerate(cases):
        h = sim.history(r)
        t = np.array([x["step"] for x in h], dtype=np.float64) * c["cfl"]   # dx/c
        wb = np.array([x["W_B"] for x in h])
        we = np.array([x["W_E"] for x in h])
        wk = np.array([0.5 * (x["W_K_minus"] + x["W_K_plus"]) for x in h])
        d = sim.diag(r)
        out.append(dict(case=c, t=t, W_B=wb, W_E=we, W_K=wk, growth=growth_rate(t, wb),
                        spectrum=spectra[r], gauss_max=d["gauss_max"],
                        energy_drift=float(np.abs((we + wb + wk) / (we[0] + wb[0] + wk[0]) - 1)
                                           .max())))
    sim.close()
    return out


def cfl_scan(pic, sigmas=(0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0), orders=(1, 2), theta=0.501,
             t_end=400.0, n=NCELL, ppc=PPC, **kw):
    """Fig. 4: growth of W_B for each CFL number and shape order, to t_end
    (dx/c) for every run (steps = t_end / min sigma)."""
    cases = [dict(n=n, ppc=ppc, cfl=s, theta=theta, order=o) for o in orders for s in sigmas]
    steps = int(math.ceil(t_end / min(sigmas)))
    return run_batch(pic, cases, steps, **kw)


def theta_scan(pic, thetas=(0.5, 0.501, 0.502, 0.503), orders=(1, 2), sigma=1.0, t_end=5000.0,
               n=NCELL, ppc=PPC, **kw):
    """Figs. 5-6: the slowly growing mode at sigma = 1 for several
    implicitness factors and shape orders, to t_end (dx/c)."""
    cases = [dict(n=n, ppc=ppc, cfl=sigma, theta=th, order=o) for o in orders for th in thetas]
    steps = int(math.ceil(t_end / sigma))
    return run_batch(pic, cases, steps, **kw)


def spectrum_peaks(power, count=20):
    """The `count` largest entries of a power map ([ny][nx], DFT order) as
    (kx dx, ky dy, power) with wavenumbers in (-pi, pi]."""
    ny, nx = power.shape
    flat = np.argsort(power, axis=None)[::-1][:count]
    jy, ix = np.unravel_index(flat, power.shape)
    kx = 2 * np.pi * np.where(ix > nx // 2, ix - nx, ix) / nx
    ky = 2 * np.pi * np.where(jy > ny // 2, jy - ny, jy) / ny
    return kx, ky, power[jy, ix]


def locus_distance(kx_dx, ky_dy, sigma):
    """Distance in ky dy of each point to the nearer branch (+ or -) of the
    Eq. (17) curve at its kx (inf where the curve has no point at that kx)."""
    ky = cherenkov_locus(np.abs(kx_dx), sigma)
    d = np.abs(np.abs(ky_dy) - ky)
    return np.where(np.isfinite(d), d, np.inf)
