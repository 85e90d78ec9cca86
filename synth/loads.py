"""Seeded synthetic plasma loads shared by the oracle-side tests and the GPU side.

Nothing here is arithmetic of the simulation method (gather, push, deposit,
field solve); these are the initial conditions both sides are handed.

Recipe (readings of the paper's set-up, Sec. 3 first paragraph and Sec. 4):
  * positions: exactly ``ppc`` particles per cell per species, uniform inside
    the cell ("stratified"); electrons and positrons share positions, so the
    initial charge density vanishes and E = B = 0 satisfies Gauss's law.
  * momenta: Maxwell-Juettner with temperature T (units of m c^2) in the flow
    rest frame, then boosted to bulk Lorentz factor gamma0 along +x or -x with
    the flipping method of Zenitani (2015, Phys. Plasmas 22, 042116, Sec. III),
    so the lab-frame ensemble is the drifting Juettner-Synge distribution.
  * the rest-frame speed magnitude is drawn by exact rejection from a
    two-piece envelope (derivation in ``mj_speed``).

Particle k of a species sits in cell k // ppc (row-major, x fastest), so the
load is reproducible item by item from (seed, species, k) alone.
"""
import math

import numpy as np

from .philox import Stream

TAG_POS = 1
TAG_MOM = 2


def _mj_envelope(T):
    """Constants of the two-piece rejection envelope for f(u) ~ u^2 exp(-(g-1)/T)."""
    uc = 5.0 * math.sqrt(T)
    gc = math.sqrt(1.0 + uc * uc)
    s2 = 0.5 * (1.0 + gc) * T          # Gaussian piece variance
    s = math.sqrt(s2)
    # piece A is proposed from the untruncated chi-3 and draws beyond u_c are
    # refused, so its weight is the untruncated mass s^3 sqrt(pi/2)
    mass_a = s ** 3 * math.sqrt(math.pi / 2.0)
    vc = uc / gc                        # slope of the tangent of gamma at uc
    lam = vc / T
    c1 = uc * uc / lam
    c2 = 2.0 * uc / lam ** 2
    c3 = 2.0 / lam ** 3
    mass_b = math.exp(-(gc - 1.0) / T) * (c1 + c2 + c3)
    return dict(uc=uc, gc=gc, s=s, vc=vc, lam=lam,
                pa=mass_a / (mass_a + mass_b),
                mix=(c1 / (c1 + c2 + c3), (c1 + c2) / (c1 + c2 + c3)))


def mj_speed(stream, items, T, first_block=1):
    """Rest-frame Maxwell-Juettner momentum magnitudes u = gamma*v (c = 1).

    Target density f(u) ~ u^2 exp(-(gamma(u) - 1)/T), gamma = sqrt(1 + u^2).
    Envelope, split at u_c:
      u <= u_c: gamma - 1 = u^2/(1 + gamma) >= u^2/(1 + gamma_c), so
                f <= u^2 exp(-u^2/((1 + gamma_c) T))  (a truncated chi-3);
      u >  u_c: gamma is convex, so gamma >= gamma_c + v_c (u - u_c) with
                v_c = u_c/gamma_c, and f <= u^2 exp(-(gamma_c - 1 + v_c(u-u_c))/T),
                i.e. (u_c + w)^2 exp(-lambda w), a 3-term Gamma mixture in w.
    Piece A is proposed from the untruncated chi-3 and given zero acceptance
    beyond u_c, piece B only covers u > u_c; accepting with probability
    f/envelope on each piece then gives exact samples of f.
    Every attempt of item k uses its own counter blocks (first_block + 3*attempt
    + {0,1,2}), so the draw is reproducible per item.
    """
    env = _mj_envelope(T)
    items = np.asarray(items, dtype=np.int64)
    out = np.empty(items.shape, dtype=np.float64)
    todo = np.arange(items.size)
    attempt = 0
    while todo.size:
        it = items[todo]
        blk = first_block + 3 * attempt
        a0, a1 = stream.uniforms(it, blk)        # piece choice, acceptance
        b0, b1 = stream.uniforms(it, blk + 1)    # normals / gamma pieces
        c0, c1 = stream.uniforms(it, blk + 2)
        u = np.empty(it.shape)
        acc = np.zeros(it.shape, dtype=bool)
        pa = a0 < env["pa"]
        # piece A: chi-3 with scale s, from three normals (Box-Muller on b, c)
        r1 = np.sqrt(-2.0 * np.log(b0))
        n1 = r1 * np.cos(2.0 * np.pi * b1)
        n2 = r1 * np.sin(2.0 * np.pi * b1)
        n3 = np.sqrt(-2.0 * np.log(c0)) * np.cos(2.0 * np.pi * c1)
        ua = env["s"] * np.sqrt(n1 * n1 + n2 * n2 + n3 * n3)
        ga = np.sqrt(1.0 + ua * ua)
        loga = -(ga - 1.0) / T + ua * ua / ((1.0 + env["gc"]) * T)
        ok_a = pa & (ua <= env["uc"]) & (np.log(a1) <= loga)
        # piece B: w ~ Gamma(k, 1/lambda), k in {1,2,3} chosen by b0
        e1 = -np.log(b1)
        e2 = -np.log(c0)
        e3 = -np.log(c1)
        k = np.where(b0 < env["mix"][0], 1, np.where(b0 < env["mix"][1], 2, 3))
        w = (e1 + np.where(k >= 2, e2, 0.0) + np.where(k >= 3, e3, 0.0)) / env["lam"]
        ub = env["uc"] + w
        gb = np.sqrt(1.0 + ub * ub)
        logb = -(gb - env["gc"] - env["vc"] * w) / T
        ok_b = (~pa) & (np.log(a1) <= logb)
        u = np.where(pa, ua, ub)
        acc = ok_a | ok_b
        out[todo[acc]] = u[acc]
        todo = todo[~acc]
        attempt += 1
        if attempt > 200:
            raise RuntimeError("Maxwell-Juettner sampler failed to converge")
    return out


def drifting_mj(seed, species, n, T, gamma0, direction=+1, first_item=0):
    """Lab-frame momenta (ux, uy, uz) of n particles, items first_item..first_item+n-1.

    Rest frame: isotropic direction on the unit sphere times a Maxwell-Juettner
    magnitude. Lab frame: flipping method then a Lorentz boost with bulk
    velocity beta = direction*sqrt(1 - 1/gamma0^2) along x:
      if -beta * v'_x > U then u'_x -> -u'_x;  u_x = gamma0 (u'_x + beta gamma').
    """
    stream = Stream(seed, TAG_MOM + 16 * int(species))
    items = np.arange(first_item, first_item + n, dtype=np.int64)
    umag = mj_speed(stream, items, T, first_block=2) if T > 0 else np.zeros(n)
    d0, d1 = stream.uniforms(items, 0)         # direction
    f0, _ = stream.uniforms(items, 1)          # flip decision
    mu = 2.0 * d0 - 1.0
    phi = 2.0 * np.pi * d1
    st = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    ux = umag * mu
    uy = umag * st * np.cos(phi)
    uz = umag * st * np.sin(phi)
    if gamma0 > 1.0:
        beta = float(direction) * math.sqrt(1.0 - 1.0 / (gamma0 * gamma0))
        gp = np.sqrt(1.0 + umag * umag)
        vx = ux / gp
        flip = (-beta * vx) > f0
        ux = np.where(flip, -ux, ux)
        ux = gamma0 * (ux + beta * gp)
    return ux, uy, uz


def stratified_positions(seed, nx, ny, dx, dy, ppc, first_item=0, n=None, x_cells=None):
    """Positions (x, y) of particles k = first_item.., ppc per cell, row-major cells.

    x_cells optionally restricts the load to cells with i in [x_cells[0], x_cells[1]).
    Positions are shared by all species (species-independent stream).
    """
    stream = Stream(seed, TAG_POS)
    if n is None:
        n = nx * ny * ppc - first_item
    items = np.arange(first_item, first_item + n, dtype=np.int64)
    cell = items // ppc
    ci = cell % nx
    cj = cell // nx
    r0, r1 = stream.uniforms(items, 0)
    x = (ci + r0) * dx
    y = (cj + r1) * dy
    return x, y


def pair_plasma(nx, ny, dx, dy, ppc, gamma0, T, seed, direction=+1):
    """Electron/positron load: list of two dicts with x, y, ux, uy, uz (float64)."""
    x, y = stratified_positions(seed, nx, ny, dx, dy, ppc)
    n = x.size
    out = []
    for s in range(2):
        ux, uy, uz = drifting_mj(seed, s, n, T, gamma0, direction)
        out.append(dict(x=x.copy(), y=y.copy(), ux=ux, uy=uy, uz=uz))
    return out


def macro_charge(gamma0, dx, dy, ppc):
    """|q| = m of a macro-particle in units where the flow-frame plasma frequency
    omega_pe = sqrt(4 pi n0 e^2 / (m gamma0)) is one and c = 1 (Sec. 4's
    normalisation, with n0 the lab density of one species)."""
    return gamma0 * dx * dy / (4.0 * math.pi * ppc)


def pair_plasma_cells(nx, ny, ppc, gamma0, T, seed, direction=+1, chunk=1 << 20, workers=None):
    """Same load as pair_plasma, returned as cell index + in-cell offset
    (exact: offset = the uniform draw) and generated in parallel chunks.

    Returns a list of two dicts with ix, iy (int32), fx, fy, ux, uy, uz (float64).
    """
    import os
    from concurrent.futures import ThreadPoolExecutor

    n = nx * ny * ppc
    out = [dict(ix=np.empty(n, np.int32), iy=np.empty(n, np.int32), fx=np.empty(n),
                fy=np.empty(n), ux=np.empty(n), uy=np.empty(n), uz=np.empty(n))
           for _ in range(2)]
    pos = Stream(seed, TAG_POS)

    def work(k0):
        k1 = min(n, k0 + chunk)
        items = np.arange(k0, k1, dtype=np.int64)
        cell = items // ppc
        r0, r1 = pos.uniforms(items, 0)
        for s in range(2):
            o = out[s]
            o["ix"][k0:k1] = cell % nx
            o["iy"][k0:k1] = cell // nx
            o["fx"][k0:k1] = r0
            o["fy"][k0:k1] = r1
            ux, uy, uz = drifting_mj(seed, s, k1 - k0, T, gamma0, direction, first_item=k0)
            o["ux"][k0:k1] = ux
            o["uy"][k0:k1] = uy
            o["uz"][k0:k1] = uz

    workers = workers or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        list(ex.map(work, range(0, n, chunk)))
    return out


def shock_load(x_out, ny, ppc, gamma0, T, seed):
    """Initial plasma of a shock run: the flow fills the cells with i < x_out,
    moving towards -x (the reflecting wall is at x = 0). Same recipe as
    pair_plasma_cells on an x_out x ny grid."""
    return pair_plasma_cells(x_out, ny, ppc, gamma0, T, seed, direction=-1)


def shock_injection(x_out, ny, ppc, gamma0, T, seed, step, cfl):
    """Flow entering a shock run through x_out = x_out cells before step `step`.

    The stream moves w = beta0 * cfl cells per step (beta0 = sqrt(1 - 1/gamma0^2)),
    so a slab of width w behind x_out is refilled each step at ppc per cell:
    per row, floor(ppc w (step+1)) - floor(ppc w step) particles, at x uniform
    in (x_out - w, x_out) and y uniform in the row; electrons and positrons
    co-located; momenta drifting Maxwell-Juettner towards -x. Items continue
    after those of shock_load, so every injected particle has its own counter.
    Returns a list of two dicts (ix, iy, fx, fy, ux, uy, uz).
    """
    beta0 = math.sqrt(1.0 - 1.0 / (gamma0 * gamma0)) if gamma0 > 1.0 else 0.0
    w = beta0 * cfl
    done = math.floor(ppc * w * step)
    per_row = math.floor(ppc * w * (step + 1)) - done
    n = per_row * ny
    base = x_out * ny * ppc + done * ny
    items = np.arange(base, base + n, dtype=np.int64)
    r0, r1 = Stream(seed, TAG_POS).uniforms(items, 0)
    X = x_out - w * r0
    ix = np.floor(X).astype(np.int32)
    row = (np.arange(n) // max(per_row, 1)).astype(np.int32)
    out = []
    for s in range(2):
        ux, uy, uz = drifting_mj(seed, s, n, T, gamma0, -1, first_item=base)
        out.append(dict(ix=ix.copy(), iy=row.copy(), fx=X - ix, fy=r1.copy(), ux=ux, uy=uy,
                        uz=uz))
    return out
