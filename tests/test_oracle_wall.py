"""Pins of the oracle's shock set-up (a reading: conducting walls at x = 0 and
x = (nx-1) dx, specular reflection at x = 0, outflow at x_out; the paper only
says the flow is injected at one side and reflected at the other, Sec. 4).

The Laplacian form of Eq. (7) needs boundary rows at the walls; they are
checked against what does not depend on them: the curl form of Eqs. (5)-(6)
with the conductor nodes held at zero, energy conservation of the
Crank-Nicolson case (theta = 1/2) in vacuum, symmetry and definiteness of the
operator, a dense solve, and the discrete continuity equation of the folded
deposit."""
import numpy as np
import pytest

import oracle

DX = 0.1


def _p(X, Y, ux, uy, uz, q=1.0, m=1.0):
    X = np.asarray(X, float)
    Y = np.asarray(Y, float)
    ix = np.floor(X).astype(np.int32)
    iy = np.floor(Y).astype(np.int32)
    return oracle.Particles(ix, iy, X - ix, Y - iy, ux, uy, uz, q, m)


def test_specular_reflection_single_particle():
    nx, ny = 16, 8
    u = -3.0                                   # moving towards the wall
    p = _p([0.3], [4.5], [u], [0.4], [0.2])
    sim = oracle.Sim(nx, ny, DX, DX, 1.0, 0.6, 2, [p], bc="shock")
    g = np.sqrt(1 + u * u + 0.4 ** 2 + 0.2 ** 2)
    X1 = 0.3 + sim.dt * u / g / DX             # fields are zero: u is unchanged
    assert X1 < 0
    sim.step()
    q = sim.species[0]
    assert q.n == 1
    assert q.ix[0] + q.fx[0] == pytest.approx(-X1, abs=1e-15)
    assert q.ux[0] == -u and q.uy[0] == 0.4 and q.uz[0] == 0.2


def test_outflow_removes_particles():
    nx, ny = 16, 8
    xo = nx - oracle.WALL_GAP
    p = _p([xo - 0.2, xo - 3.0], [2.5, 2.5], [5.0, 5.0], [0.0, 0.0], [0.0, 0.0])
    sim = oracle.Sim(nx, ny, DX, DX, 1.0, 0.6, 1, [p], bc="shock")
    sim.step()
    q = sim.species[0]
    assert q.n == 1 and q.ids[0] == 1


@pytest.mark.parametrize("order", [1, 2, 3])
def test_folded_deposit_keeps_continuity(order):
    nx, ny = 16, 10
    rng = np.random.default_rng(order)
    n = 200
    X = rng.uniform(0.0, 2.5, n)
    Y = rng.uniform(0.0, ny, n)
    ux = rng.uniform(-8.0, 8.0, n)             # many cross the wall
    uy = rng.uniform(-3.0, 3.0, n)
    uz = rng.uniform(-1.0, 1.0, n)
    p = _p(X, Y, ux, uy, uz, q=0.7)
    rho0 = oracle.charge_wall(nx, ny, order, DX, DX, p)
    sim = oracle.Sim(nx, ny, DX, DX, 0.9, 0.6, order, [p], bc="shock")
    old = p.copy()
    oracle.move(p, sim.dt, DX, DX)
    crossed = int(np.sum(p.ix < 0))
    assert crossed > 20
    J = [np.zeros((ny, nx)) for _ in range(3)]
    oracle.deposit_wall(nx, ny, order, DX, DX, sim.dt, old, p, J)
    oracle.boundary_wall(nx, ny, p)
    assert p.n == n and np.all(p.ix >= 0)
    rho1 = oracle.charge_wall(nx, ny, order, DX, DX, p)
    div = oracle.div_e(nx, ny, DX, DX, J[0], J[1])
    res = (rho1 - rho0) / sim.dt + div
    scale = np.abs(rho1 - rho0).max() / sim.dt
    # every node off the wall line (node 0 holds the wall's surface charge)
    assert np.abs(res[:, 1:nx - 1]).max() <= 1e-12 * scale


def _dense(nx, ny, c, theta=0.6, cfl=1.0):
    n = nx * ny
    M = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        M[:, k] = oracle.apply_A_wall(nx, ny, DX, DX, cfl * DX, theta, c,
                                      e.reshape(ny, nx)).ravel()
    return M


def _fixed_cols(nx, c):
    return [0, nx - 1] if c == 0 else [nx - 1]


@pytest.mark.parametrize("c", [0, 1, 2])
def test_wall_operator_symmetric_positive(c):
    nx, ny = 9, 6
    M = _dense(nx, ny, c)
    fixed = np.zeros((ny, nx), bool)
    fixed[:, _fixed_cols(nx, c)] = True
    f = fixed.ravel()
    # fixed rows are identity rows and free rows do not couple to them
    assert np.array_equal(M[f][:, f], np.eye(f.sum()))
    assert np.all(M[~f][:, f] == 0) and np.all(M[f][:, ~f] == 0)
    A = M[~f][:, ~f]
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(A).min() >= 1.0 - 1e-12


@pytest.mark.parametrize("c", [0, 1, 2])
def test_wall_cg_matches_dense_solve(c):
    nx, ny = 9, 6
    M = _dense(nx, ny, c)
    b = np.random.default_rng(10 + c).standard_normal((ny, nx))
    b[:, _fixed_cols(nx, c)] = 0.0
    x, it, rel = oracle.cg_wall(nx, ny, DX, DX, DX, 0.6, c, b, rtol=1e-14, maxit=500)
    assert rel <= 1e-13
    ref = np.linalg.solve(M, b.ravel()).reshape(ny, nx)
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()


def _walled_fields(nx, ny, rng):
    """E zero on the conductor nodes; B divergence-free with Bx zero on both
    walls: Bx = d psi/dy, By = -d psi/dx from psi at nodes, psi = 0 on the
    wall lines; By, Bz zero in the outside column."""
    E = [rng.standard_normal((ny, nx)) for _ in range(3)]
    E[1][:, 0] = E[2][:, 0] = 0.0
    E[0][:, nx - 1] = E[1][:, nx - 1] = E[2][:, nx - 1] = 0.0
    psi = rng.standard_normal((ny, nx))
    psi[:, 0] = psi[:, nx - 1] = 0.0
    bx = (np.roll(psi, -1, axis=0) - psi) / DX
    by = -(np.roll(psi, -1, axis=1) - psi) / DX
    bz = rng.standard_normal((ny, nx))
    by[:, nx - 1] = 0.0
    bz[:, nx - 1] = 0.0
    return E, [bx, by, bz]


def _curl_e(nx, ny, F):
    """forward-difference curl at the B points (same as the periodic oracle's)"""
    fx, fy, fz = F
    cx = (np.roll(fz, -1, axis=0) - fz) / DX
    cy = -(np.roll(fz, -1, axis=1) - fz) / DX
    cz = (np.roll(fy, -1, axis=1) - fy) / DX - (np.roll(fx, -1, axis=0) - fx) / DX
    return [cx, cy, cz]


@pytest.mark.parametrize("theta", [0.5, 0.6, 1.0])
def test_wall_solve_satisfies_curl_form(theta):
    """dB from the Laplacian form with wall rows equals
    -dt curl_E((1-theta) E^n + theta E^{n+1}) at every free B row."""
    nx, ny = 12, 8
    rng = np.random.default_rng(int(theta * 10))
    E, B = _walled_fields(nx, ny, rng)
    J = [rng.standard_normal((ny, nx)) for _ in range(3)]
    oracle.mask_wall_currents(nx, ny, J)
    sim = oracle.Sim(nx, ny, DX, DX, 1.0, theta, 1, [], rtol=1e-14, maxit=1000, bc="shock")
    sim.E = [a.copy() for a in E]
    sim.B = [a.copy() for a in B]
    sim.J = J
    db, its, rels = sim.field_solve()
    assert max(rels) <= 1e-13
    mix = [(1 - theta) * E[k] + theta * sim.E[k] for k in range(3)]
    ce = _curl_e(nx, ny, mix)
    for c in range(3):
        cols = np.ones(nx, bool)
        cols[_fixed_cols(nx, c)] = False
        ref = -sim.dt * ce[c]
        err = np.abs(db[c] - ref)[:, cols].max()
        assert err <= 1e-11 * np.abs(ref).max(), (c, err)
        assert np.all(db[c][:, ~cols] == 0.0)
    # the conductor E nodes stay zero
    assert np.all(sim.E[1][:, 0] == 0) and np.all(sim.E[2][:, 0] == 0)
    assert np.all(sim.E[0][:, nx - 1] == 0) and np.all(sim.E[2][:, nx - 1] == 0)


def test_crank_nicolson_vacuum_energy_with_walls():
    nx, ny = 14, 10
    rng = np.random.default_rng(3)
    E, B = _walled_fields(nx, ny, rng)
    sim = oracle.Sim(nx, ny, DX, DX, 1.0, 0.5, 1, [], rtol=1e-14, maxit=1000, bc="shock")
    sim.E = E
    sim.B = B
    w0 = sum(sim.field_energy())
    for _ in range(20):
        sim.field_solve()
    w1 = sum(sim.field_energy())
    assert abs(w1 - w0) <= 1e-10 * w0


# staggered offsets (cells) of Ex, Ey, Ez, Bx, By, Bz on the Yee grid
STAG = [(0.5, 0.0), (0.0, 0.5), (0.0, 0.0), (0.0, 0.5), (0.5, 0.0), (0.5, 0.5)]
ODD = (False, True, True, True, False, False)   # conductor image of each component


def _near_wall(order, n=300, seed=0):
    rng = np.random.default_rng(seed + order)
    # within the reach of the shape behind the wall: x in [0, 2.5) cells
    return _p(rng.uniform(0.0, 2.5, n), rng.uniform(3.0, 7.0, n), np.zeros(n), np.zeros(n),
              np.zeros(n))


def _interp_x(order, X, s, value_at):
    """sum_i S_p(X - s - i) value_at(i) over the support (numpy, for the
    values that a wrong image rule would give)"""
    out = np.zeros_like(X)
    for k, x in enumerate(X):
        for i in range(int(np.floor(x - s)) - 2, int(np.floor(x - s)) + 3):
            out[k] += oracle.shape(order, x - s - i) * value_at(i)
    return out


@pytest.mark.parametrize("order", [1, 2, 3])
def test_wall_gather_odd_images(order):
    """Integer-x components (Ey, Ez, Bx) vanish on the wall line and continue
    as odd images behind it: a field a x (y + 1) with x their own coordinate
    is reproduced exactly at every particle near the wall, as the odd
    extension of a x is a x itself. An even image, or a mirror one column off,
    would give other values there (checked below: the shape reaches behind
    the wall)."""
    nx, ny = 24, 10
    p = _near_wall(order)
    X, Y = p.ix + p.fx, p.iy + p.fy
    J, I = np.mgrid[0:ny, 0:nx].astype(float)
    f = []
    for (sx, sy), odd in zip(STAG, ODD):
        f.append(0.7 * (I + sx) * (J + sy + 1.0) if odd else np.zeros((ny, nx)))
    g = oracle.gather_wall(nx, ny, order, f, p, mode="staggered")
    for c, odd in enumerate(ODD):
        if odd:
            assert np.allclose(g[c], 0.7 * X * (Y + 1.0), rtol=0, atol=1e-12), c
    # the test separates the image rules: along x, an even image (|i|) or a
    # mirror one column off (i + 1 behind the wall) differ from x itself
    # (the linear shape of order 1 never reaches an integer column behind x = 0)
    exact = _interp_x(order, X, 0.0, lambda i: float(i))
    assert np.allclose(exact, X, atol=1e-12)
    for wrong in (lambda i: float(abs(i)), lambda i: float(i if i >= 0 else i + 1)):
        d = np.abs(_interp_x(order, X, 0.0, wrong) - X).max()
        assert (d > 1e-2) if order >= 2 else (d < 1e-12)


@pytest.mark.parametrize("order", [1, 2, 3])
def test_wall_gather_even_images(order):
    """Half-integer-x components (Ex, By, Bz) continue as even images about
    the wall line (index -i-1 mirrors i, both at distance i + 1/2): a field
    b + x^2 in their own coordinate gathers to b + X^2 + m_p(X - 1/2), the
    value of the even extension (the shape's second moment m_p is (p+1)/12
    for p >= 2 and f(1 - f) for p = 1). A uniform field is reproduced exactly.
    An odd image or a mirror one column off would give other values."""
    nx, ny = 24, 10
    p = _near_wall(order, seed=10)
    X = p.ix + p.fx
    J, I = np.mgrid[0:ny, 0:nx].astype(float)
    f = []
    for (sx, sy), odd in zip(STAG, ODD):
        f.append(np.zeros((ny, nx)) if odd else 0.4 + (I + sx) ** 2)
    g = oracle.gather_wall(nx, ny, order, f, p, mode="staggered")
    t = X - 0.5
    fr = t - np.floor(t)
    m = (order + 1) / 12.0 if order >= 2 else fr * (1 - fr)
    want = 0.4 + X ** 2 + m
    for c, odd in enumerate(ODD):
        if not odd:
            assert np.allclose(g[c], want, rtol=0, atol=1e-11), c
    u = [np.zeros((ny, nx)) if odd else np.full((ny, nx), -1.3) for odd in ODD]
    gu = oracle.gather_wall(nx, ny, order, u, p, mode="staggered")
    for c, odd in enumerate(ODD):
        if not odd:
            assert np.allclose(gu[c], -1.3, rtol=0, atol=1e-13), c
    # the test separates the image rules: index i >= 0 holds 0.4 + (i + 1/2)^2;
    # behind the wall the even image (index -i-1) holds the same function of
    # the position, an odd image its negative, a mirror one column off (-i)
    # the value one cell further out
    val = lambda i: 0.4 + (i + 0.5) ** 2
    exact = _interp_x(order, X, 0.5, lambda i: val(i) if i >= 0 else val(-i - 1))
    assert np.allclose(exact, want, atol=1e-11)
    for wrong in (lambda i: val(i) if i >= 0 else -val(-i - 1),
                  lambda i: val(i) if i >= 0 else val(-i)):
        assert np.abs(_interp_x(order, X, 0.5, wrong) - want).max() > 1e-2


@pytest.mark.parametrize("order", [1, 2, 3])
def test_wall_nodal_gather_images(order):
    """The node-averaged gather with the conductor images: the odd components
    (Ey, Ez, Bx) of a field a x (y + 1) in their own coordinates average onto
    the nodes as a x (y + 1) (linear; the y average of Ey and Bx is exact) and
    are reproduced at every particle near the wall; the even components (Ex,
    By, Bz) of b + x^2 average onto node i as b + i^2 + 1/4, behind the wall
    too (their even image is the same function of the position), and gather
    to b + X^2 + m_p(X) + 1/4. An odd image of an even component, or a
    mirror one column off, changes the averages of the first columns and
    fails."""
    nx, ny = 24, 10
    p = _near_wall(order, seed=20)
    X, Y = p.ix + p.fx, p.iy + p.fy
    J, I = np.mgrid[0:ny, 0:nx].astype(float)
    f = []
    for (sx, sy), odd in zip(STAG, ODD):
        f.append(0.7 * (I + sx) * (J + sy + 1.0) if odd else 0.4 + (I + sx) ** 2)
    g = oracle.gather_wall(nx, ny, order, f, p, mode="nodal")
    fr = X - np.floor(X)
    m = (order + 1) / 12.0 if order >= 2 else fr * (1 - fr)
    for c, odd in enumerate(ODD):
        want = 0.7 * X * (Y + 1.0) if odd else 0.4 + X ** 2 + m + 0.25
        assert np.allclose(g[c], want, rtol=0, atol=1e-11), c
