"""Pins of the oracle's particle steps (shape, gather, push, move, deposit)
against closed forms, invariants and hand cases; CPU only."""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

HERE = os.path.dirname(__file__)
HAND = json.load(open(os.path.join(HERE, "golden", "hand_cases.json")))
ORDERS = (1, 2, 3)


# ---------------------------------------------------------------- shapes
@pytest.mark.parametrize("order", ORDERS)
def test_shape_moments(ora, order):
    """B-spline of degree p: partition of unity and exact first moment at any
    position; the second moment about x is (p+1)/12 (the variance of p+1
    convolved unit boxes) for p >= 2, and f(1-f) for p = 1 (f = frac x)."""
    rng = np.random.default_rng(order)
    for x in rng.uniform(-5, 5, 50):
        nodes = np.arange(math.floor(x) - 4, math.floor(x) + 5)
        w = np.array([ora.shape(order, x - i) for i in nodes])
        assert abs(w.sum() - 1.0) < 1e-14
        assert abs((w * nodes).sum() - x) < 1e-13
        m2 = (w * (nodes - x) ** 2).sum()
        f = x - math.floor(x)
        want = (order + 1) / 12.0 if order >= 2 else f * (1 - f)
        assert abs(m2 - want) < 1e-13


@pytest.mark.parametrize("order", (2, 3))
def test_shape_is_box_convolution(ora, order):
    """S_p(d) = integral of S_{p-1} over [d - 1/2, d + 1/2] (B-spline recursion)."""
    for d in np.linspace(-2.3, 2.3, 37):
        ref, _ = integrate.quad(lambda t: ora.shape(order - 1, t), d - 0.5, d + 0.5,
                                points=[-1.5, -1, -0.5, 0, 0.5, 1, 1.5], limit=200)
        assert abs(ora.shape(order, d) - ref) < 1e-12


@pytest.mark.parametrize("order", ORDERS)
def test_node_weights_hand(ora, order):
    want = HAND["node_weights"][str(order)]
    got = [ora.shape(order, d) for d in (-1.0, 0.0, 1.0)]
    assert np.allclose(got, want, rtol=0, atol=1e-15)


# ---------------------------------------------------------------- gather
def _particles(ora, rng, n, nx, ny, lo=3, hi=None):
    hi = (nx - 3) if hi is None else hi
    x = rng.uniform(lo, hi, n)
    y = rng.uniform(lo, ny - 3, n)
    z = np.zeros(n)
    return ora.Particles.from_xy(x, y, z, z, z, 1.0, 1.0, 1.0, 1.0)


STAG = [(0.5, 0.0), (0.0, 0.5), (0.0, 0.0), (0.0, 0.5), (0.5, 0.0), (0.5, 0.5)]


def _second_moment(order, t):
    """sum_i S_p(t - i) i^2 - t^2: (p+1)/12 for p >= 2, frac(t)(1 - frac(t))
    for p = 1 (closed forms of the B-spline's second moment)."""
    f = t - np.floor(t)
    return np.full_like(t, (order + 1) / 12.0) if order >= 2 else f * (1 - f)


@pytest.mark.parametrize("order", ORDERS)
def test_gather_quadratic_pins_shape_order_per_axis(ora, order):
    """Staggered gather (the alternative reading): a field quadratic in one
    coordinate of each component's own staggered points gathers to
    t^2 + m_p(t) along that axis, with m_p the order-p second moment: every
    component must use the full order-p shape in both directions. A component
    interpolated with a lower order along its staggered direction, or a wrong
    stagger offset, fails."""
    nx = ny = 20
    rng = np.random.default_rng(40 + order)
    p = _particles(ora, rng, 300, nx, ny, lo=4, hi=nx - 4)
    J, I = np.mgrid[0:ny, 0:nx].astype(float)
    X = p.ix + p.fx
    Y = p.iy + p.fy
    for axis in (0, 1):
        f = []
        for sx, sy in STAG:
            t = (I + sx) if axis == 0 else (J + sy)
            f.append(0.2 + t * t)
        g = ora.gather(nx, ny, order, f, p, mode="staggered")
        for c, (sx, sy) in enumerate(STAG):
            # sum_i S(P - s - i) (i + s)^2 = P^2 + m_p(P - s), P the particle's
            # coordinate and s the component's stagger along the axis
            P, sh = (X, sx) if axis == 0 else (Y, sy)
            want = 0.2 + P ** 2 + _second_moment(order, P - sh)
            assert np.allclose(g[c], want, rtol=0, atol=1e-11), (axis, c)


@pytest.mark.parametrize("mode", ["nodal", "staggered"])
@pytest.mark.parametrize("order", ORDERS)
def test_gather_uniform_and_linear(ora, order, mode):
    """Both gathers: uniform fields are reproduced exactly; a field linear in
    the physical coordinate of each component's own staggered points is
    reproduced at the particle position (a wrong stagger offset, or an
    average onto the nodes taken with the wrong neighbour, is caught)."""
    nx = ny = 16
    rng = np.random.default_rng(10 + order)
    p = _particles(ora, rng, 200, nx, ny)
    consts = [1.5, -2.0, 0.25, 3.0, -0.5, 7.0]
    f = [np.full((ny, nx), c) for c in consts]
    g = ora.gather(nx, ny, order, f, p, mode=mode)
    for c in range(6):
        assert np.allclose(g[c], consts[c], rtol=0, atol=1e-13)
    J, I = np.mgrid[0:ny, 0:nx].astype(float)
    f = [0.3 + 0.7 * (I + sx) - 1.1 * (J + sy) for sx, sy in STAG]
    g = ora.gather(nx, ny, order, f, p, mode=mode)
    X = p.ix + p.fx
    Y = p.iy + p.fy
    for c in range(6):
        assert np.allclose(g[c], 0.3 + 0.7 * X - 1.1 * Y, rtol=0, atol=1e-12)


@pytest.mark.parametrize("order", ORDERS)
def test_nodal_gather_quadratic_pins_averaging(ora, order):
    """Node-averaged gather (the method's momentum-conserving interpolation):
    a field quadratic in one coordinate t of each component's own Yee points
    averages onto node i as i^2 + 1/4 along an axis where the component is
    staggered (((i - 1/2)^2 + (i + 1/2)^2)/2) and i^2 where it is not, and the
    node-centred order-p shape then adds its second moment m_p(P): the
    gathered value is c + P^2 + m_p(P) + (1/4 if staggered along that axis).
    An average taken along the wrong axis, with the wrong neighbour (i + 1
    instead of i - 1 shifts the value by 2P + 1), over two instead of four
    points for Bz, or a shape of another order fails."""
    nx = ny = 20
    rng = np.random.default_rng(70 + order)
    p = _particles(ora, rng, 300, nx, ny, lo=4, hi=nx - 4)
    J, I = np.mgrid[0:ny, 0:nx].astype(float)
    X = p.ix + p.fx
    Y = p.iy + p.fy
    for axis in (0, 1):
        f = []
        for sx, sy in STAG:
            t = (I + sx) if axis == 0 else (J + sy)
            f.append(0.2 + t * t)
        g = ora.gather(nx, ny, order, f, p, mode="nodal")
        for c, (sx, sy) in enumerate(STAG):
            P, sh = (X, sx) if axis == 0 else (Y, sy)
            want = 0.2 + P ** 2 + _second_moment(order, P) + (0.25 if sh else 0.0)
            assert np.allclose(g[c], want, rtol=0, atol=1e-11), (axis, c)


@pytest.mark.parametrize("order", ORDERS)
def test_nodal_gather_periodic_translation(ora, order):
    """Periodic wrap of the averages: shifting the fields by (mx, my) cells and
    every particle by the same amount leaves the gathered values unchanged,
    also for particles whose shape or averages reach across the edges."""
    nx, ny = 12, 10
    rng = np.random.default_rng(90 + order)
    f = [rng.normal(size=(ny, nx)) for _ in range(6)]
    x = rng.uniform(0, nx, 200)
    y = rng.uniform(0, ny, 200)
    x[:20] = rng.uniform(0, 1.5, 20)           # near the low edges
    y[20:40] = rng.uniform(ny - 1.5, ny, 20)    # near the high edges
    u = np.zeros((3, 200))
    p = ora.Particles.from_xy(x, y, u[0], u[1], u[2], 1.0, 1.0, 1.0, 1.0)
    g0 = ora.gather(nx, ny, order, f, p, mode="nodal")
    for mx, my in ((3, 0), (0, 4), (5, 7)):
        fs = [np.roll(np.roll(a, my, axis=0), mx, axis=1) for a in f]
        ps = ora.Particles.from_xy((x + mx) % nx, (y + my) % ny, u[0], u[1], u[2], 1.0, 1.0,
                                   1.0, 1.0)
        g1 = ora.gather(nx, ny, order, fs, ps, mode="nodal")
        assert np.allclose(g1, g0, rtol=0, atol=1e-12), (mx, my)


# ---------------------------------------------------------------- push
def test_boris_quarter_turn_hand(ora):
    h = HAND["boris_quarter_turn"]
    p = ora.Particles(np.array([3]), np.array([3]), np.array([0.5]), np.array([0.5]),
                      [h["u0"][0]], [h["u0"][1]], [h["u0"][2]], 1.0, 1.0)
    e3 = np.zeros(3)
    b3 = np.array(h["B"], dtype=float)
    ora.boris(p, 1.0, e3, b3)
    assert np.allclose([p.ux[0], p.uy[0], p.uz[0]], h["u1"], rtol=0, atol=1e-15)


def test_boris_pure_b_rotation(ora):
    """Pure magnetic field: |u| is preserved and u_perp turns by 2 atan(|t|)
    per step with t = q dt B/(2 m gamma)."""
    rng = np.random.default_rng(3)
    n = 500
    u = rng.normal(size=(3, n)) * 2.0
    B = rng.normal(size=(3, n)) * 3.0
    q, m, dt = -0.7, 0.7, 0.1
    p = ora.Particles(np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n), u[0], u[1], u[2], q, m)
    ora.boris(p, dt, np.zeros((3, n)), B)
    u1 = np.vstack([p.ux, p.uy, p.uz])
    assert np.allclose(np.linalg.norm(u1, axis=0), np.linalg.norm(u, axis=0), rtol=1e-14)
    gam = np.sqrt(1 + (u * u).sum(0))
    bn = np.linalg.norm(B, axis=0)
    bh = B / bn
    angle_want = 2 * np.arctan(abs(q) * dt * bn / (2 * m * gam))
    up0 = u - (u * bh).sum(0) * bh
    up1 = u1 - (u1 * bh).sum(0) * bh
    cosang = (up0 * up1).sum(0) / (np.linalg.norm(up0, axis=0) * np.linalg.norm(up1, axis=0))
    assert np.allclose(np.arccos(np.clip(cosang, -1, 1)), angle_want, atol=1e-7)
    # the parallel component is untouched
    assert np.allclose((u1 * bh).sum(0), (u * bh).sum(0), rtol=1e-12, atol=1e-12)
    # sense of rotation: q (v x B) direction for the first small step
    cross = np.cross(up0.T, up1.T).T
    assert np.all(np.sign((cross * bh).sum(0)) == -np.sign(q))


@pytest.mark.parametrize("order", ORDERS)
def test_uniform_e_kick(ora, order):
    """Uniform E on the whole grid: after one push du = (q/m) E dt exactly."""
    nx = ny = 8
    rng = np.random.default_rng(20 + order)
    n = 64
    x = rng.uniform(0, nx, n)
    y = rng.uniform(0, ny, n)
    u = rng.normal(size=(3, n))
    q, m, dt = 1.0, 1.0, 1.0
    p = ora.Particles.from_xy(x, y, u[0], u[1], u[2], q, m, 1.0, 1.0)
    E0 = (0.3, -0.2, 0.1)
    f = [np.full((ny, nx), E0[0]), np.full((ny, nx), E0[1]), np.full((ny, nx), E0[2])] + \
        [np.zeros((ny, nx)) for _ in range(3)]
    g = ora.gather(nx, ny, order, f, p)
    ora.boris(p, dt, g[0:3], g[3:6])
    for c, arr in enumerate((p.ux, p.uy, p.uz)):
        assert np.allclose(arr - u[c], q / m * E0[c] * dt, rtol=0, atol=1e-14)


def test_move_cell_crossing(ora):
    """x^{n+1} = x^n + dt u/gamma, with the offset kept in [0, 1)."""
    rng = np.random.default_rng(5)
    n = 2000
    x = rng.uniform(2, 6, n)
    y = rng.uniform(2, 6, n)
    u = rng.normal(size=(3, n)) * 5
    p = ora.Particles.from_xy(x, y, u[0], u[1], u[2], 1.0, 1.0, 0.1, 0.2)
    dt = 0.09
    ora.move(p, dt, 0.1, 0.2)
    g = np.sqrt(1 + (u * u).sum(0))
    assert np.allclose(p.x(0.1), x + dt * u[0] / g, rtol=0, atol=1e-14)
    assert np.allclose(p.y(0.2), y + dt * u[1] / g, rtol=0, atol=1e-14)
    assert np.all((p.fx >= 0) & (p.fx < 1) & (p.fy >= 0) & (p.fy < 1))


# ---------------------------------------------------------------- deposit
def _random_moves(ora, rng, n, nx, ny, dx, dy, dt, q):
    x = rng.uniform(0, nx * dx, n)
    y = rng.uniform(0, ny * dy, n)
    u = rng.normal(size=(3, n)) * 3.0
    p = ora.Particles.from_xy(x, y, u[0], u[1], u[2], q, abs(q), dx, dy)
    old = p.copy()
    ora.move(p, dt, dx, dy)
    return old, p


@pytest.mark.parametrize("order", ORDERS)
def test_esirkepov_continuity(ora, order):
    """Discrete charge continuity (rho1 - rho0)/dt + div J = 0 to roundoff,
    including particles that cross the periodic boundary."""
    nx, ny, dx, dy = 12, 10, 0.1, 0.13
    dt = 0.9 * min(dx, dy)
    rng = np.random.default_rng(30 + order)
    old, new = _random_moves(ora, rng, 400, nx, ny, dx, dy, dt, q=-0.37)
    J = [np.zeros((ny, nx)) for _ in range(3)]
    ora.deposit(nx, ny, order, dx, dy, dt, old, new, J)
    ora.wrap(nx, ny, new)
    rho0 = ora.charge(nx, ny, order, dx, dy, old)
    rho1 = ora.charge(nx, ny, order, dx, dy, new)
    divj = ora.div_e(nx, ny, dx, dy, J[0], J[1])
    resid = (rho1 - rho0) / dt + divj
    scale = np.abs(rho0).max() / dt
    assert np.abs(resid).max() < 1e-13 * scale


@pytest.mark.parametrize("order", ORDERS)
def test_esirkepov_total_current(ora, order):
    """sum J dx dy = q dx_p/dt (x, y) and q vz (z) for every particle."""
    nx, ny, dx, dy = 10, 9, 0.2, 0.1
    dt = 0.08
    rng = np.random.default_rng(40 + order)
    for _ in range(20):
        old, new = _random_moves(ora, rng, 1, nx, ny, dx, dy, dt, q=0.8)
        J = [np.zeros((ny, nx)) for _ in range(3)]
        ora.deposit(nx, ny, order, dx, dy, dt, old, new, J)
        dxp = new.x(dx)[0] - old.x(dx)[0]
        dyp = new.y(dy)[0] - old.y(dy)[0]
        g = math.sqrt(1 + new.ux[0] ** 2 + new.uy[0] ** 2 + new.uz[0] ** 2)
        assert abs(J[0].sum() * dx * dy - 0.8 * dxp / dt) < 1e-13
        assert abs(J[1].sum() * dx * dy - 0.8 * dyp / dt) < 1e-13
        assert abs(J[2].sum() * dx * dy - 0.8 * new.uz[0] / g) < 1e-13


@pytest.mark.parametrize("order", ORDERS)
def test_esirkepov_jz_path_average(ora, order):
    """Jz dx dy/(q vz) equals the average over the straight path of the
    linearly interpolated node shapes, int_0^1 (S0x + s DSx)(S0y + s DSy) ds,
    which fixes the 1/2 and 1/3 coefficients of Wz."""
    nx = ny = 12
    rng = np.random.default_rng(50 + order)
    old, new = _random_moves(ora, rng, 1, nx, ny, 1.0, 1.0, 0.9, q=1.0)
    J = [np.zeros((ny, nx)) for _ in range(3)]
    ora.deposit(nx, ny, order, 1.0, 1.0, 0.9, old, new, J)
    g = math.sqrt(1 + new.ux[0] ** 2 + new.uy[0] ** 2 + new.uz[0] ** 2)
    vz = new.uz[0] / g
    X0, Y0 = old.ix[0] + old.fx[0], old.iy[0] + old.fy[0]
    X1, Y1 = new.ix[0] + new.fx[0], new.iy[0] + new.fy[0]
    for j in range(int(Y0) - 3, int(Y0) + 5):
        for i in range(int(X0) - 3, int(X0) + 5):
            s0x, s1x = ora.shape(order, X0 - i), ora.shape(order, X1 - i)
            s0y, s1y = ora.shape(order, Y0 - j), ora.shape(order, Y1 - j)
            ref, _ = integrate.quad(lambda s: (s0x + s * (s1x - s0x)) * (s0y + s * (s1y - s0y)), 0, 1)
            assert abs(J[2][j % ny, i % nx] - vz * ref) < 1e-13


@pytest.mark.parametrize("order", ORDERS)
def test_esirkepov_diagonal_symmetry(ora, order):
    """A particle moving along the diagonal x = y gives Jx(i+1/2, j) =
    Jy(j, i+1/2): the density decomposition treats x and y symmetrically
    (an asymmetric split such as Wx = DSx S0y, Wy = DSy S1x would also conserve
    charge but fails this)."""
    nx = ny = 12
    rng = np.random.default_rng(60 + order)
    for _ in range(10):
        a0 = rng.uniform(4, 6)
        d = rng.uniform(-0.9, 0.9)
        p0 = ora.Particles.from_xy([a0], [a0], [d], [d], [0.3], 1.0, 1.0, 1.0, 1.0)
        p1 = p0.copy()
        ora.move(p1, 1.0, 1.0, 1.0)
        J = [np.zeros((ny, nx)) for _ in range(3)]
        ora.deposit(nx, ny, order, 1.0, 1.0, 1.0, p0, p1, J)
        assert np.allclose(J[0], J[1].T, rtol=0, atol=1e-14)


def test_esirkepov_order1_hand(ora):
    h = HAND["esirkepov_order1"]
    nx = ny = 8
    old = ora.Particles.from_xy([h["x0"]], [h["y0"]], [0.0], [0.0], [0.0], 1.0, 1.0, 1.0, 1.0)
    new = ora.Particles.from_xy([h["x1"]], [h["y1"]], [0.0], [0.0], [0.0], 1.0, 1.0, 1.0, 1.0)
    J = [np.zeros((ny, nx)) for _ in range(3)]
    ora.deposit(nx, ny, 1, 1.0, 1.0, 1.0, old, new, J)
    want = np.zeros((ny, nx))
    for j, i, v in h["jx_nonzero"]:
        want[j, i] = v
    assert np.allclose(J[0], want, rtol=0, atol=1e-15)
    assert np.abs(J[1]).max() == 0.0 and np.abs(J[2]).max() == 0.0


def test_charge_order2_hand(ora):
    h = HAND["charge_order2_on_node"]
    p = ora.Particles.from_xy([h["x"]], [h["y"]], [0.0], [0.0], [0.0], 1.0, 1.0, 1.0, 1.0)
    rho = ora.charge(8, 8, 2, 1.0, 1.0, p)
    want = np.zeros((8, 8))
    for j, i, v in h["rho"]:
        want[j, i] = v
    assert np.allclose(rho, want, rtol=0, atol=1e-15)
