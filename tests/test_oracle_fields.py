"""Pins of the oracle's implicit field solver (RHS of Eq. (7), CG, update of
Eqs. (5)-(6)) against closed forms; CPU only."""
import json
import os

import numpy as np
import pytest

from oracle import spectral

HAND = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")))


def _curl_e_of(ora, nx, ny, dx, dy, az):
    """A divergence-free B from a potential Az at E_z points: Bx = dAz/dy,
    By = -dAz/dx with forward differences (discrete div of it vanishes)."""
    bx = (np.roll(az, -1, axis=0) - az) / dy
    by = -(np.roll(az, -1, axis=1) - az) / dx
    return bx, by


def _curl_e(nx, ny, dx, dy, e):
    cx = (np.roll(e[2], -1, 0) - e[2]) / dy
    cy = -(np.roll(e[2], -1, 1) - e[2]) / dx
    cz = (np.roll(e[1], -1, 1) - e[1]) / dx - (np.roll(e[0], -1, 0) - e[0]) / dy
    return [cx, cy, cz]


def _curl_b(nx, ny, dx, dy, b):
    cx = (b[2] - np.roll(b[2], 1, 0)) / dy
    cy = -(b[2] - np.roll(b[2], 1, 1)) / dx
    cz = (b[1] - np.roll(b[1], 1, 1)) / dx - (b[0] - np.roll(b[0], 1, 0)) / dy
    return [cx, cy, cz]


@pytest.mark.parametrize("sigma,theta", [(0.5, 0.5), (1.0, 0.6), (0.8, 1.0)])
def test_cg_matches_fft_solve(ora, sigma, theta):
    nx, ny, dx, dy = 24, 16, 0.1, 0.07
    dt = sigma * min(dx, dy)
    b = np.random.default_rng(1).normal(size=(ny, nx))
    x, it, rel = ora.cg(nx, ny, dx, dy, dt, theta, b, rtol=1e-13, maxit=500)
    ref = spectral.fft_solve(b, dx, dy, dt, theta)
    assert rel <= 1e-13
    assert np.abs(x - ref).max() <= 1e-12 * np.abs(ref).max()
    # the operator itself against the Fourier symbol
    ax = ora.apply_A(nx, ny, dx, dy, dt, theta, ref)
    assert np.abs(ax - b).max() <= 1e-12 * np.abs(b).max()


def test_cg_zero_rhs_and_maxit(ora):
    nx = ny = 8
    x, it, rel = ora.cg(nx, ny, 1.0, 1.0, 1.0, 0.6, np.zeros((ny, nx)))
    assert it == 0 and rel == 0.0 and np.all(x == 0)
    b = np.random.default_rng(2).normal(size=(ny, nx))
    x, it, rel = ora.cg(nx, ny, 1.0, 1.0, 1.0, 0.6, b, rtol=1e-14, maxit=2)
    assert it == 2 and rel > 1e-6


def _random_state(rng, nx, ny, dx, dy):
    E = [rng.normal(size=(ny, nx)) for _ in range(3)]
    bx, by = _curl_e_of(None, nx, ny, dx, dy, rng.normal(size=(ny, nx)))
    B = [bx, by, rng.normal(size=(ny, nx))]
    J = [rng.normal(size=(ny, nx)) for _ in range(3)]
    return E, B, J


@pytest.mark.parametrize("theta", [0.5, 0.6, 1.0])
def test_solve_satisfies_eqs_5_6(ora, theta):
    """Eq. (7) solved by CG, then the update, reproduce the original
    theta-weighted Maxwell discretisation Eqs. (5)-(6) for a divergence-free
    B^n, with 4 pi and c = 1, to the CG tolerance."""
    nx, ny, dx, dy = 20, 14, 0.1, 0.1
    dt = 1.0 * dx
    rng = np.random.default_rng(7)
    E, B, J = _random_state(rng, nx, ny, dx, dy)
    E0 = [a.copy() for a in E]
    B0 = [a.copy() for a in B]
    b = ora.rhs(nx, ny, dx, dy, dt, theta, E, B, J)
    db = [ora.cg(nx, ny, dx, dy, dt, theta, b[c], rtol=1e-14, maxit=500)[0] for c in range(3)]
    ora.update(nx, ny, dx, dy, dt, theta, E, B, db, J)
    # Eq. (5): (B1 - B0)/dt = -curl_E(theta E1 + (1 - theta) E0)
    mix_e = [theta * E[c] + (1 - theta) * E0[c] for c in range(3)]
    ce = _curl_e(nx, ny, dx, dy, mix_e)
    for c in range(3):
        lhs = (B[c] - B0[c]) / dt
        assert np.abs(lhs + ce[c]).max() <= 1e-10 * np.abs(ce[c]).max()
    # Eq. (6): (E1 - E0)/dt = curl_B(theta B1 + (1 - theta) B0) - 4 pi J
    mix_b = [theta * B[c] + (1 - theta) * B0[c] for c in range(3)]
    cb = _curl_b(nx, ny, dx, dy, mix_b)
    for c in range(3):
        lhs = (E[c] - E0[c]) / dt
        rhs = cb[c] - 4 * np.pi * J[c]
        assert np.abs(lhs - rhs).max() <= 1e-11 * np.abs(rhs).max()
    # div B stays zero
    assert np.abs(ora.div_b(nx, ny, dx, dy, B[0], B[1])).max() < 1e-9


@pytest.mark.parametrize("sigma", [0.5, 0.7, 1.0])
@pytest.mark.parametrize("theta", [0.5, 0.6, 1.0])
@pytest.mark.parametrize("kind", ["TE", "TM"])
def test_vacuum_mode_amplification_eq10(ora, sigma, theta, kind):
    """A single vacuum Fourier mode evolves with amplification factors equal to
    the roots of Eq. (10): the eigenvalues of the solver's one-step map on
    that mode are z = (1 +- 2iS(1-theta))/(1 -+ 2iS theta)."""
    nx, ny, dx, dy = 16, 12, 0.1, 0.1
    dt = sigma * dx
    k = (2 * np.pi * 3 / (nx * dx), 2 * np.pi * 2 / (ny * dy))
    Sx, Sy = spectral.S_param(k[0] * dx, k[1] * dy, dt / dx, dt / dy)
    S = np.hypot(Sx, Sy)
    # Build the one-step map on span{Re, Im} of the mode for the evolving
    # pair (TE: Bz and the E it induces; project everything onto exp(i k.x)).
    jj, ii = np.mgrid[0:ny, 0:nx]
    J0 = [np.zeros((ny, nx)) for _ in range(3)]
    if kind == "TE":
        pos = {"E0": (0.5, 0.0), "E1": (0.0, 0.5), "B2": (0.5, 0.5)}
        comps = [("E", 0), ("E", 1), ("B", 2)]
    else:
        pos = {"E2": (0.0, 0.0), "B0": (0.0, 0.5), "B1": (0.5, 0.0)}
        comps = [("E", 2), ("B", 0), ("B", 1)]

    def phase(name):
        sx, sy = pos[name]
        return np.exp(1j * (k[0] * (ii + sx) * dx + k[1] * (jj + sy) * dy))

    names = [f"{f}{c}" for f, c in comps]

    def project(E, B):
        v = []
        for f, c in comps:
            arr = (E if f == "E" else B)[c]
            v.append(np.sum(arr * np.conj(phase(f"{f}{c}"))) / (nx * ny))
        return np.array(v)

    # one-step map on complex amplitudes (the real fields carry +k and -k;
    # projecting onto +k isolates it because the scheme is real and linear)
    M = np.zeros((3, 3), dtype=complex)
    for col in range(3):
        E = [np.zeros((ny, nx)) for _ in range(3)]
        B = [np.zeros((ny, nx)) for _ in range(3)]
        f, c = comps[col]
        (E if f == "E" else B)[c][...] = np.real(phase(names[col]))
        b = ora.rhs(nx, ny, dx, dy, dt, theta, E, B, J0)
        db = [ora.cg(nx, ny, dx, dy, dt, theta, b[cc], rtol=1e-14, maxit=500)[0] for cc in range(3)]
        ora.update(nx, ny, dx, dy, dt, theta, E, B, db, J0)
        M[:, col] = 2.0 * project(E, B)
    ev = np.linalg.eigvals(M)
    zp, zm = spectral.z_roots(S, theta)
    # one eigenvalue is the static (curl-free / divergence) mode, eigenvalue 1
    # for TE (longitudinal E) and for TM (B with nonzero divergence); the
    # other two are the electromagnetic roots of Eq. (10)
    ev = sorted(ev, key=lambda z: abs(z - 1.0))
    em = sorted(ev[1:], key=lambda z: z.imag)
    want = sorted([zp, zm], key=lambda z: z.imag)
    assert abs(ev[0] - 1.0) < 1e-9 or kind == "TM"
    for a, b in zip(em, want):
        assert abs(a - b) < 1e-10, (em, want)


def test_vacuum_mode_hand_8x8(ora):
    """App.-style hand case: k = (2 pi/8, 0) on 8x8, theta = 0.6, sigma = 1,
    a travelling TE mode shrinks by |z| and turns by arg z per step."""
    h = HAND["vacuum_mode"]
    nx = ny = 8
    dx = dy = dt = 1.0
    theta = h["theta"]
    ii = np.arange(nx)
    k = 2 * np.pi / 8
    S = h["S"]
    zp, _ = spectral.z_roots(S, theta)
    # eigenvector of the TE pair (Ey at i, Bz at i+1/2) for root zp:
    # Bz amplitude 1, Ey amplitude from Eq. (5): (z-1) Bz = -dt(theta z + 1 - theta) (dEy/dx)
    dfac = (np.exp(1j * k) - 1.0) * np.exp(-1j * k / 2) / dx   # d/dx on the staggered pair
    ey_amp = -(zp - 1.0) / (dt * (theta * zp + 1 - theta) * dfac)
    E = [np.zeros((ny, nx)) for _ in range(3)]
    B = [np.zeros((ny, nx)) for _ in range(3)]
    bz0 = np.exp(1j * k * (ii + 0.5))
    ey0 = ey_amp * np.exp(1j * k * ii)
    E[1][...] = np.real(ey0)[None, :]
    B[2][...] = np.real(bz0)[None, :]
    J0 = [np.zeros((ny, nx)) for _ in range(3)]
    for n in range(1, 6):
        b = ora.rhs(nx, ny, dx, dy, dt, theta, E, B, J0)
        db = [ora.cg(nx, ny, dx, dy, dt, theta, b[c], rtol=1e-15, maxit=500)[0] for c in range(3)]
        ora.update(nx, ny, dx, dy, dt, theta, E, B, db, J0)
        want = np.real(zp ** n * bz0)
        assert np.abs(B[2][0] - want).max() < 1e-12
    assert abs(abs(zp) - h["abs_z"]) < 1e-15 and abs(np.angle(zp) - h["arg_z"]) < 1e-15


def test_crank_nicolson_energy_invariant(ora):
    """theta = 1/2 in vacuum: |z| = 1 for every mode, so sum(E^2 + B^2) is
    conserved; theta > 1/2 makes it decay monotonically (Sec. 2)."""
    nx, ny, dx, dy = 16, 16, 0.1, 0.1
    dt = dx
    rng = np.random.default_rng(11)
    for theta, expect in ((0.5, "const"), (0.6, "decay")):
        E, B, _ = _random_state(rng, nx, ny, dx, dy)
        J0 = [np.zeros((ny, nx)) for _ in range(3)]
        energy = [sum(float((a * a).sum()) for a in E + B)]
        for _ in range(10):
            b = ora.rhs(nx, ny, dx, dy, dt, theta, E, B, J0)
            db = [ora.cg(nx, ny, dx, dy, dt, theta, b[c], rtol=1e-14, maxit=500)[0] for c in range(3)]
            ora.update(nx, ny, dx, dy, dt, theta, E, B, db, J0)
            energy.append(sum(float((a * a).sum()) for a in E + B))
        energy = np.array(energy)
        if expect == "const":
            assert np.abs(energy / energy[0] - 1).max() < 1e-11
        else:
            assert np.all(np.diff(energy) < 0)


def test_dispersion_closed_forms():
    """Exact roots satisfy Eq. (10); at theta = 1/2 they reduce to Eq. (15) and
    the printed Eqs. (11)-(12) agree with them; for theta > 1/2 the printed
    forms differ from the exact root (a reading recorded in the design notes)."""
    for theta in (0.5, 0.501, 0.6, 1.0):
        for S in (0.1, 0.5, 1.0, 1.4142):
            zp, zm = spectral.z_roots(S, theta)
            assert abs(spectral.eq10_residual(zp, S, theta)) < 1e-13
            assert abs(spectral.eq10_residual(zm, S, theta)) < 1e-13
            assert abs(zp) <= 1.0 + 1e-15
    for S in (0.1, 0.5, 1.0, 1.4):
        re, im = spectral.omega_exact(S, 0.5)
        assert abs(re - spectral.omega_cn(S)) < 1e-14 and abs(im) < 1e-15
        pre, pim = spectral.omega_printed(S, 0.5)
        assert abs(pre - re) < 1e-14 and abs(pim) < 1e-15
    re, im = spectral.omega_exact(1.0, 0.6)
    assert abs(re - 1.550799) < 1e-6 and abs(im - 0.198651) < 1e-6
    pre, pim = spectral.omega_printed(1.0, 0.6)
    assert abs(pim - 0.379977) < 1e-6


def test_cherenkov_locus_on_cn_surface():
    """Eq. (17) points lie on both omega = V kx and the Eq. (15) surface."""
    sigma, V = 0.5, 0.9999
    kx = np.linspace(0.05, np.pi, 200)
    ky = spectral.cherenkov_ky(kx, V, sigma, sigma)
    ok = np.isfinite(ky)
    assert ok.sum() > 10
    S = np.hypot(*spectral.S_param(kx[ok], ky[ok], sigma, sigma))
    assert np.allclose(spectral.omega_cn(S), V * sigma * kx[ok], atol=1e-12)


# ---------------------------------------------------------------- explicit FDTD (Eqs. (3)-(4))
def _mode_map(ora, nx, ny, dx, dy, k, kind, step):
    """3x3 one-step map of a scheme on the complex amplitudes of one Fourier
    mode of the TE (Ex, Ey, Bz) or TM (Ez, Bx, By) triple, each component
    projected at its own staggered points."""
    jj, ii = np.mgrid[0:ny, 0:nx]
    if kind == "TE":
        comps = [("E", 0, (0.5, 0.0)), ("E", 1, (0.0, 0.5)), ("B", 2, (0.5, 0.5))]
    else:
        comps = [("E", 2, (0.0, 0.0)), ("B", 0, (0.0, 0.5)), ("B", 1, (0.5, 0.0))]

    def phase(s):
        return np.exp(1j * (k[0] * (ii + s[0]) * dx + k[1] * (jj + s[1]) * dy))

    M = np.zeros((3, 3), dtype=complex)
    for col, (f, c, s) in enumerate(comps):
        E = [np.zeros((ny, nx)) for _ in range(3)]
        B = [np.zeros((ny, nx)) for _ in range(3)]
        (E if f == "E" else B)[c][...] = np.real(phase(s))
        step(E, B)
        for row, (f2, c2, s2) in enumerate(comps):
            arr = (E if f2 == "E" else B)[c2]
            M[row, col] = 2.0 * np.sum(arr * np.conj(phase(s2))) / (nx * ny)
    return M


@pytest.mark.parametrize("sigma", [0.3, 0.5, 0.7])
@pytest.mark.parametrize("kind", ["TE", "TM"])
def test_explicit_vacuum_mode_eq16(ora, sigma, kind):
    """The explicit FDTD advance moves a vacuum Fourier mode by the roots of
    Eq. (16): the one-step map on the mode has eigenvalues
    z = 1 - 2S^2 +- 2S sqrt(S^2 - 1) (|z| = 1 below the Courant limit) and 1
    (the static mode)."""
    nx, ny, dx, dy = 16, 12, 0.1, 0.1
    dt = sigma * dx
    k = (2 * np.pi * 3 / (nx * dx), 2 * np.pi * 2 / (ny * dy))
    S = np.hypot(*spectral.S_param(k[0] * dx, k[1] * dy, dt / dx, dt / dy))
    J0 = [np.zeros((ny, nx)) for _ in range(3)]
    M = _mode_map(ora, nx, ny, dx, dy, k, kind,
                  lambda E, B: ora.update_explicit(nx, ny, dx, dy, dt, E, B, J0))
    ev = sorted(np.linalg.eigvals(M), key=lambda z: abs(z - 1.0))
    em = sorted(ev[1:], key=lambda z: z.imag)
    want = sorted(spectral.z_explicit(S), key=lambda z: z.imag)
    assert abs(ev[0] - 1.0) < 1e-9
    for a, b in zip(em, want):
        assert abs(a - b) < 1e-10, (em, want)
    assert abs(abs(want[0]) - 1.0) < 1e-14
    # the phase of the root is Eq. (16)'s omega dt
    assert abs(abs(np.angle(want[1])) - spectral.omega_explicit(S)) < 1e-12


def test_explicit_courant_instability(ora):
    """Beyond the Courant limit (sigma = 0.8 > 1/sqrt(2) at dx = dy) a short
    mode (k dx = k dy = 5 pi/6, S = 0.8 sqrt(2) sin(5 pi/12) > 1) grows by the
    real root of Eq. (16) with |z| > 1 per step."""
    nx = ny = 12
    dx = dy = 0.1
    dt = 0.8 * dx
    k = (5 * np.pi / 6 / dx, 5 * np.pi / 6 / dy)
    S = np.hypot(*spectral.S_param(5 * np.pi / 6, 5 * np.pi / 6, 0.8, 0.8))
    assert S > 1.0
    J0 = [np.zeros((ny, nx)) for _ in range(3)]
    M = _mode_map(ora, nx, ny, dx, dy, k, "TM",
                  lambda E, B: ora.update_explicit(nx, ny, dx, dy, dt, E, B, J0))
    ev = np.linalg.eigvals(M)
    zp, zm = spectral.z_explicit(S)
    assert abs(zm.imag) < 1e-15 and abs(zm.real) > 1.0
    assert min(abs(ev - zm)) < 1e-9 and min(abs(ev - zp)) < 1e-9


def test_explicit_is_the_yee_leapfrog(ora):
    """Two explicit steps from (E^0, B^0) with currents J^{1/2}, J^{3/2}
    reproduce the leapfrog of Eqs. (3)-(4) written out here with B at half
    steps (B^{1/2} = B^0 - dt/2 curl E^0): E^1, E^2 agree, and the carried
    B^1 is the mean of B^{1/2} and B^{3/2}."""
    nx, ny, dx, dy = 20, 14, 0.1, 0.08
    dt = 0.5 * dx
    rng = np.random.default_rng(17)
    E, B, J0 = _random_state(rng, nx, ny, dx, dy)
    J1 = [rng.normal(size=(ny, nx)) for _ in range(3)]
    Eh = [a.copy() for a in E]
    bh0 = [b - 0.5 * dt * c for b, c in zip(B, _curl_e(nx, ny, dx, dy, Eh))]
    e1 = [e + dt * c - 4 * np.pi * dt * j for e, c, j in zip(Eh, _curl_b(nx, ny, dx, dy, bh0), J0)]
    bh1 = [b - dt * c for b, c in zip(bh0, _curl_e(nx, ny, dx, dy, e1))]
    e2 = [e + dt * c - 4 * np.pi * dt * j for e, c, j in zip(e1, _curl_b(nx, ny, dx, dy, bh1), J1)]
    ora.update_explicit(nx, ny, dx, dy, dt, E, B, J0)
    for c in range(3):
        assert np.abs(E[c] - e1[c]).max() <= 1e-12 * np.abs(e1[c]).max()
        assert np.abs(B[c] - 0.5 * (bh0[c] + bh1[c])).max() <= 1e-12 * np.abs(bh1[c]).max()
    ora.update_explicit(nx, ny, dx, dy, dt, E, B, J1)
    for c in range(3):
        assert np.abs(E[c] - e2[c]).max() <= 1e-12 * np.abs(e2[c]).max()


def test_explicit_vacuum_energy_invariant(ora):
    """In vacuum the Yee leapfrog conserves sum(E^n . E^n + B^{n-1/2} . B^{n+1/2})
    below the Courant limit, with B^{n -/+ 1/2} = B^n +/- dt/2 curl E^n."""
    nx, ny, dx, dy = 16, 16, 0.1, 0.1
    dt = 0.6 * dx
    rng = np.random.default_rng(5)
    E, B, _ = _random_state(rng, nx, ny, dx, dy)
    J0 = [np.zeros((ny, nx)) for _ in range(3)]

    def invariant():
        ce = _curl_e(nx, ny, dx, dy, E)
        bm = [b + 0.5 * dt * c for b, c in zip(B, ce)]
        bp = [b - 0.5 * dt * c for b, c in zip(B, ce)]
        return sum(float((e * e).sum()) for e in E) + sum(float((a * b).sum())
                                                          for a, b in zip(bm, bp))
    w0 = invariant()
    for _ in range(25):
        ora.update_explicit(nx, ny, dx, dy, dt, E, B, J0)
        assert abs(invariant() / w0 - 1) < 1e-12


def test_power_spectrum_pins():
    """The k-space power of the oracle: Parseval (the total power is the mean
    square of the field), a single real mode puts a quarter of its squared
    amplitude on each of +k and -k, and a staggered copy of the field (a
    half-cell shift, as between Yee components) has the same power."""
    nx, ny = 40, 24
    rng = np.random.default_rng(3)
    f = rng.normal(size=(ny, nx))
    p = spectral.power_spectrum(f)
    assert abs(p.sum() - (f * f).mean()) < 1e-14 * (f * f).mean()
    J, I = np.mgrid[0:ny, 0:nx]
    m = 2.5 * np.cos(2 * np.pi * (3 * I / nx + 5 * J / ny) + 0.3)
    pm = spectral.power_spectrum(m)
    assert abs(pm[5, 3] - 2.5 ** 2 / 4) < 1e-13 and abs(pm[ny - 5, nx - 3] - 2.5 ** 2 / 4) < 1e-13
    assert pm.sum() - pm[5, 3] - pm[ny - 5, nx - 3] < 1e-20
    shifted = 2.5 * np.cos(2 * np.pi * (3 * (I + 0.5) / nx + 5 * J / ny) + 0.3)
    assert np.allclose(spectral.power_spectrum(shifted), pm, rtol=0, atol=1e-13)
