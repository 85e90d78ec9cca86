"""Closed forms of the paper's field solver on periodic grids (numpy).

TEST INFRASTRUCTURE ONLY (oracle side; never imported by the GPU package).

* fft_solve: the exact solution of Eq. (7) on a periodic grid. The 5-point
  Laplacian is diagonal in Fourier space with eigenvalue
  -4 (sin^2(kx dx/2)/dx^2 + sin^2(ky dy/2)/dy^2), so
  A = 1 - (theta c dt)^2 L has eigenvalue
  1 + 4 (theta c dt)^2 (sin^2(kx dx/2)/dx^2 + sin^2(ky dy/2)/dy^2).
* dispersion: the vacuum dispersion relation of the implicit scheme, Eq. (10),
  solved exactly. With z = exp(i omega dt) and S^2 = Sx^2 + Sy^2
  (Sx, Sy of Eqs. (13)-(14)), Eq. (10) reads ((z-1)/(theta(z-1)+1))^2 = -4 S^2,
  so (z-1) = +-2iS (theta(z-1)+1) and
      z = (1 +- 2iS(1-theta)) / (1 -+ 2iS theta).
  |z| <= 1 for theta >= 1/2, equality only at theta = 1/2, matching the
  paper's statement that the scheme damps unless theta = 1/2 (Sec. 2). The
  per-step amplification of a vacuum eigenmode is therefore z.
  Re(omega dt) = arg z, Im(omega dt) = -ln|z| (positive means damping in the
  paper's convention).
* the forms printed as Eqs. (11)-(12), kept for comparison: they agree with
  the exact root only at theta = 1/2, where both reduce to Eq. (15).
* Eq. (15) (theta = 1/2), Eq. (16) (explicit FDTD) and Eq. (17) (Cherenkov
  resonance locus).
"""
import numpy as np


def helmholtz_symbol(nx, ny, dx, dy, dt, theta):
    kx = 2.0 * np.pi * np.fft.fftfreq(nx)       # k dx
    ky = 2.0 * np.pi * np.fft.fftfreq(ny)
    sx = np.sin(kx / 2.0) ** 2 / dx ** 2
    sy = np.sin(ky / 2.0) ** 2 / dy ** 2
    return 1.0 + 4.0 * (theta * dt) ** 2 * (sy[:, None] + sx[None, :])


def fft_solve(b, dx, dy, dt, theta):
    """Exact periodic solution of (1 - (theta dt)^2 L) x = b, Eq. (7)."""
    ny, nx = b.shape
    lam = helmholtz_symbol(nx, ny, dx, dy, dt, theta)
    return np.real(np.fft.ifft2(np.fft.fft2(b) / lam))


def S_param(kx_dx, ky_dy, sigma_x, sigma_y):
    """Sx, Sy of Eqs. (13)-(14): c dt/dx sin(kx dx/2), c dt/dy sin(ky dy/2)."""
    return sigma_x * np.sin(kx_dx / 2.0), sigma_y * np.sin(ky_dy / 2.0)


def z_roots(S, theta):
    """Both roots z = exp(i omega dt) of Eq. (10) for S = sqrt(Sx^2 + Sy^2)."""
    S = np.asarray(S, dtype=np.complex128)
    zp = (1.0 + 2j * S * (1.0 - theta)) / (1.0 - 2j * S * theta)
    zm = (1.0 - 2j * S * (1.0 - theta)) / (1.0 + 2j * S * theta)
    return zp, zm


def eq10_residual(z, S, theta):
    return ((z - 1.0) / (theta * (z - 1.0) + 1.0)) ** 2 + 4.0 * S * S


def omega_exact(S, theta):
    """(Re omega dt, Im omega dt) of the exact root with Re > 0."""
    zp, _ = z_roots(S, theta)
    return np.angle(zp), -np.log(np.abs(zp))


def omega_printed(S, theta):
    """Eqs. (11)-(12) exactly as printed (exact only at theta = 1/2)."""
    S = np.asarray(S, dtype=np.float64)
    inv = 1.0 / (S * S)
    den = (theta - 0.5) ** 2 + 0.25 * inv
    re = 2.0 * np.arctan(0.25 * np.sqrt(inv) / den)
    im = 2.0 * np.arctan(0.5 * (theta - 0.5) / den)
    return re, im


def omega_cn(S):
    """Eq. (15): tan^2(omega dt/2) = S^2 at theta = 1/2."""
    return 2.0 * np.arctan(S)


def omega_explicit(S):
    """Eq. (16): sin^2(omega dt/2) = S^2 for explicit FDTD (|S| <= 1)."""
    return 2.0 * np.arcsin(S)


def z_explicit(S):
    """Both amplification factors z = exp(i omega dt) of Eq. (16):
    sin^2(omega dt/2) = S^2 gives z + 1/z = 2 - 4 S^2, so
    z = 1 - 2 S^2 +- 2 S sqrt(S^2 - 1) (complex, |z| = 1, for S <= 1; real
    with |z| > 1 for S > 1, the Courant instability)."""
    S = np.asarray(S, dtype=np.complex128)
    r = 2.0 * S * np.sqrt(S * S - 1.0)
    return 1.0 - 2.0 * S * S + r, 1.0 - 2.0 * S * S - r


def power_spectrum(f):
    """|F(kx, ky)|^2 / (nx ny)^2 of a [ny][nx] field, F the discrete Fourier
    transform sum f(i, j) exp(-2 pi i (kx i/nx + ky j/ny)) (numpy's FFT), in
    the transform's index order: the k-space maps of Sec. 3.1 (Fig. 3)."""
    ny, nx = f.shape
    F = np.fft.fft2(np.asarray(f, dtype=np.float64))
    return (np.abs(F) / (nx * ny)) ** 2


def cherenkov_ky(kx_dx, V, sigma_x, sigma_y):
    """Eq. (17): ky dy where omega = V kx meets Eq. (15); NaN where none."""
    # omega dt = V kx dt = V sigma_x (kx dx) with c = 1
    wdt = V * sigma_x * kx_dx
    Sx = sigma_x * np.sin(kx_dx / 2.0)
    arg = np.tan(wdt / 2.0) ** 2 - Sx ** 2
    with np.errstate(invalid="ignore"):
        inner = np.sqrt(arg) / sigma_y
        return 2.0 * np.arcsin(inner)
