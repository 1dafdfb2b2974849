"""Closed-form potentials used to check the method's accuracy (not parity).

TEST INFRASTRUCTURE ONLY (see oracle/nested.py).  G is a parameter; all
functions take Cartesian coordinate arrays x, y, z relative to the origin.

* Uniform sphere and the binary of two spheres: Sect. 2 accuracy tests.
* Homogeneous ellipsoid: Sect. 2 accuracy tests (closed form of
  Chandrasekhar 1969), written here with Carlson's symmetric integrals
  R_F and R_D (Carlson 1995).
* Plummer sphere: a smooth, centrally concentrated test density.
* "Smooth polytrope" rho = rho0 (1 - r^2/R^2)^2 inside R: compact and C^1,
  used for the second-order convergence check (Sect. 7, convergence test).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import elliprd, elliprf


def _r(x, y, z, centre=(0.0, 0.0, 0.0)):
    return np.sqrt((x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2)


def uniform_sphere(x, y, z, M, R, centre=(0.0, 0.0, 0.0), G=1.0):
    """Phi of a homogeneous sphere: -GM/r outside, -GM(3R^2 - r^2)/(2R^3)
    inside."""
    r = _r(x, y, z, centre)
    inside = -G * M * (3 * R ** 2 - r ** 2) / (2 * R ** 3)
    with np.errstate(divide="ignore"):
        outside = -G * M / r
    return np.where(r < R, inside, outside)


def uniform_sphere_acceleration(x, y, z, M, R, centre=(0.0, 0.0, 0.0), G=1.0):
    """g = -grad Phi of `uniform_sphere` as (g_x, g_y, g_z): -G M d / r^3
    outside, -G M d / R^3 inside, d the offset from the centre."""
    dx, dy, dz = x - centre[0], y - centre[1], z - centre[2]
    r = _r(x, y, z, centre)
    with np.errstate(divide="ignore", invalid="ignore"):
        f = np.where(r < R, -G * M / R ** 3, -G * M / r ** 3)
    return f * dx, f * dy, f * dz


def binary_spheres(x, y, z, R=0.2, sep=0.5, rho_left=2.0, rho_right=1.0, G=1.0):
    """Phi of the binary star of Sect. 2: two homogeneous spheres of radius R
    centred at x = -sep and x = +sep, the left one twice as massive (its
    density twice the right one's)."""
    m = 4.0 / 3.0 * math.pi * R ** 3
    return (uniform_sphere(x, y, z, rho_left * m, R, (-sep, 0.0, 0.0), G)
            + uniform_sphere(x, y, z, rho_right * m, R, (sep, 0.0, 0.0), G))


def binary_spheres_acceleration(x, y, z, R=0.2, sep=0.5, rho_left=2.0, rho_right=1.0, G=1.0):
    """g of `binary_spheres` as (g_x, g_y, g_z)."""
    m = 4.0 / 3.0 * math.pi * R ** 3
    a = uniform_sphere_acceleration(x, y, z, rho_left * m, R, (-sep, 0.0, 0.0), G)
    b = uniform_sphere_acceleration(x, y, z, rho_right * m, R, (sep, 0.0, 0.0), G)
    return tuple(u + v for u, v in zip(a, b))


def binary_spheres_density(x, y, z, R=0.2, sep=0.5, rho_left=2.0, rho_right=1.0):
    """The binary's density sampled at the points (cell centres)."""
    return (rho_left * ((x + sep) ** 2 + y ** 2 + z ** 2 <= R * R)
            + rho_right * ((x - sep) ** 2 + y ** 2 + z ** 2 <= R * R)).astype(float)


def plummer(x, y, z, M, a, centre=(0.0, 0.0, 0.0), G=1.0):
    """Phi of a Plummer sphere: -GM / sqrt(r^2 + a^2)."""
    r = _r(x, y, z, centre)
    return -G * M / np.sqrt(r ** 2 + a ** 2)


def plummer_density(x, y, z, M, a, centre=(0.0, 0.0, 0.0)):
    r = _r(x, y, z, centre)
    return 3 * M / (4 * math.pi * a ** 3) * (1 + r ** 2 / a ** 2) ** (-2.5)


def polytrope2_mass(rho0, R):
    """Total mass of rho0 (1 - r^2/R^2)^2 inside R: 32 pi rho0 R^3 / 105."""
    return 32.0 * math.pi * rho0 * R ** 3 / 105.0


def polytrope2(x, y, z, rho0, R, centre=(0.0, 0.0, 0.0), G=1.0):
    """Phi of rho0 (1 - r^2/R^2)^2 (zero outside R).

    Spherical symmetry: Phi(r) = -G [M(<r)/r + 4 pi int_r^R rho r' dr'] with
    M(<r) = 4 pi rho0 (r^3/3 - 2 r^5/(5 R^2) + r^7/(7 R^4)) and
    int_r^R rho r' dr' = rho0 (R^2/6 - r^2/2 + r^4/(2R^2) - r^6/(6R^4))."""
    r = _r(x, y, z, centre)
    M = polytrope2_mass(rho0, R)
    rc = np.minimum(r, R)
    Min = 4 * math.pi * rho0 * (rc ** 3 / 3 - 2 * rc ** 5 / (5 * R ** 2) + rc ** 7 / (7 * R ** 4))
    tail = rho0 * (R ** 2 / 6 - rc ** 2 / 2 + rc ** 4 / (2 * R ** 2) - rc ** 6 / (6 * R ** 4))
    with np.errstate(divide="ignore", invalid="ignore"):
        inner = -G * (np.where(rc > 0, Min / np.where(rc > 0, rc, 1.0), 0.0) + 4 * math.pi * tail)
        outer = -G * M / r
    return np.where(r < R, inner, outer)


def polytrope2_density(x, y, z, rho0, R, centre=(0.0, 0.0, 0.0)):
    r = _r(x, y, z, centre)
    return np.where(r < R, rho0 * (1 - (r / R) ** 2) ** 2, 0.0)


def _ellipsoid_lambda(x, y, z, a):
    """Largest root lambda >= 0 of sum x_i^2 / (a_i^2 + lambda) = 1 (0 inside)."""
    x2, y2, z2 = x * x, y * y, z * z
    a2 = [a[0] ** 2, a[1] ** 2, a[2] ** 2]
    q = x2 / a2[0] + y2 / a2[1] + z2 / a2[2]
    lam = np.zeros_like(q)
    out = q > 1.0
    if not np.any(out):
        return lam
    xs, ys, zs = x2[out], y2[out], z2[out]
    lo = np.zeros_like(xs)
    hi = np.maximum(xs + ys + zs, 1e-300)  # sum at hi is <= 1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        f = xs / (a2[0] + mid) + ys / (a2[1] + mid) + zs / (a2[2] + mid)
        gt = f > 1.0
        lo = np.where(gt, mid, lo)
        hi = np.where(gt, hi, mid)
    lam[out] = 0.5 * (lo + hi)
    return lam


def ellipsoid(x, y, z, a, rho=1.0, centre=(0.0, 0.0, 0.0), G=1.0):
    """Phi of a homogeneous ellipsoid with semi-axes a = (a1, a2, a3) along
    (x, y, z):

    Phi = -pi G rho a1 a2 a3 * int_lam^inf (1 - sum x_i^2/(a_i^2+u)) du / Delta(u)
    with Delta(u) = sqrt(prod (a_i^2 + u)); lam = 0 inside.  In Carlson form,
    int du/Delta = 2 R_F and int du/((a_i^2+u) Delta) = (2/3) R_D(.., a_i^2+lam)."""
    x = np.asarray(x, dtype=np.float64) - centre[0]
    y = np.asarray(y, dtype=np.float64) - centre[1]
    z = np.asarray(z, dtype=np.float64) - centre[2]
    x, y, z = np.broadcast_arrays(x, y, z)
    lam = _ellipsoid_lambda(x, y, z, a)
    A = [a[0] ** 2 + lam, a[1] ** 2 + lam, a[2] ** 2 + lam]
    I = 2.0 * elliprf(A[0], A[1], A[2])
    Ax = (2.0 / 3.0) * elliprd(A[1], A[2], A[0])
    Ay = (2.0 / 3.0) * elliprd(A[2], A[0], A[1])
    Az = (2.0 / 3.0) * elliprd(A[0], A[1], A[2])
    return -math.pi * G * rho * a[0] * a[1] * a[2] * (I - x * x * Ax - y * y * Ay - z * z * Az)


def ellipsoid_acceleration(x, y, z, a, rho=1.0, centre=(0.0, 0.0, 0.0), G=1.0):
    """g = -grad Phi of the homogeneous ellipsoid of `ellipsoid`, as
    (g_x, g_y, g_z).  Differentiating under the integral, the term from the
    lower limit lam(x) vanishes (its integrand is zero on the confocal
    surface), so g_i = -2 pi G rho a1 a2 a3 x_i (2/3) R_D(a_j^2+lam,
    a_k^2+lam, a_i^2+lam)."""
    x = np.asarray(x, dtype=np.float64) - centre[0]
    y = np.asarray(y, dtype=np.float64) - centre[1]
    z = np.asarray(z, dtype=np.float64) - centre[2]
    x, y, z = np.broadcast_arrays(x, y, z)
    lam = _ellipsoid_lambda(x, y, z, a)
    A = [a[0] ** 2 + lam, a[1] ** 2 + lam, a[2] ** 2 + lam]
    Ax = (2.0 / 3.0) * elliprd(A[1], A[2], A[0])
    Ay = (2.0 / 3.0) * elliprd(A[2], A[0], A[1])
    Az = (2.0 / 3.0) * elliprd(A[0], A[1], A[2])
    k = -2.0 * math.pi * G * rho * a[0] * a[1] * a[2]
    return k * x * Ax, k * y * Ay, k * z * Az


def ellipsoid_index_sum(a):
    """Sum of the dimensionless interior coefficients a1 a2 a3 int du /((a_i^2+u) Delta)
    over i; equals 2 for any ellipsoid (a classical identity)."""
    A = [a[0] ** 2, a[1] ** 2, a[2] ** 2]
    s = (elliprd(A[1], A[2], A[0]) + elliprd(A[2], A[0], A[1]) + elliprd(A[0], A[1], A[2]))
    return a[0] * a[1] * a[2] * (2.0 / 3.0) * s


def relative_error(num, ana):
    """err_Phi of Sect. 2: |(Phi_num - Phi_an) / Phi_an|."""
    return np.abs((num - ana) / ana)
