"""Closed-form solutions used to pin the oracle (test-side mathematics only).

Lattice units, c_s^2 = 1/3, nu = (tau - 1/2)/3 (Sec. 2).  Channel geometry:
solid rows y = 0 and y = ny-1 with halfway bounce-back, so the hydrodynamic
walls sit at y = 1/2 and y = ny - 3/2 and the width is W = ny - 2.
"""
import numpy as np
from scipy.integrate import quad


def nu_of_tau(tau):
    return (tau - 0.5) / 3.0


def poiseuille_exact(ny, tau, g):
    """Exact steady solution of D2Q9 BGK with the velocity-shift body force and
    halfway bounce-back, for the reported velocity u = j/rho + g/2 at rows
    y = 1..ny-2 (He, Zou, Luo & Dembo, J. Stat. Phys. 87 (1997): the parabola
    plus a tau-dependent slip g (16 (tau-1/2)^2 - 3) / (24 nu))."""
    nu = nu_of_tau(tau)
    y = np.arange(1, ny - 1, dtype=np.float64)
    return g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y) + g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)


def poiseuille_startup(ny, tau, g, t, nmodes=400):
    """Start-up of channel flow from rest: the steady profile minus the
    Fourier series of odd sine modes decaying as exp(-m^2 pi^2 nu t / W^2)."""
    nu = nu_of_tau(tau)
    W = ny - 2
    y = np.arange(1, ny - 1, dtype=np.float64)
    eta = (y - 0.5) / W
    us = poiseuille_exact(ny, tau, g)
    s = np.zeros_like(us)
    for m in range(1, 2 * nmodes, 2):
        s += 4 * g * W * W / (nu * np.pi ** 3 * m ** 3) * np.sin(m * np.pi * eta) * np.exp(
            -m * m * np.pi ** 2 * nu * t / W ** 2)
    return us - s


def powerlaw_shear_rate(sigma, n, xi, nu_lo, nu_hi):
    """Shear rate solving sigma = nu_c(gd) gd with nu_c = clamp(xi gd^(n-1),
    nu_lo, nu_hi) (Eqs. nn1 and nn4 with kappa = 2^(n-1), rho = 1); nu_c gd is
    continuous and increasing, so the three branches are separated by the
    stresses where the clamp switches on."""
    if n == 1.0:
        return sigma / min(max(xi, nu_lo), nu_hi)
    g_hi = (nu_hi / xi) ** (1.0 / (n - 1.0))
    g_lo = (nu_lo / xi) ** (1.0 / (n - 1.0))
    if n < 1.0:
        s1, s2 = nu_hi * g_hi, nu_lo * g_lo
        if sigma <= s1:
            return sigma / nu_hi
        if sigma <= s2:
            return (sigma / xi) ** (1.0 / n)
        return sigma / nu_lo
    s1, s2 = nu_lo * g_lo, nu_hi * g_hi
    if sigma <= s1:
        return sigma / nu_lo
    if sigma <= s2:
        return (sigma / xi) ** (1.0 / n)
    return sigma / nu_hi


def powerlaw_channel(ny, n, xi, g, tau_min, tau_max):
    """Steady power-law channel with the viscosity clamp: u(y) is the integral
    of the shear rate from |y| to the wall, stress g s at distance s from the
    centre line.  Without an active clamp it is Eqs. nn6-nn7."""
    W = ny - 2
    h = W / 2.0
    yc = (ny - 1) / 2.0
    nu_lo, nu_hi = nu_of_tau(tau_min), nu_of_tau(tau_max)
    out = []
    for y in range(1, ny - 1):
        a = abs(y - yc)
        val, _ = quad(lambda s: powerlaw_shear_rate(g * s, n, xi, nu_lo, nu_hi), a, h,
                      limit=400, epsabs=1e-16, epsrel=1e-12)
        out.append(val)
    return np.array(out)


def powerlaw_channel_unclamped(ny, n, xi, g):
    """Eqs. nn6-nn7 with y measured from the centre line."""
    W = ny - 2
    yc = (ny - 1) / 2.0
    y = np.arange(1, ny - 1, dtype=np.float64)
    u0 = (g / xi) ** (1.0 / n) * (W / 2.0) ** (1.0 + 1.0 / n) * n / (n + 1.0)
    return u0 * (1.0 - np.abs(2.0 * (y - yc) / W) ** (1.0 + 1.0 / n))


def couette_torque(nu, omega, r_in, r_out, rho=1.0):
    """Steady torque per unit length on an inner cylinder of radius r_in rotating
    at omega inside a fixed cylinder r_out: -4 pi mu omega r_in^2 r_out^2 /
    (r_out^2 - r_in^2)."""
    mu = rho * nu
    return -4.0 * np.pi * mu * omega * r_in ** 2 * r_out ** 2 / (r_out ** 2 - r_in ** 2)


def square_array_drag(mu, U, phi):
    """Drag per unit length on a cylinder in a square periodic array at solid
    fraction phi and superficial velocity U (Hasimoto 1959; Sangani & Acrivos
    1982 dilute expansion)."""
    return 4.0 * np.pi * mu * U / (-0.5 * np.log(phi) - 0.738 + phi - 0.887 * phi ** 2
                                   + 2.038 * phi ** 3)
